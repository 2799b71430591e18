"""Element-wise parity bounds shared by the GPU tests.

A kernel result x_i is compared with the FP64 oracle's x_i^ref particle by
particle:

    |x_i - x_i^ref| <= C * E_i        for every i,

where E_i is the oracle's first-order error magnitude of that particle
(``OracleTree.force_bound`` / ``adjoint_bound``: per pair, the pair's
sensitivity times the uncertainty of its offset when group-relative offsets
are rounded with the kernel's unit roundoff u, summed over the list) and C
counts how many times that magnitude can be spent:

    C = K + P + L_ref * u64 / u

  K     the longest sum the kernel forms in working precision before it is
        added in FP64 (force: one lane's partial over a 32-entry chunk of a tile;
        adjoint: one lane's i-side partial over the 64 entries of its row in
        a tile, longer than the j-side's 4-term register sum and 16-lane
        row sum),
  P     the roundings in evaluating one pair, counted to first order
        (offsets and their difference, r^2, s^2, rsq, r, the degree-8
        polynomial of eq. (cutoff) in Horner form, products): 64,
  L_ref the longest list the oracle sums in FP64 (its own error).

E_i = 0 (nothing within r_cut) demands exact equality.
"""
import sys

import numpy as np

U32 = 2.0 ** -24
U64 = 2.0 ** -53
P_PAIR = 64
K_FORCE = 32
K_ADJOINT = 64


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def unit(precision_fp64: bool) -> float:
    return U64 if precision_fp64 else U32


def constant(kind: str, fp64: bool, max_list: int) -> float:
    k = K_FORCE if kind == "force" else K_ADJOINT
    return k + P_PAIR + max_list * U64 / unit(fp64)


def max_list(ot) -> int:
    nj = np.diff(ot.lists.poff) + np.diff(ot.lists.noff)
    return int(nj.max()) if nj.size else 0


def check(got, ref, E, C, what):
    """Assert |got_i - ref_i| <= C E_i for every row i (vector rows use the
    Euclidean norm).  Returns the largest |got_i - ref_i| / E_i, the
    constant actually needed."""
    got = np.asarray(got, dtype=np.float64).reshape(len(E), -1)
    ref = np.asarray(ref, dtype=np.float64).reshape(len(E), -1)
    d = np.linalg.norm(got - ref, axis=1)
    pos = E > 0
    need = float(np.max(d[pos] / E[pos])) if pos.any() else 0.0
    zero_ok = bool(np.all(d[~pos] == 0.0))
    bad = np.flatnonzero(d > C * E)
    say(f"    {what}: max |diff| / E = {need:.3g} (bound C = {C:.4g}); {int((~pos).sum())} exact zeros "
        f"{'equal' if zero_ok else 'DIFFER'}")
    assert zero_ok, f"{what}: a particle with nothing within r_cut differs from zero"
    assert bad.size == 0, (f"{what}: {bad.size} particles beyond C E, first {bad[:5]}: "
                           f"{d[bad[:5]]} > {C * E[bad[:5]]}")
    return need
