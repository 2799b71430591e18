"""Pins of the quadrupole accuracy variant of the oracle (CPU).

The quadrupole term of a cell is the second-order term of the Taylor
expansion of sum_k m_k F(D + delta_k) about the centre of mass (Sec. 1
multipole expansion taken one order past the monopole), with F the cutoff
pair force of Sec. 2.  Pinned by: g'' against differences of g'; the term
against a finite-difference Hessian of the oracle's pair force; the error
of monopole + quadrupole against the exact cluster sum falling as h^3 (the
monopole's as h^2); the second moments against the parallel-axis theorem
over each cell's children; and the tree force with quadrupoles closer to
the direct sum than the monopole tree at the same theta.
"""
import numpy as np
import pytest

import oracle
import synth


def test_gcut_second_derivative():
    xi = np.linspace(0.01, 1.99, 397)
    h = 1e-6
    fd = (oracle.gcut(xi + h)[1] - oracle.gcut(xi - h)[1]) / (2 * h)
    assert np.max(np.abs(oracle.gcut_deriv2(xi) - fd)) < 1e-8
    # continuous at 1, zero from 2 on
    lo, hi = oracle.gcut_deriv2(np.array([1.0 - 1e-12, 1.0 + 1e-12]))
    assert abs(lo - hi) < 1e-9 and abs(lo - 1.4) < 1e-9
    assert np.all(oracle.gcut_deriv2(np.array([2.0, 2.3])) == 0.0)


def random_sym(rng):
    A = rng.normal(size=(3, 3))
    S = A @ A.T
    return np.array([S[0, 0], S[1, 1], S[2, 2], S[0, 1], S[0, 2], S[1, 2]]), S


@pytest.mark.parametrize("xi", [0.3, 0.8, 1.2, 1.7])
@pytest.mark.parametrize("eps", [1e-6, 2e-3])
def test_quad_term_is_half_the_hessian_contraction(xi, eps):
    rng = np.random.default_rng(int(xi * 10) + int(eps * 1e6))
    rc = 0.1
    u = rng.normal(size=3)
    D = u / np.linalg.norm(u) * xi * rc / 2
    S6, S = random_sym(rng)
    h = 1e-4 * np.linalg.norm(D)
    H = np.zeros((3, 3, 3))   # H[a, b] = d_a d_b F
    E = np.eye(3) * h
    for a in range(3):
        for b in range(3):
            f = lambda sa, sb: oracle.pair_force(D + sa * E[a] + sb * E[b], rc, eps)
            H[a, b] = (f(1, 1) - f(1, -1) - f(-1, 1) + f(-1, -1)) / (4 * h * h)
    ref = 0.5 * np.einsum("ab,abc->c", S, H)
    got = oracle.quad_term(D, S6, rc, eps)
    assert np.linalg.norm(got - ref) <= 2e-6 * np.linalg.norm(ref)


@pytest.mark.parametrize("xi", [0.4, 1.3])
def test_quadrupole_error_is_third_order(xi):
    """A cluster of 6 masses scaled by h about its centre of mass at offset D:
    the monopole error falls as h^2, the monopole + quadrupole error as h^3."""
    rng = np.random.default_rng(5)
    rc, eps = 0.1, 1e-5
    m = rng.uniform(0.5, 1.5, 6)
    dl = rng.normal(size=(6, 3))
    dl -= (m[:, None] * dl).sum(0) / m.sum()      # centre of mass at 0
    u = rng.normal(size=3)
    D = u / np.linalg.norm(u) * xi * rc / 2
    S1 = np.einsum("k,ka,kb->ab", m, dl, dl)
    S6 = np.array([S1[0, 0], S1[1, 1], S1[2, 2], S1[0, 1], S1[0, 2], S1[1, 2]])
    mono, quad = [], []
    for h in (2e-3, 1e-3, 5e-4):
        exact = sum(mk * oracle.pair_force(D + h * d, rc, eps) for mk, d in zip(m, dl))
        F0 = m.sum() * oracle.pair_force(D, rc, eps)
        mono.append(np.linalg.norm(exact - F0))
        quad.append(np.linalg.norm(exact - F0 - oracle.quad_term(D, h * h * S6, rc, eps)))
    for k in range(2):
        assert 3.5 < mono[k] / mono[k + 1] < 4.5
        assert 7.0 < quad[k] / quad[k + 1] < 9.0
    assert quad[-1] < 0.25 * mono[-1]


def test_second_moments_parallel_axis():
    ps = synth.small_clustered(3000, 61, r_cut=0.1, eps=1e-3, theta=0.5, per_halo=500)
    ot = oracle.OracleTree(ps.x, ps.y, ps.z, ps.m, ps.params)
    S = ot.second_moments()
    t = ot.tree
    checked = 0
    for c in np.flatnonzero(t.leaf == 0)[:400]:
        kids = t.child[c][t.child[c] >= 0]
        acc = np.zeros(6)
        for q in kids:
            d = ot.X[q] - ot.X[c]
            acc += S[q] + ot.M[q] * np.array([d[0] * d[0], d[1] * d[1], d[2] * d[2],
                                              d[0] * d[1], d[0] * d[2], d[1] * d[2]])
        # rounding of each offset x_k - X (about 2.2e-16 absolute for
        # coordinates in [0, 1)) changes S by up to 2 * 2.2e-16 * M * max|delta|
        # with max|delta| <= sqrt(3) * side, on both sides of the identity
        side = 2.0 ** -float(t.level[c])
        tol = 4e-15 * ot.M[c] * side + 1e-13 * np.max(np.abs(S[c, :3]))
        assert np.max(np.abs(acc - S[c])) <= tol
        checked += 1
    assert checked > 50
    # a cell with a single particle has no second moment (up to the rounding
    # of X = m x / m, below one ulp of x)
    single = np.flatnonzero(t.count == 1)
    assert single.size > 0
    assert np.all(np.abs(S[single]) <= (ot.M[single] * 1.3e-32)[:, None])


def test_quadrupole_tree_closer_to_direct_sum():
    ps = synth.small_clustered(6000, 62, r_cut=0.1, eps=2e-4, theta=0.7, per_halo=1000)
    ref = oracle.brute_force(ps.x, ps.y, ps.z, ps.m, 1.0, ps.params.r_cut, ps.params.eps)
    for theta in (0.5, 0.8):
        p = synth.Params(1.0, ps.params.r_cut, ps.params.eps, theta, 64, 16)
        ot = oracle.OracleTree(ps.x, ps.y, ps.z, ps.m, p)
        e1 = oracle.relative_errors(ot.force(), ref)[1]
        e2 = oracle.relative_errors(ot.force_quadrupole(), ref)[1]
        # most particles of this set see no cell at theta = 0.5 (median ~1e-16),
        # so the comparison is on the global figures
        assert e2["l2"] < 0.5 * e1["l2"] and e2["rms"] < 0.5 * e1["rms"], (theta, e1, e2)
    # theta = 0: no cells, so no quadrupole terms
    p0 = synth.Params(1.0, ps.params.r_cut, ps.params.eps, 0.0, 64, 16)
    ot0 = oracle.OracleTree(ps.x, ps.y, ps.z, ps.m, p0)
    assert np.array_equal(ot0.force_quadrupole(), ot0.force())
