"""GPU parity of the short-range potential of the split against the FP64
oracle, through the C ABI.

The potential is a sum of terms of one sign (q >= 0 on [0, 2]), so its
relative error is that of the terms: FP32 group-relative offsets give
about 1e-7 per pair (more where q is a small difference, at xi -> 1 of the
inner polynomial or xi -> 2, where (2 - xi)^6 amplifies the rounding of r
by 6 / (2 - xi)).  Tolerances: rms relative error <= 1e-5 (FP32) and
<= 1e-12 (FP64) against the same-list oracle.
"""
import ctypes as C
import dataclasses
import sys

import numpy as np
import pytest
import torch

import oracle
import paper_1211_4406_amd as srf
import synth

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5
FP64_TOL = 1e-12


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_potential(ps, params=None, precision=srf.FP32_REL):
    p = srf.Params.of(params or ps.params, precision)
    x = torch.tensor(ps.positions(), dtype=torch.float64, device="cuda")
    m = torch.tensor(ps.m, dtype=torch.float64, device="cuda")
    tree = srf.tree_build(x, m, p)
    lists = srf.make_lists(tree, p)
    phi = srf.short_range_potential(tree, lists, p)
    torch.cuda.synchronize()
    return tree, lists, phi.cpu().numpy()


def rel(phi, ref):
    """rms and max of |phi - ref| / |ref| over the particles with ref != 0;
    where ref == 0 (nothing within r_cut) phi must be exactly 0."""
    nz = ref != 0.0
    assert np.all(phi[~nz] == 0.0)
    e = np.abs(phi[nz] - ref[nz]) / np.abs(ref[nz])
    return {"rms": float(np.sqrt(np.mean(e * e))), "max": float(e.max()), "n": int(nz.sum())}


CASES = {
    "cfg1-uniform-4096": lambda: synth.make_config(1),
    "clustered-20000": lambda: synth.small_clustered(20000, 101, r_cut=0.1, eps=2e-4, theta=0.5, per_halo=1000),
    "clustered-tight-12000": lambda: synth.small_clustered(12000, 102, r_cut=0.1, eps=5e-5, theta=0.7,
                                                           per_halo=3000, a_range=(2e-4, 2e-3)),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("theta", [0.0, 0.5, 1.0])
def test_potential_matches_oracle(name, theta):
    ps = CASES[name]()
    params = synth.Params(1.0, ps.params.r_cut, ps.params.eps, theta, 64, 16)
    say(f"[gpu] potential {name} theta={theta} n={ps.n}")
    ot = oracle.OracleTree(ps.x, ps.y, ps.z, ps.m, params)
    ref = ot.potential()
    _, _, p32 = gpu_potential(ps, params, srf.FP32_REL)
    s32 = rel(p32, ref)
    say(f"    fp32 vs oracle: {s32}")
    assert s32["rms"] <= FP32_TOL
    _, _, p64 = gpu_potential(ps, params, srf.FP64)
    s64 = rel(p64, ref)
    say(f"    fp64 vs oracle: {s64}")
    assert s64["rms"] <= FP64_TOL


def test_potential_theta0_is_direct_sum():
    """At theta = 0 every partner within r_cut is a particle entry: the tree
    potential is the O(N^2) minimum-image sum."""
    ps = synth.small_clustered(6000, 141, r_cut=0.1, eps=1e-3, theta=0.0, per_halo=600)
    say(f"[gpu] potential theta=0 vs direct sum n={ps.n}")
    ref = oracle.brute_force_potential(ps.x, ps.y, ps.z, ps.m, 1.0, 0.1, 1e-3)
    _, _, p64 = gpu_potential(ps, precision=srf.FP64)
    _, _, p32 = gpu_potential(ps)
    s64, s32 = rel(p64, ref), rel(p32, ref)
    say(f"    fp64 {s64}\n    fp32 {s32}")
    assert s64["rms"] <= FP64_TOL and s32["rms"] <= FP32_TOL


def test_potential_two_bodies_and_isolated():
    """Two particles across the periodic face: phi_0 = -G m_1 q(2r/r_cut) / s,
    phi_1 = -G m_0 q / s, 0 from r_cut on; a lone particle's potential is 0
    (its own entry is left out)."""
    rc, eps, G = 0.1, 1e-3, 2.0
    m = np.array([0.25, 0.75])
    for r in (0.0004, 0.003, 0.02, 0.049, 0.05, 0.07, 0.09, 0.0999, 0.1 * (1 + 1e-6), 0.12):
        x = np.array([[0.995, 0.5, 0.5], [0.995 + r, 0.5, 0.5]])
        ps = synth.ParticleSet(x[:, 0].copy(), x[:, 1].copy(), x[:, 2].copy(), m.copy(),
                               synth.Params(G, rc, eps, 0.5, 64, 16))
        _, _, p32 = gpu_potential(ps)
        _, _, p64 = gpu_potential(ps, precision=srf.FP64)
        d = np.mod(x[1, 0], 1.0) - x[0, 0]
        d -= np.rint(d)
        q = oracle.qcut(np.array([2.0 * abs(d) / rc]))[0] if abs(d) < rc else 0.0
        ref = -G * np.array([m[1], m[0]]) * q / np.sqrt(d * d + eps * eps)
        if r >= rc:
            assert np.all(p32 == 0.0) and np.all(p64 == 0.0)
            continue
        # rounding of r (relative 6e-8 in FP32) is amplified by 6 xi / (2 - xi)
        xi = 2 * r / rc
        assert np.allclose(p64, ref, rtol=1e-14 * (1 + xi / (2 - xi)), atol=0)
        assert np.allclose(p32, ref, rtol=2e-6 + 1e-6 * xi / (2 - xi), atol=0)
    lone = synth.ParticleSet(np.array([0.3]), np.array([0.4]), np.array([0.5]), np.array([1.0]),
                             synth.Params(1.0, rc, eps, 0.5, 64, 16))
    _, _, p = gpu_potential(lone)
    assert p[0] == 0.0


def test_potential_coincident_particles():
    """Coincident particles see each other at the softened distance eps:
    m q(0) / eps each; only a particle's own entry is left out."""
    rng = np.random.default_rng(5)
    pos = np.concatenate([np.full((150, 3), 0.123456789), rng.random((500, 3))])
    n = len(pos)
    p = synth.Params(1.0, 0.1, 1e-3, 0.5, 64, 16)
    ps = synth.ParticleSet(pos[:, 0].copy(), pos[:, 1].copy(), pos[:, 2].copy(), np.full(n, 1.0 / n), p)
    ref = oracle.OracleTree(ps.x, ps.y, ps.z, ps.m, p).potential()
    _, _, p64 = gpu_potential(ps, p, srf.FP64)
    _, _, p32 = gpu_potential(ps, p)
    assert rel(p64, ref)["rms"] <= FP64_TOL and rel(p32, ref)["rms"] <= FP32_TOL
    # the coincident block alone contributes 149 / n / eps to each member
    assert np.all(-p64[:150] >= 149.0 / n / 1e-3)


def test_potential_strided_output_and_errors():
    ps = synth.make_config(1)
    p = srf.Params.of(ps.params)
    x = torch.tensor(ps.positions(), dtype=torch.float64, device="cuda")
    m = torch.tensor(ps.m, dtype=torch.float64, device="cuda")
    tree = srf.tree_build(x, m, p)
    lists = srf.make_lists(tree, p)
    dense = srf.short_range_potential(tree, lists, p)
    buf = torch.full((ps.n, 3), 7.0, dtype=torch.float64, device="cuda")
    srf.short_range_potential(tree, lists, p, out=buf[:, 1])
    torch.cuda.synchronize()
    assert torch.equal(buf[:, 1], dense)
    assert torch.all(buf[:, 0] == 7.0) and torch.all(buf[:, 2] == 7.0)
    L = srf.lib()
    cp = p.c()
    assert L.srf_short_range_potential(tree.handle, lists.handle, C.byref(cp), None, 1, None) == -1
    assert L.srf_short_range_potential(tree.handle, lists.handle, C.byref(cp), C.c_void_p(dense.data_ptr()),
                                       0, None) == -1
    cb = dataclasses.replace(p, r_cut=0.11).c()
    assert L.srf_short_range_potential(tree.handle, lists.handle, C.byref(cb), C.c_void_p(dense.data_ptr()),
                                       1, None) == -5   # SRF_EMISMATCH
    with pytest.raises(ValueError):
        srf.short_range_potential(tree, lists, p, out=torch.empty(ps.n, dtype=torch.float32, device="cuda"))
