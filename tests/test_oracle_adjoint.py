"""Pins of the oracle's gradient of L = sum_i w_i . a_i.

The tree gradient is the gradient of the discrete forward with the sort
order, cells, groups and lists held fixed.  It is pinned by central finite
differences of the oracle's own fixed-structure forward (h = 1e-6 in box
units for positions, a relative 1e-6 for masses), by translation invariance
(sum_k dL/dx_k = 0), by linearity in w, and at theta = 0 by the brute-force
gradient, which is itself pinned by finite differences of the brute-force
sum."""
import numpy as np
import pytest

import oracle
import synth


def _set(theta=0.5):
    ps = synth.small_clustered(3000, 51, r_cut=0.06, eps=3e-4, theta=theta, per_halo=500)
    w = synth.loss_weights(ps.n, 61)
    return ps, w


def _fd_tree(ot, w, k_sorted, axis, h):
    u = [ot.ux.copy(), ot.uy.copy(), ot.uz.copy()]
    up = [a.copy() for a in u]
    um = [a.copy() for a in u]
    up[axis][k_sorted] += h
    um[axis][k_sorted] -= h
    # difference the forces before the dot product: particles the step does
    # not reach give bit-identical forces and drop out exactly
    da = ot.force_sorted(*up) - ot.force_sorted(*um)
    return float(np.sum(w[ot.perm] * da)) / (2 * h)


def _fd_tree_mass(ot, w, k_sorted, rel):
    h = ot.m[k_sorted] * rel
    mp = ot.m.copy()
    mm = ot.m.copy()
    mp[k_sorted] += h
    mm[k_sorted] -= h
    da = ot.force_sorted(m=mp) - ot.force_sorted(m=mm)
    return float(np.sum(w[ot.perm] * da)) / (2 * h)


def test_tree_adjoint_matches_finite_differences():
    ps, w = _set()
    ot = oracle.OracleTree(ps.x, ps.y, ps.z, ps.m, ps.params)
    assert ot.lists.nidx.size > 0    # node sources are exercised
    gx, gm = ot.adjoint(w)
    inv = np.empty(ps.n, np.int64)
    inv[ot.perm] = np.arange(ps.n)
    rng = np.random.default_rng(7)
    errs_x, errs_m = [], []
    for k in rng.choice(ps.n, 24, replace=False):
        s = inv[k]
        for a in range(3):
            fd = _fd_tree(ot, w, s, a, 1e-6)
            errs_x.append(abs(fd - gx[k, a]) / max(np.abs(gx[k]).max(), 1e-300))
        fdm = _fd_tree_mass(ot, w, s, 1e-6)
        errs_m.append(abs(fdm - gm[k]) / max(abs(gm[k]), 1e-300))
    assert np.median(errs_x) < 1e-6 and max(errs_x) < 1e-4, (np.median(errs_x), max(errs_x))
    assert np.median(errs_m) < 1e-6 and max(errs_m) < 1e-4, (np.median(errs_m), max(errs_m))


def test_tree_adjoint_translation_invariance_and_linearity():
    ps, w = _set()
    ot = oracle.OracleTree(ps.x, ps.y, ps.z, ps.m, ps.params)
    gx, gm = ot.adjoint(w)
    assert np.linalg.norm(gx.sum(0)) < 1e-12 * np.abs(gx).sum()
    w2 = synth.loss_weights(ps.n, 62)
    gx2, gm2 = ot.adjoint(w2)
    gx3, gm3 = ot.adjoint(w + 2.5 * w2)
    assert np.allclose(gx3, gx + 2.5 * gx2, rtol=1e-10, atol=1e-10 * np.abs(gx3).max())
    assert np.allclose(gm3, gm + 2.5 * gm2, rtol=1e-10, atol=1e-10 * np.abs(gm3).max())


def test_theta_zero_tree_adjoint_equals_brute_force():
    ps, w = _set(theta=0.0)
    ot = oracle.OracleTree(ps.x, ps.y, ps.z, ps.m, ps.params)
    gx, gm = ot.adjoint(w)
    bx, bm = oracle.brute_force_adjoint(ps.x, ps.y, ps.z, ps.m, w, 1.0, ps.params.r_cut, ps.params.eps)
    assert np.max(np.abs(gx - bx)) < 1e-10 * np.abs(bx).max()
    assert np.max(np.abs(gm - bm)) < 1e-10 * np.abs(bm).max()


def test_brute_force_adjoint_matches_finite_differences():
    ps = synth.small_clustered(1500, 52, r_cut=0.08, eps=5e-4, theta=0.5, per_halo=300)
    w = synth.loss_weights(ps.n, 63)
    p = ps.params
    bx, bm = oracle.brute_force_adjoint(ps.x, ps.y, ps.z, ps.m, w, 1.0, p.r_cut, p.eps)

    def force(x, y, z, m):
        return oracle.brute_force(x, y, z, m, 1.0, p.r_cut, p.eps)

    rng = np.random.default_rng(8)
    for k in rng.choice(ps.n, 8, replace=False):
        for a, arr in enumerate((ps.x, ps.y, ps.z)):
            h = 1e-6
            cols_p = [ps.x.copy(), ps.y.copy(), ps.z.copy()]
            cols_m = [ps.x.copy(), ps.y.copy(), ps.z.copy()]
            cols_p[a][k] += h
            cols_m[a][k] -= h
            fd = float(np.sum(w * (force(*cols_p, ps.m) - force(*cols_m, ps.m)))) / (2 * h)
            assert abs(fd - bx[k, a]) <= 1e-4 * np.abs(bx[k]).max()
        mp, mm = ps.m.copy(), ps.m.copy()
        hm = 1e-6 * ps.m[k]
        mp[k] += hm
        mm[k] -= hm
        fd = float(np.sum(w * (force(ps.x, ps.y, ps.z, mp) - force(ps.x, ps.y, ps.z, mm)))) / (2 * hm)
        assert abs(fd - bm[k]) <= 1e-6 * abs(bm[k])


def test_two_particle_gradient():
    # L = w0 . a0 + w1 . a1 with a0 = m1 F(d), a1 = -m0 F(d), d = x1 - x0
    rc, eps = 0.1, 1e-3
    x = np.array([0.3, 0.33])
    y = np.array([0.5, 0.52])
    z = np.array([0.7, 0.69])
    m = np.array([2.0, 5.0])
    w = np.array([[1.0, -2.0, 0.5], [0.3, 0.7, -1.1]])
    gx, gm = oracle.brute_force_adjoint(x, y, z, m, w, 1.0, rc, eps)
    d = np.array([x[1] - x[0], y[1] - y[0], z[1] - z[0]])
    F = oracle.pair_force(d, rc, eps)
    assert np.isclose(gm[0], -w[1] @ F, rtol=1e-13)
    assert np.isclose(gm[1], w[0] @ F, rtol=1e-13)
    # dL/dx1 = m1 J w0 - m0 J w1 = -dL/dx0
    v = m[1] * w[0] - m[0] * w[1]
    jv = oracle.pair_jac(d, v, rc, eps)
    assert np.allclose(gx[1], jv, rtol=1e-13) and np.allclose(gx[0], -jv, rtol=1e-13)
