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


def _same_structure(a, b):
    if not np.array_equal(a.perm, b.perm):
        return False
    for k in ("level", "prefix", "first", "count"):
        if not np.array_equal(getattr(a.tree, k), getattr(b.tree, k)):
            return False
    if not (np.array_equal(a.gfirst, b.gfirst) and np.array_equal(a.gcount, b.gcount)):
        return False
    return all(np.array_equal(getattr(a.lists, k), getattr(b.lists, k)) for k in ("poff", "pidx", "noff", "nidx"))


def test_finite_differences_with_structure_rebuilt():
    """Central differences with the whole structure rebuilt from the moved
    positions (sort, cells, groups, lists): where the structure of both moved
    sets equals the original one the result is the fixed-structure gradient;
    the steps that change it (list flips) are counted and must be rare.  The
    forces are differenced before the dot product with w, and the error is
    taken relative to max(|dL/dx_k|, rms of dL/dx) (the rebuilt group boxes
    move the group-relative coordinates at the rounding level)."""
    ps, w = _set()
    ot = oracle.OracleTree(ps.x, ps.y, ps.z, ps.m, ps.params)
    gx, _ = ot.adjoint(w)
    rms = float(np.sqrt(np.mean(gx ** 2)))
    X = np.stack([ps.x, ps.y, ps.z], axis=1)
    rng = np.random.default_rng(11)
    h = 1e-6
    errs, flips, total = [], 0, 0
    for k in rng.choice(ps.n, 24, replace=False):
        for a in range(3):
            forces, same = [], True
            for sgn in (1.0, -1.0):
                Y = X.copy()
                Y[k, a] += sgn * h
                o2 = oracle.OracleTree(Y[:, 0], Y[:, 1], Y[:, 2], ps.m, ps.params)
                same = same and _same_structure(ot, o2)
                forces.append(o2.force())
            total += 1
            if not same:
                flips += 1
                continue
            fd = float(np.sum(w * (forces[0] - forces[1]))) / (2 * h)
            errs.append(abs(fd - gx[k, a]) / max(np.abs(gx[k]).max(), rms))
    print(f"structure changed in {flips} of {total} steps; agreement elsewhere: median {np.median(errs):.2e}, "
          f"max {max(errs):.2e}")
    assert flips <= total // 4
    assert np.median(errs) < 1e-6 and max(errs) < 1e-4
