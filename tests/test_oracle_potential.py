"""Pins of the short-range potential (accuracy variant of the split): q
against the force factor g (g = q - xi q'), its values at 0, 1, 2 and its
continuity; minus the gradient of the brute-force potential against the
brute-force force; the tree potential at theta = 0 against brute force and
its error falling with theta."""
import numpy as np

import oracle
import synth


def test_q_values_and_relation_to_g():
    q = oracle.qcut(np.array([0.0, 1.0 - 1e-15, 1.0, 2.0, 2.5]))
    assert q[0] == 1.0 and abs(q[1] - 0.05) < 1e-13 and abs(q[2] - 0.05) < 1e-15 and q[3] == 0.0 and q[4] == 0.0
    xi = np.linspace(0.01, 1.99, 397)
    h = 1e-6
    dq = (oracle.qcut(xi + h) - oracle.qcut(xi - h)) / (2 * h)
    assert np.max(np.abs(oracle.qcut(xi) - xi * dq - oracle.gcut(xi)[0])) < 1e-9


def test_potential_gradient_is_the_force():
    rng = np.random.default_rng(21)
    n = 200
    P = rng.random((n, 3))
    m = rng.uniform(0.5, 1.5, n) / n
    rc, eps = 0.2, 1e-9
    a = oracle.brute_force(P[:, 0], P[:, 1], P[:, 2], m, 1.0, rc, eps, method="n2")
    h = 1e-6
    for i in rng.choice(n, 10, replace=False):
        g = np.empty(3)
        for ax in range(3):
            Pp, Pm = P.copy(), P.copy()
            Pp[i, ax] += h
            Pm[i, ax] -= h
            fp = oracle.brute_force_potential(Pp[:, 0], Pp[:, 1], Pp[:, 2], m, 1.0, rc, eps)[i]
            fm = oracle.brute_force_potential(Pm[:, 0], Pm[:, 1], Pm[:, 2], m, 1.0, rc, eps)[i]
            g[ax] = (fp - fm) / (2 * h)
        assert np.max(np.abs(-g - a[i])) < 1e-6 * np.max(np.abs(a[i])) + 1e-9


def test_tree_potential_at_theta_zero_is_brute_force():
    ps = synth.small_clustered(3000, 52, r_cut=0.08, eps=3e-4, theta=0.0, per_halo=500)
    ot = oracle.OracleTree(ps.x, ps.y, ps.z, ps.m, ps.params)
    bf = oracle.brute_force_potential(ps.x, ps.y, ps.z, ps.m, 1.0, ps.params.r_cut, ps.params.eps)
    assert np.max(np.abs(ot.potential() - bf)) < 1e-12 * np.max(np.abs(bf))
    nz = bf != 0.0
    errs = []
    for th in (0.3, 0.5, 0.7):
        ot5 = oracle.OracleTree(ps.x, ps.y, ps.z, ps.m, synth.Params(1.0, 0.08, 3e-4, th, 64, 16))
        errs.append(np.median(np.abs(ot5.potential()[nz] - bf[nz]) / np.abs(bf[nz])))
    assert errs[0] < errs[1] < errs[2] < 1e-2

