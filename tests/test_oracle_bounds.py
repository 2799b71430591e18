"""Pins of the oracle's per-particle error magnitudes (force_bound,
adjoint_bound), which scale the element-wise parity bounds of the GPU tests.

They are pinned against things other than themselves:
  - the pair coefficients: nJ against the spectral norm of the oracle's
    Jacobian J = dF/dd (nJ >= ||J|| >= nJ / 3) and nH against finite
    differences of J w along random directions, for two bodies at separations
    from below eps up to the cutoff;
  - coverage of every list entry: the magnitude with unit rounding bounds the
    sum over the list of |m_j F(d_ij)|, computed pair by pair through the
    oracle's pair force;
  - the perturbation they describe: moving every particle by up to eta (with
    the structure held fixed) changes the oracle's own force and gradient by
    no more than the magnitude with e_abs = 2 eta, and by a fair fraction of
    it (the bound is not vacuous).
"""
import numpy as np

import oracle
import synth

U64 = 2.0 ** -53


def _two_body(r, rc=0.1, eps=1e-3, direction=(0.6, 0.0, 0.8)):
    d = np.array(direction) / np.linalg.norm(direction)
    x = np.array([[0.497, 0.501, 0.503], [0.497, 0.501, 0.503] + r * d])
    m = np.array([0.3, 0.7])
    p = synth.Params(1.0, rc, eps, 0.0, 64, 16)
    return oracle.OracleTree(x[:, 0], x[:, 1], x[:, 2], m, p), x, m


def test_pair_coefficients_bound_jacobian_and_its_derivative():
    rng = np.random.default_rng(5)
    rc, eps = 0.1, 1e-3
    ratios = []
    for r in (2e-4, 1e-3, 4e-3, 0.02, 0.049, 0.05, 0.051, 0.08, 0.0995):
        ot, x, m = _two_body(r, rc, eps)
        d = x[1] - x[0]
        # nJ from the force magnitude with a unit position uncertainty
        E = ot.force_bound(u_k=0.0, u_c=0.0, e_abs=1.0)
        nJ = E[0] / m[1]
        assert np.isclose(E[1] / m[0], nJ, rtol=1e-12)
        J = np.stack([oracle.pair_jac(d, e, rc, eps) for e in np.eye(3)], axis=1)
        sv = np.linalg.norm(J, 2)
        assert sv <= nJ * (1 + 1e-12) and nJ <= 3.0 * sv * (1 + 1e-12), (r, sv, nJ)
        # nH from the gradient magnitude: unit weight on particle 0 only
        w = np.zeros((2, 3))
        w[0] = rng.standard_normal(3)
        w[0] /= np.linalg.norm(w[0])
        Ex, _ = ot.adjoint_bound(w, u_k=0.0, u_c=0.0, e_abs=1.0)
        nH = Ex[0] / m[1]
        # ||d(J v)/dd u|| over unit u, v: the radial pair (u = v = d/r) and
        # random directions (the oracle's J, differenced)
        h = 1e-7 * r
        dh = d / np.linalg.norm(d)
        worst = 0.0
        dirs = [(dh, dh)] + [(rng.standard_normal(3), rng.standard_normal(3)) for _ in range(60)]
        for u, v in dirs:
            u, v = u / np.linalg.norm(u), v / np.linalg.norm(v)
            dj = (oracle.pair_jac(d + h * u, v, rc, eps) - oracle.pair_jac(d - h * u, v, rc, eps)) / (2 * h)
            worst = max(worst, float(np.linalg.norm(dj)))
        assert worst <= nH * (1 + 1e-5), (r, worst, nH)
        ratios.append(nH / worst)
    # 3 |psi| r + |chi| r^3 is the triangle inequality on the radial and
    # transverse parts: attained where they do not cancel
    assert min(ratios) <= 1.5, ratios


def test_force_bound_covers_every_list_entry():
    ps = synth.small_clustered(1500, 71, r_cut=0.08, eps=3e-4, theta=0.5, per_halo=300)
    ot = oracle.OracleTree(ps.x, ps.y, ps.z, ps.m, ps.params)
    L = ot.lists
    assert L.nidx.size > 0
    rc, eps = ps.params.r_cut, ps.params.eps
    S = np.zeros(ot.n)
    for g in range(ot.n_groups):
        for i in range(ot.gfirst[g], ot.gfirst[g] + ot.gcount[g]):
            xi = np.array([ot.ux[i], ot.uy[i], ot.uz[i]])
            for j in L.pidx[L.poff[g]:L.poff[g + 1]]:
                d = np.array([ot.ux[j], ot.uy[j], ot.uz[j]]) - xi
                d -= np.rint(d)
                S[i] += ot.m[j] * np.linalg.norm(oracle.pair_force(d, rc, eps))
            for c in L.nidx[L.noff[g]:L.noff[g + 1]]:
                d = ot.X[c] - xi
                d -= np.rint(d)
                S[i] += ot.M[c] * np.linalg.norm(oracle.pair_force(d, rc, eps))
    E1 = ot.force_bound_sorted(u_k=1.0, u_c=0.0)
    assert np.all(E1 >= S * (1 - 1e-12))
    assert np.all((S > 0) == (E1 > 0))


def _perturbed(ot, eta, seed):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((ot.n, 3))
    v *= (eta * rng.random(ot.n) / np.linalg.norm(v, axis=1))[:, None]
    return ot.ux + v[:, 0], ot.uy + v[:, 1], ot.uz + v[:, 2]


def test_force_bound_covers_a_position_perturbation():
    ps = synth.small_clustered(3000, 72, r_cut=0.06, eps=3e-4, theta=0.5, per_halo=500)
    ot = oracle.OracleTree(ps.x, ps.y, ps.z, ps.m, ps.params)
    eta = 1e-9
    a0 = ot.force_sorted()
    a1 = ot.force_sorted(*_perturbed(ot, eta, 3))
    delta = np.linalg.norm(a1 - a0, axis=1)
    E = ot.force_bound_sorted(u_k=0.0, u_c=0.0, e_abs=2 * eta)
    noise = 64 * U64 * ot.force_bound_sorted(u_k=1.0, u_c=0.0)
    assert np.all(delta <= E * (1 + 1e-3) + noise)
    ratio = delta[E > 0] / E[E > 0]
    print(f"force: max |delta| / E = {ratio.max():.3f}, median {np.median(ratio):.3f}")
    assert ratio.max() > 0.05


def test_adjoint_bound_covers_a_position_perturbation():
    ps = synth.small_clustered(3000, 73, r_cut=0.06, eps=3e-4, theta=0.5, per_halo=500)
    w = synth.loss_weights(ps.n, 74)
    ot = oracle.OracleTree(ps.x, ps.y, ps.z, ps.m, ps.params)
    assert ot.lists.nidx.size > 0
    eta = 1e-9
    gx0, gm0 = ot.adjoint(w)
    gx1, gm1 = ot.adjoint(w, *_perturbed(ot, eta, 4))
    dx = np.linalg.norm(gx1 - gx0, axis=1)
    dm = np.abs(gm1 - gm0)
    Ex, Em = ot.adjoint_bound(w, u_k=0.0, u_c=0.0, e_abs=2 * eta)
    nx, nm = ot.adjoint_bound(w, u_k=1.0, u_c=0.0)
    assert np.all(dx <= Ex * (1 + 1e-3) + 64 * U64 * nx)
    assert np.all(dm <= Em * (1 + 1e-3) + 64 * U64 * nm)
    rx, rm = dx[Ex > 0] / Ex[Ex > 0], dm[Em > 0] / Em[Em > 0]
    print(f"adjoint: max ratio dL/dx {rx.max():.3f}, dL/dm {rm.max():.3f}")
    assert rx.max() > 0.05 and rm.max() > 0.05


def test_bounds_are_zero_only_without_interactions():
    # a particle with nothing within r_cut has a zero force, a zero gradient
    # and a zero bound: the element-wise test then demands exact zeros
    x = np.array([[0.1, 0.1, 0.1], [0.6, 0.6, 0.6], [0.62, 0.6, 0.6]])
    p = synth.Params(1.0, 0.05, 1e-3, 0.5, 64, 16)
    ot = oracle.OracleTree(x[:, 0], x[:, 1], x[:, 2], np.full(3, 1 / 3), p)
    E = ot.force_bound(2.0 ** -24)
    Ex, Em = ot.adjoint_bound(np.ones((3, 3)), 2.0 ** -24)
    a = ot.force()
    assert E[0] == 0.0 and Ex[0] == 0.0 and Em[0] == 0.0 and np.all(a[0] == 0.0)
    assert np.all(E[1:] > 0) and np.all(Ex[1:] > 0) and np.all(Em[1:] > 0)
