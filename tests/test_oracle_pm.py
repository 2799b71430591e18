"""Pins of the long-range (PM) oracle and of the Ewald sum that checks it.

Ewald: independent of the splitting parameter, zero force on a simple cubic
lattice, pairwise antisymmetry, and the Newtonian limit for a close pair.
PM: TSC weights and mass conservation, the S2 shape's transform against a
direct quadrature of the S2 density of the force split (Sec. 2), the
Newtonian limit of the Green's function, momentum conservation, and the
total (brute-force PP + PM) against Ewald, with an error that falls as the
split radius grows in mesh cells."""
import numpy as np
from scipy.integrate import quad

import oracle
from oracle import pm


def test_ewald_independent_of_splitting_parameter():
    rng = np.random.default_rng(1)
    P = rng.random((40, 3))
    m = rng.uniform(0.5, 1.5, 40)
    a5 = pm.ewald_force(P[:, 0], P[:, 1], P[:, 2], m, 1.0, alpha=5.0, n_real=2, k_max=12)
    a7 = pm.ewald_force(P[:, 0], P[:, 1], P[:, 2], m, 1.0, alpha=7.0, n_real=2, k_max=14)
    assert np.max(np.abs(a5 - a7)) < 1e-9 * np.max(np.abs(a5))


def test_ewald_lattice_and_antisymmetry():
    g = (np.arange(4) + 0.5) / 4
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    a = pm.ewald_force(X.ravel(), Y.ravel(), Z.ravel(), np.ones(64), 1.0)
    assert np.max(np.abs(a)) < 1e-10
    P = np.array([[0.1, 0.2, 0.3], [0.45, 0.25, 0.9]])
    m = np.array([1.0, 3.0])
    a = pm.ewald_force(P[:, 0], P[:, 1], P[:, 2], m, 1.0)
    assert np.allclose(m[0] * a[0], -m[1] * a[1], rtol=0, atol=1e-12)


def test_ewald_newtonian_limit():
    d = 1e-3
    P = np.array([[0.3, 0.3, 0.3], [0.3 + d, 0.3, 0.3]])
    a = pm.ewald_force(P[:, 0], P[:, 1], P[:, 2], np.array([1.0, 1.0]), 1.0)
    # images and the neutralising background correct 1/d^2 at relative O(d^3)
    assert abs(a[0, 0] - 1.0 / d ** 2) < 1e-6 / d ** 2
    assert abs(a[0, 1]) < 1e-6 and abs(a[0, 2]) < 1e-6


def test_tsc_weights_and_mass_conservation():
    idx, w = pm.tsc_stencil(np.array([3.0, 3.5 - 1e-12, 7.9]), 8)
    assert np.allclose(w[0], [0.125, 0.75, 0.125]) and list(idx[0]) == [2, 3, 4]
    # half-way between mesh points: split evenly between points 3 and 4
    assert np.allclose(w[1], [0.0, 0.5, 0.5], atol=1e-11) and list(idx[1]) == [2, 3, 4]
    # periodic wrap: nearest point 8 = 0
    assert list(idx[2]) == [7, 0, 1] and np.isclose(w[2].sum(), 1.0)
    rng = np.random.default_rng(2)
    P = rng.random((500, 3))
    m = rng.uniform(0.1, 2.0, 500)
    rho = pm.tsc_assign(P[:, 0], P[:, 1], P[:, 2], m, 16)
    assert abs(rho.sum() / 16 ** 3 - m.sum()) < 1e-12 * m.sum()


def test_s2_shape_against_quadrature_of_the_split_density():
    # the S2 density of the split with radius R = r_cut/2: rho(r) = 3/(pi R^3) (1 - r/R)
    R = 0.05
    for k in (0.5, 10.0, 40.0, 90.0):
        val = quad(lambda r: 3.0 / (np.pi * R ** 3) * (1 - r / R) * 4 * np.pi * r * np.sin(k * r) / k, 0, R,
                   epsabs=1e-14, epsrel=1e-12)[0]
        assert abs(pm.s2_shape(np.array([k * R]))[0] - val) < 1e-10


def test_green_function_newtonian_limit():
    n, r_cut = 32, 3.0 / 32
    g = pm.green(n, r_cut, 1.0)
    k = 2 * np.pi
    # smallest wave vector: S ~ 1, W ~ 1, so g ~ -4 pi / k^2
    assert abs(g[1, 0, 0] / (-4 * np.pi / k ** 2) - 1) < 5e-3
    assert g[0, 0, 0] == 0.0


def test_pm_momentum_conservation():
    rng = np.random.default_rng(3)
    P = rng.random((300, 3))
    m = rng.uniform(0.5, 1.5, 300)
    a = pm.pm_force(P[:, 0], P[:, 1], P[:, 2], m, 1.0, 3.0 / 16, 16)
    assert np.linalg.norm((m[:, None] * a).sum(0)) < 1e-12 * np.sum(m * np.linalg.norm(a, axis=1))


def _total_vs_ewald(n_mesh, cells, n=256, seed=4):
    rng = np.random.default_rng(seed)
    P = rng.random((n, 3))
    m = np.full(n, 1.0 / n)
    r_cut = cells / n_mesh
    eps = 1e-6
    a_pp = oracle.brute_force(P[:, 0], P[:, 1], P[:, 2], m, 1.0, r_cut, eps, method="n2")
    a_pm = pm.pm_force(P[:, 0], P[:, 1], P[:, 2], m, 1.0, r_cut, n_mesh)
    a_ew = pm.ewald_force(P[:, 0], P[:, 1], P[:, 2], m, 1.0)
    e = np.linalg.norm(a_pp + a_pm - a_ew, axis=1) / np.linalg.norm(a_ew, axis=1)
    return float(np.sqrt(np.mean(e ** 2))), float(np.median(e))


def test_total_force_matches_ewald_and_improves_with_split_radius():
    rms3, med3 = _total_vs_ewald(16, 3.0)
    rms5, med5 = _total_vs_ewald(16, 5.0)
    print(f"PP + PM vs Ewald: r_cut = 3 cells: rms {rms3:.2e} median {med3:.2e}; 5 cells: rms {rms5:.2e} median {med5:.2e}")
    assert med3 < 5e-2 and rms3 < 8e-2
    assert med5 < 1e-2 and med5 < med3 / 3 and rms5 < rms3 / 3
