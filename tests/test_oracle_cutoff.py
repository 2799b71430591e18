"""Pins of the oracle's cutoff function g_P3M and pair kernel.

g is pinned to its definition (Sec. 2: the force between two particles
that carry the S2 density of eq. (density), found by spatial integration),
computed here by numerical quadrature of that definition, and to closed
forms of the printed polynomial (values, the factored form on [1,2],
smoothness at xi = 1 and xi = 2).
"""
from math import pi, sqrt

import numpy as np
import pytest
from scipy.integrate import quad

import oracle


def _s2_mass_within(s):
    """Mass of a unit S2 cloud of radius 1 inside radius s: rho = (3/pi)(1 - s)."""
    return 4 * s ** 3 - 3 * s ** 4 if s < 1.0 else 1.0


def s2_s2_force(r):
    """Force between two unit-mass S2 clouds of radius 1 whose centres are r
    apart, by quadrature: cloud B's density times the field of cloud A,
    averaged over shells of B (radius t) and over their directions (mu)."""
    def inner(t):
        if t == 0.0:
            return 0.0

        def f(mu):
            s = sqrt(max(r * r + t * t + 2 * r * t * mu, 0.0))
            if s == 0.0:
                return 0.0
            return _s2_mass_within(s) * (r + t * mu) / s ** 3

        mk = (1 - r * r - t * t) / (2 * r * t)
        pts = [mk] if -1 < mk < 1 else None
        val = quad(f, -1, 1, points=pts, epsabs=1e-15, epsrel=1e-13, limit=200)[0]
        return 4 * pi * t * t * (3 / pi) * (1 - t) * 0.5 * val

    pts = [p for p in (abs(1 - r), r) if 0 < p < 1]
    return quad(inner, 0, 1, points=pts or None, epsabs=1e-15, epsrel=1e-13, limit=200)[0]


def test_s2_density_normalisation():
    # eq. (density): 4 pi int_0^{rc/2} r^2 rho_PM dr = m, so rho_PP integrates to 0.
    rc, m = 0.37, 2.5
    rho = lambda r: 3 * m / pi * (2 / rc) ** 3 * (1 - r / (rc / 2))
    tot = quad(lambda r: 4 * pi * r * r * rho(r), 0, rc / 2, epsabs=1e-14)[0]
    assert abs(tot - m) < 1e-12


@pytest.mark.filterwarnings("ignore::scipy.integrate.IntegrationWarning")
@pytest.mark.parametrize("xi", [0.05, 0.3, 0.7, 1.0, 1.3, 1.7, 1.95, 2.0, 2.2, 2.7])
def test_g_equals_point_minus_cloud_force(xi):
    # With clouds of radius rc/2 = 1, xi = 2 r / rc = r; g = 1 - r^2 F_S2S2(r).
    ref = 1.0 - xi * xi * s2_s2_force(xi)
    g = oracle.gcut(xi)[0][0]
    assert abs(g - ref) < 1e-10


def test_g_special_values():
    g, dg = oracle.gcut([0.0, 1.0, 2.0, 2.0 + 1e-12, 3.0, 100.0])
    assert g[0] == 1.0
    assert abs(g[1] - 43.0 / 140.0) < 1e-15
    assert abs(g[2]) < 1e-14
    assert g[3] == 0.0 and g[4] == 0.0 and g[5] == 0.0
    assert dg[0] == 0.0
    assert abs(dg[1] + 1.0) < 1e-14


def test_g_matches_printed_form():
    # the oracle evaluates the printed polynomial of eq. (cutoff) on [0,1] and
    # its factored form on [1,2]; both agree with the printed zeta-branch form
    xi = np.linspace(0.0, 2.5, 2501)
    g, _ = oracle.gcut(xi)
    assert np.max(np.abs(g - oracle.gcut_printed(xi))) < 5e-14   # printed form: O(10) terms
    # printed form factors as -(xi-2)^5 (7 xi^3 + 22 xi^2 + 10 xi + 4)/140 on [1,2]
    x = np.linspace(1.0, 2.0, 101)
    closed = -((x - 2) ** 5) * (7 * x ** 3 + 22 * x ** 2 + 10 * x + 4) / 140.0
    assert np.max(np.abs(oracle.gcut_printed(x) - closed)) < 5e-14


def test_g_relative_accuracy_near_cutoff():
    # g ~ (6/5)(2 - xi)^5 as xi -> 2: the oracle keeps relative accuracy there
    for h in (1e-2, 1e-3, 1e-4):
        g, _ = oracle.gcut([2.0 - h])
        lead = 168.0 / 140.0 * h ** 5
        assert abs(g[0] / lead - 1.0) < 2.0 * h


def test_g_smooth_at_branch_and_end():
    h = 1e-4
    gl, _ = oracle.gcut([1 - 2 * h, 1 - h, 1.0])
    gr, _ = oracle.gcut([1.0, 1 + h, 1 + 2 * h])
    # one-sided second differences agree (g'' = 7/5 from both sides)
    d2l = (gl[2] - 2 * gl[1] + gl[0]) / h ** 2
    d2r = (gr[2] - 2 * gr[1] + gr[0]) / h ** 2
    assert abs(d2l - 1.4) < 1e-3 and abs(d2r - 1.4) < 1e-3
    # derivative continuous and equal to -1 at xi = 1
    _, d = oracle.gcut([1 - 1e-9, 1 + 1e-9])
    assert abs(d[0] + 1) < 1e-7 and abs(d[1] + 1) < 1e-7
    # g and its first four derivatives vanish at xi = 2: g ~ (2 - xi)^5
    for h in (1e-1, 3e-2, 1e-2):
        g, _ = oracle.gcut([2 - h])
        assert abs(g[0] / h ** 5 - 168.0 / 140.0) < 1.5 * h


def test_g_derivative_matches_differences():
    xi = np.linspace(0.01, 2.3, 231)
    h = 1e-6
    gp, _ = oracle.gcut(xi + h)
    gm, _ = oracle.gcut(xi - h)
    _, dg = oracle.gcut(xi)
    mask = np.abs(xi - 2.0) > 2 * h
    assert np.max(np.abs((gp - gm) / (2 * h) - dg)[mask]) < 1e-8


def test_pair_force_limits():
    rc, eps = 0.1, 1e-3
    # far inside the softening: F ~ d / eps^3
    d = np.array([1e-7, -2e-7, 3e-8])
    f = oracle.pair_force(d, rc, eps)
    assert np.allclose(f, d / eps ** 3, rtol=1e-6)
    # eps << r << rc: Newtonian d / r^3
    d = np.array([1e-4, 0.0, 0.0])
    f = oracle.pair_force(d, rc, 1e-9)
    assert abs(f[0] - 1.0 / 1e-8) / 1e8 < 1e-5
    # at and beyond the cutoff: exactly zero
    for r in (rc, rc * (1 + 1e-12), 0.2, 0.49):
        assert np.all(oracle.pair_force(np.array([0.0, r, 0.0]), rc, eps) == 0.0)
    # antisymmetric
    d = np.array([0.013, -0.02, 0.031])
    assert np.array_equal(oracle.pair_force(d, rc, eps), -oracle.pair_force(-d, rc, eps))


def test_pair_jacobian_matches_differences():
    rc, eps = 0.1, 1e-3
    rng = np.random.default_rng(5)
    for _ in range(20):
        d = rng.uniform(-0.06, 0.06, 3)
        w = rng.standard_normal(3)
        jw = oracle.pair_jac(d, w, rc, eps)
        h = 1e-7
        num = np.zeros(3)
        for a in range(3):
            e = np.zeros(3)
            e[a] = h
            num += (oracle.pair_force(d + e, rc, eps) - oracle.pair_force(d - e, rc, eps)) / (2 * h) * w[a]
        assert np.allclose(jw, num, rtol=1e-5, atol=1e-6 * np.abs(jw).max())
    # at d = 0: J = phi(0) I = eps^-3 I
    assert np.allclose(oracle.pair_jac(np.zeros(3), np.array([1.0, 2.0, 3.0]), rc, eps),
                       np.array([1.0, 2.0, 3.0]) / eps ** 3, rtol=1e-14)
