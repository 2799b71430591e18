"""Pins of the oracle's multiple-stepsize integrator: time reversibility,
momentum conservation, and the reduction to two leapfrog steps of dt/2
when the long-range force is switched off."""
import numpy as np

import oracle
from oracle import integrate, pm


def _system(n=64, seed=5):
    rng = np.random.default_rng(seed)
    x = rng.random((n, 3))
    v = 0.05 * rng.standard_normal((n, 3))
    m = np.full(n, 1.0 / n)
    return x, v, m


def _forces(m, r_cut=3.0 / 16, eps=1e-2, n_mesh=16):
    def pp(x):
        return oracle.brute_force(x[:, 0], x[:, 1], x[:, 2], m, 1.0, r_cut, eps, method="n2")

    def pmf(x):
        return pm.pm_force(x[:, 0], x[:, 1], x[:, 2], m, 1.0, r_cut, n_mesh)
    return pp, pmf


def test_time_reversible():
    x0, v0, m = _system()
    pp, pmf = _forces(m)
    x1, v1 = integrate.integrate(x0, v0, pp, pmf, 2e-3, 6)
    x2, v2 = integrate.integrate(x1, -v1, pp, pmf, 2e-3, 6)
    dx = x2 - x0
    dx -= np.rint(dx)
    assert np.max(np.abs(dx)) < 1e-12 and np.max(np.abs(v2 + v0)) < 1e-11


def test_momentum_conserved():
    x0, v0, m = _system()
    pp, pmf = _forces(m)
    x1, v1 = integrate.integrate(x0, v0, pp, pmf, 2e-3, 6)
    p0, p1 = (m[:, None] * v0).sum(0), (m[:, None] * v1).sum(0)
    assert np.max(np.abs(p1 - p0)) < 1e-12 * np.sum(m * np.linalg.norm(v1, axis=1))


def test_without_long_range_force_is_two_leapfrog_steps():
    x0, v0, m = _system()
    pp, _ = _forces(m)
    zero = lambda x: np.zeros_like(x)   # noqa: E731
    x1, v1, _, _ = integrate.respa_step(x0, v0, pp, zero, 2e-3)
    x, v = x0.copy(), v0.copy()
    h = 1e-3
    for _ in range(2):   # kick-drift-kick of h
        v = v + 0.5 * h * pp(x)
        x = np.mod(x + h * v, 1.0)
        v = v + 0.5 * h * pp(x)
    assert np.max(np.abs(x1 - x)) < 1e-15 and np.max(np.abs(v1 - v)) < 1e-15
