"""GPU multiple-stepsize TreePM integrator against the oracle integrator.

theta = 0 makes the GPU PP sum the exact pair sum within r_cut, so with the
FP64 kernels the GPU trajectory equals the oracle's (brute-force PP + PM)
to rounding after a few steps; the FP32 kernels stay within FP32 error.
Reversibility and momentum conservation are checked on the GPU as well."""
import sys

import numpy as np
import pytest
import torch

import oracle
import paper_1211_4406_amd as srf
from oracle import integrate, pm

pytestmark = pytest.mark.gpu

R_CUT, EPS, N_MESH, DT, STEPS = 3.0 / 16, 1e-2, 16, 2e-3, 6


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _system(n=512, seed=9):
    rng = np.random.default_rng(seed)
    return rng.random((n, 3)), 0.05 * rng.standard_normal((n, 3)), np.full(n, 1.0 / n)


def _oracle_run(x, v, m, steps=STEPS):
    def pp(p):
        return oracle.brute_force(p[:, 0], p[:, 1], p[:, 2], m, 1.0, R_CUT, EPS, method="n2")

    def pmf(p):
        return pm.pm_force(p[:, 0], p[:, 1], p[:, 2], m, 1.0, R_CUT, N_MESH)
    return integrate.integrate(x, v, pp, pmf, DT, steps)


def _gpu_run(x, v, m, precision, steps=STEPS, sign=1.0):
    p = srf.Params(G=1.0, r_cut=R_CUT, eps=EPS, theta=0.0, precision=precision)
    xt = torch.tensor(x, dtype=torch.float64, device="cuda")
    vt = torch.tensor(v * sign, dtype=torch.float64, device="cuda")
    mt = torch.tensor(m, dtype=torch.float64, device="cuda")
    it = srf.TreePMIntegrator(p, N_MESH)
    for _ in range(steps):
        it.step(xt, vt, mt, DT)
    torch.cuda.synchronize()
    return xt.cpu().numpy(), vt.cpu().numpy()


def _pdiff(a, b):
    d = a - b
    return np.max(np.abs(d - np.rint(d)))


@pytest.mark.parametrize("precision,tol_x,tol_v", [(srf.FP64, 1e-11, 1e-9), (srf.FP32_REL, 1e-8, 1e-6)])
def test_trajectory_matches_oracle(precision, tol_x, tol_v):
    x, v, m = _system()
    say(f"[gpu] integrator precision={precision} n={x.shape[0]} steps={STEPS}")
    xo, vo = _oracle_run(x, v, m)
    xg, vg = _gpu_run(x, v, m, precision)
    dx, dv = _pdiff(xg, xo), np.max(np.abs(vg - vo))
    say(f"    max |dx| {dx:.3e}, max |dv| {dv:.3e} (|v| ~ {np.abs(vo).max():.2e})")
    assert dx < tol_x and dv < tol_v


def test_reversible_and_momentum_conserving():
    x, v, m = _system()
    x1, v1 = _gpu_run(x, v, m, srf.FP64)
    x2, v2 = _gpu_run(x1, v1, m, srf.FP64, sign=-1.0)
    p0, p1 = (m[:, None] * v).sum(0), (m[:, None] * v1).sum(0)
    say(f"[gpu] reversibility: max |dx| {_pdiff(x2, x):.3e}, max |dv| {np.max(np.abs(v2 + v)):.3e}; "
        f"momentum change {np.max(np.abs(p1 - p0)):.3e}")
    assert _pdiff(x2, x) < 1e-11 and np.max(np.abs(v2 + v)) < 1e-9
    assert np.max(np.abs(p1 - p0)) < 1e-12 * np.sum(m * np.linalg.norm(v1, axis=1))
