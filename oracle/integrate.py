"""FP64 CPU oracle of the multiple-stepsize TreePM integrator -- TEST
INFRASTRUCTURE (same import rules as the rest of ``oracle``).

One step of length dt (Sec. 3: one PM cycle and two PP cycles), an impulse
splitting of the long-range and short-range forces:

    v += dt/2 a_PM(x)
    repeat 2:  v += dt/4 a_PP(x);  x += dt/2 v (mod 1);  v += dt/4 a_PP(x)
    v += dt/2 a_PM(x)

``pp`` and ``pm`` are callables (x [N,3] -> a [N,3]); the accelerations of
a step's end are those of the next step's start.
"""
from __future__ import annotations

import numpy as np


def respa_step(x, v, pp, pm, dt, a_pp=None, a_pm=None):
    """One step; returns (x, v, a_pp, a_pm) at the step's end (new arrays)."""
    x = np.array(x, dtype=np.float64)
    v = np.array(v, dtype=np.float64)
    if a_pp is None:
        a_pp = pp(x)
    if a_pm is None:
        a_pm = pm(x)
    v = v + 0.5 * dt * a_pm
    for _ in range(2):
        v = v + 0.25 * dt * a_pp
        x = np.mod(x + 0.5 * dt * v, 1.0)
        x[x >= 1.0] = 0.0
        a_pp = pp(x)
        v = v + 0.25 * dt * a_pp
    a_pm = pm(x)
    v = v + 0.5 * dt * a_pm
    return x, v, a_pp, a_pm


def integrate(x, v, pp, pm, dt, n_steps):
    a_pp = a_pm = None
    for _ in range(n_steps):
        x, v, a_pp, a_pm = respa_step(x, v, pp, pm, dt, a_pp, a_pm)
    return x, v
