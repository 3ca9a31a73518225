"""Linear growth rate of the Kelvin-Helmholtz instability from an energy log.

Host-side post-processing of the per-step kinetic-energy logs that the step
kernels write (lbm_step / lbm_batch_step ke_log): no field data is touched.

Sec. IV of arXiv:1010.4124 measures the growth rate gamma from the peak
perturbed kinetic energy: in the linear stage the perturbation amplitude
grows like exp(gamma t), the energy like exp(2 gamma t), so gamma is half the
least-squares slope of ln E_max(t) over the linear stage (Sec. IV.A). With
the interface normal along y here, the perturbed energy is rho u_y^2 / 2.
Sec. IV.A also quotes the classical sharp-interface rate
gamma_c = k sqrt(rho1 rho2) (v1 - v2) / (rho1 + rho2), an upper bound that
finite transition layers only lower.
"""
from __future__ import annotations

import math

import numpy as np


def growth_rate(ke, dt, window=(0.02, 0.1), column=1):
    """gamma = (1/2) d ln E / dt, least squares over t in [window[0], window[1]].

    ke: (nsteps, 2) log with ke[n] = (sum, max) of rho u_y^2 / 2 in the state
    at time t_n = n dt; column 1 (the maximum) is the paper's diagnostic,
    column 0 (the domain integral) the smoother alternative. Returns
    (gamma, r2) with r2 the coefficient of determination of the fit.
    """
    ke = np.asarray(ke, dtype=np.float64)
    t = np.arange(ke.shape[0]) * float(dt)
    sel = (t >= window[0] - 0.5 * dt) & (t <= window[1] + 0.5 * dt)
    if sel.sum() < 3:
        raise ValueError("fewer than three samples inside the fit window")
    E = ke[sel, column]
    if not np.all(E > 0):
        raise ValueError("energy must be positive inside the fit window")
    y = np.log(E)
    x = t[sel]
    A = np.stack([x - x.mean(), np.ones_like(x)], axis=1)
    coef, *_ = np.linalg.lstsq(A, y, rcond=None)
    resid = y - A @ coef
    ss = float(((y - y.mean()) ** 2).sum())
    r2 = 1.0 - float((resid ** 2).sum()) / ss if ss > 0 else 1.0
    return 0.5 * float(coef[0]), r2


def linear_stage(ke, dt, width=0.1, tmin=0.02, step=0.01, column=0):
    """Growth rate over the linear growth stage, found in the log itself.

    Sec. IV fits the slope of ln E to "the initial growth stage", after the
    initial transient and before saturation, in each run separately. Here
    that stage is the window [a, a + width] (a >= tmin, on a grid of `step`)
    in which ln E rises and is closest to a straight line: of the windows
    with a positive slope, the one whose least-squares fit has the largest
    coefficient of determination r2. Column 0 (the domain integral of
    rho u_n^2 / 2) is the default: with walls in y, sound waves trapped
    between them make the peak (column 1) jump from place to place, while
    both grow like exp(2 gamma t) in the linear stage.

    Returns (gamma, r2, a), or (nan, 0.0, nan) when no window rises.
    """
    ke = np.asarray(ke, dtype=np.float64)
    t_end = (ke.shape[0] - 1) * float(dt)
    best = (math.nan, 0.0, math.nan)
    for a in np.arange(tmin, t_end - width + 0.5 * step, step):
        try:
            g, r2 = growth_rate(ke, dt, window=(a, a + width), column=column)
        except ValueError:
            continue
        if g > 0.0 and r2 > best[1]:
            best = (g, r2, float(a))
    return best


def classical_rate(Lx, rho1=5.0, rho2=2.0, dv=1.0, mode=1):
    """gamma_c = k sqrt(rho1 rho2) dv / (rho1 + rho2), k = 2 pi mode / Lx."""
    k = 2.0 * math.pi * mode / Lx
    return k * math.sqrt(rho1 * rho2) * dv / (rho1 + rho2)
