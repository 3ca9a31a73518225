"""The paper's transition-layer studies (Sec. IV.A and IV.B) on the batched path.

Each study advances several copies of the paper's own shear layer
(inputs.khi_paper: interface normal to x, periodic y, outflow x) that differ
only in one transition-layer width, in one batch, logs the peak perturbed
kinetic energy E_x|max = max rho u_x^2 / 2 every step, and fits the linear
growth rate gamma = (1/2) d ln E_x|max / dt over the linear stage
(growth.growth_rate). Widths are given in grid spacings, as in the paper.

  velocity_study: rho 5 | 2, v +-0.5, p 2.5, 600 x 200 cells of 1e-3,
                  D_rho = 8, D_v varied; the paper fits ln gamma_v = a - b D_v.
  density_study:  (rho, v, p) = (5, 0.5, 1.5) | (1.25, -0.5, 1.5), cells of
                  2e-3 (300 x 100), D_v fixed, D_rho varied; the paper finds
                  gamma_rho rising with D_rho up to about 6 and flat beyond.

Host-side orchestration and post-processing only: the steps run in the HIP
library.
"""
from __future__ import annotations

import numpy as np
import torch

from . import growth, inputs, lbm

# linear stage of both studies: after the initial transient (ln E_x|max falls
# until t ~ 0.08) and before saturation
WINDOW = (0.1, 0.3)


def run_batch(setups, nsteps, graph_chunk=100, variant=None):
    """Advance the setups as one batch for nsteps; returns the (n, nsteps, 2)
    energy log on the host and the elapsed seconds (HIP events)."""
    b = lbm.Batch.from_setups(setups)
    if variant is not None:
        b.variant = variant
    fields = [s.fields() for s in setups]
    f0 = b.init(*[b.pack_scalars([f[q] for f in fields]) for q in range(4)])
    b.schedule = (b.schedule[0], graph_chunk)
    out = b.empty_f()
    ke = torch.empty((b.n, nsteps, 2), dtype=torch.float64, device=out.device)
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(st)
    lbm.lbm_batch_step(b.handle, f0, out, nsteps, ke)
    e1.record(st)
    torch.cuda.synchronize()
    return ke.cpu().numpy(), e0.elapsed_time(e1) / 1e3, b.cells


def _rates(ke, setups, window):
    return np.array([growth.growth_rate(ke[i], s.dt, window=window, column=1)[0]
                     for i, s in enumerate(setups)])


def velocity_study(widths=(4, 8, 12, 16), Drho=8, nx=600, ny=200, dx=1e-3, t_end=0.3,
                   window=WINDOW):
    """gamma_v for each D_v (grid spacings) and the fit ln gamma_v = a - b D_v."""
    setups = [inputs.khi_paper(nx, ny, dx=dx, dy=dx, Dv=w * dx, Drho=Drho * dx) for w in widths]
    nsteps = int(round(t_end / setups[0].dt)) + 1
    ke, secs, cells = run_batch(setups, nsteps)
    gam = _rates(ke, setups, window)
    slope, icpt = np.polyfit(np.asarray(widths, float), np.log(gam), 1)
    return dict(widths=list(widths), gamma=gam.tolist(), a=float(icpt), b=float(-slope),
                mlups=cells * nsteps / secs / 1e6, steps=nsteps)


def density_study(widths=(2, 4, 6, 8, 10), Dv=4, nx=300, ny=100, dx=2e-3, t_end=0.3,
                  window=WINDOW):
    """gamma_rho for each D_rho (grid spacings) and the fit gamma_rho = c + e ln D_rho
    over the widths below 6."""
    setups = [inputs.khi_paper(nx, ny, dx=dx, dy=dx, Dv=Dv * dx, Drho=w * dx, rhoL=5.0,
                               rhoR=1.25, vL=0.5, vR=-0.5, p0=1.5) for w in widths]
    nsteps = int(round(t_end / setups[0].dt)) + 1
    ke, secs, cells = run_batch(setups, nsteps)
    gam = _rates(ke, setups, window)
    w = np.asarray(widths, float)
    sel = w <= 6
    e, c = np.polyfit(np.log(w[sel]), gam[sel], 1) if sel.sum() >= 2 else (np.nan, np.nan)
    return dict(widths=list(widths), gamma=gam.tolist(), c=float(c), e=float(e),
                mlups=cells * nsteps / secs / 1e6, steps=nsteps)
