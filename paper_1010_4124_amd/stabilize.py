"""Adjoint-driven stabilisation of the shear layer.

The paper concludes that widening the velocity and density transition layers
damps the Kelvin-Helmholtz instability (Sec. IV.C and Sec. V). Here that is
turned into an optimisation: choose (D_v, D_rho) within bounds to minimise
the perturbation energy integrated over the linear stage,
J = dt sum_{n0..n1} E_y(n) (objective.KHIProblem), using the discrete
adjoint gradient. The widths are optimised in log space (theta = ln D),
where the normalised gradient d ln J / d theta = D (dJ/dD) / J is O(1), by
projected gradient descent with Armijo backtracking, so J never increases.

Host-side orchestration only: each J and gradient is one forward run and one
adjoint sweep of the HIP library.
"""
from __future__ import annotations

import math

import numpy as np


def stabilize(problem, Dv0, Drho0, amps, iters=4, step=0.5, bounds=(0.005, 0.08),
              shrink=0.5, max_halvings=6, armijo=1e-4):
    """Minimise J(D_v, D_rho) from (Dv0, Drho0); amps fixed. Returns the history
    [{"Dv", "Drho", "J", "grad": (dJ/dDv, dJ/dDrho)}, ...]."""
    lo, hi = math.log(bounds[0]), math.log(bounds[1])
    theta = np.array([math.log(Dv0), math.log(Drho0)])
    amps = np.asarray(amps, dtype=np.float64)

    def evaluate(th):
        Dv, Drho = math.exp(th[0]), math.exp(th[1])
        J, ck = problem.run(Dv, Drho, amps)
        gDv, gDrho, _ = problem.gradient(Dv, Drho, amps, ck=ck)
        return J, np.array([gDv, gDrho]), Dv, Drho

    J, g, Dv, Drho = evaluate(theta)
    hist = [dict(Dv=Dv, Drho=Drho, J=J, grad=tuple(g))]
    for _ in range(iters):
        # normalised gradient of ln J with respect to ln D
        d = np.array([Dv, Drho]) * g / J
        t = step
        for _ in range(max_halvings + 1):
            trial = np.clip(theta - t * d, lo, hi)
            Dv_t, Drho_t = math.exp(trial[0]), math.exp(trial[1])
            J_t, _ = problem.run(Dv_t, Drho_t, amps, keep_checkpoints=False)
            # sufficient decrease of ln J along the projected step
            if math.log(J_t) <= math.log(J) + armijo * float(d @ (trial - theta)):
                break
            t *= shrink
        else:
            break  # no decrease within the halvings: stationary within bounds
        theta = trial
        J, g, Dv, Drho = evaluate(theta)
        hist.append(dict(Dv=Dv, Drho=Drho, J=J, grad=tuple(g)))
    return hist
