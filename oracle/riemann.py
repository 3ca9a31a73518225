"""Exact solution of the 1-D Riemann problem for an ideal gas (test infrastructure).

The paper validates its model on the Sod shock tube against the analytical
solution (Sec. III.B). The model's energy flux rho u (2T + u^2/2)
(Sec. II.B) gives internal energy rho T = P per unit volume, i.e. a gas with
ratio of specific heats gamma = 2, which is the value used here by default.

This is the textbook exact solver: the star pressure p* is the root of
f_L(p) + f_R(p) + (u_R - u_L) = 0, with f_K the shock (Rankine-Hugoniot) or
rarefaction (isentropic) branch, solved by Newton iteration; the solution is
then sampled along x/t.
"""
from __future__ import annotations

import math

import numpy as np


def _fK(p, rho, pK, gam):
    a = math.sqrt(gam * pK / rho)
    if p > pK:  # shock branch
        A = 2.0 / ((gam + 1.0) * rho)
        B = (gam - 1.0) / (gam + 1.0) * pK
        f = (p - pK) * math.sqrt(A / (p + B))
        df = math.sqrt(A / (B + p)) * (1.0 - 0.5 * (p - pK) / (B + p))
    else:  # rarefaction branch
        f = 2.0 * a / (gam - 1.0) * ((p / pK) ** ((gam - 1.0) / (2.0 * gam)) - 1.0)
        df = 1.0 / (rho * a) * (p / pK) ** (-(gam + 1.0) / (2.0 * gam))
    return f, df


def exact_riemann(left, right, gam=2.0, tol=1e-14, maxit=200):
    """Star state of the Riemann problem.

    left, right: (rho, u, p). Returns dict with p*, u*, rho*_L, rho*_R and the
    wave speeds (shock speeds or rarefaction head/tail speeds).
    """
    rL, uL, pL = map(float, left)
    rR, uR, pR = map(float, right)
    aL, aR = math.sqrt(gam * pL / rL), math.sqrt(gam * pR / rR)
    if 2.0 * (aL + aR) / (gam - 1.0) <= uR - uL:
        raise ValueError("vacuum generated")
    p = max(tol, 0.5 * (pL + pR))
    for _ in range(maxit):
        fL, dL = _fK(p, rL, pL, gam)
        fR, dR = _fK(p, rR, pR, gam)
        pn = p - (fL + fR + uR - uL) / (dL + dR)
        pn = max(pn, tol)
        if abs(pn - p) <= tol * 0.5 * (pn + p):
            p = pn
            break
        p = pn
    fL, _ = _fK(p, rL, pL, gam)
    fR, _ = _fK(p, rR, pR, gam)
    u = 0.5 * (uL + uR) + 0.5 * (fR - fL)
    g1 = (gam - 1.0) / (gam + 1.0)
    out = {"p": p, "u": u}
    if p > pL:
        out["rhoL"] = rL * (p / pL + g1) / (g1 * p / pL + 1.0)
        out["SL"] = uL - aL * math.sqrt((gam + 1.0) / (2.0 * gam) * p / pL + (gam - 1.0) / (2.0 * gam))
        out["left_wave"] = "shock"
    else:
        out["rhoL"] = rL * (p / pL) ** (1.0 / gam)
        aLs = aL * (p / pL) ** ((gam - 1.0) / (2.0 * gam))
        out["SHL"], out["STL"] = uL - aL, u - aLs
        out["left_wave"] = "rarefaction"
    if p > pR:
        out["rhoR"] = rR * (p / pR + g1) / (g1 * p / pR + 1.0)
        out["SR"] = uR + aR * math.sqrt((gam + 1.0) / (2.0 * gam) * p / pR + (gam - 1.0) / (2.0 * gam))
        out["right_wave"] = "shock"
    else:
        out["rhoR"] = rR * (p / pR) ** (1.0 / gam)
        aRs = aR * (p / pR) ** ((gam - 1.0) / (2.0 * gam))
        out["SHR"], out["STR"] = uR + aR, u + aRs
        out["right_wave"] = "rarefaction"
    return out


def sample_riemann(left, right, x, t, x0=0.5, gam=2.0):
    """(rho, u, p) of the exact solution at positions x and time t > 0."""
    rL, uL, pL = map(float, left)
    rR, uR, pR = map(float, right)
    aL, aR = math.sqrt(gam * pL / rL), math.sqrt(gam * pR / rR)
    st = exact_riemann(left, right, gam)
    ps, us = st["p"], st["u"]
    x = np.asarray(x, dtype=np.float64)
    rho, u, p = np.empty_like(x), np.empty_like(x), np.empty_like(x)
    for n, xx in enumerate(x.ravel()):
        s = (xx - x0) / t
        if s <= us:  # left of the contact
            if st["left_wave"] == "shock":
                W = (rL, uL, pL) if s <= st["SL"] else (st["rhoL"], us, ps)
            else:
                if s <= st["SHL"]:
                    W = (rL, uL, pL)
                elif s > st["STL"]:
                    W = (st["rhoL"], us, ps)
                else:
                    c = 2.0 / (gam + 1.0) + (gam - 1.0) / ((gam + 1.0) * aL) * (uL - s)
                    W = (rL * c ** (2.0 / (gam - 1.0)),
                         2.0 / (gam + 1.0) * (aL + 0.5 * (gam - 1.0) * uL + s),
                         pL * c ** (2.0 * gam / (gam - 1.0)))
        else:
            if st["right_wave"] == "shock":
                W = (rR, uR, pR) if s >= st["SR"] else (st["rhoR"], us, ps)
            else:
                if s >= st["SHR"]:
                    W = (rR, uR, pR)
                elif s < st["STR"]:
                    W = (st["rhoR"], us, ps)
                else:
                    c = 2.0 / (gam + 1.0) - (gam - 1.0) / ((gam + 1.0) * aR) * (uR - s)
                    W = (rR * c ** (2.0 / (gam - 1.0)),
                         2.0 / (gam + 1.0) * (-aR + 0.5 * (gam - 1.0) * uR + s),
                         pR * c ** (2.0 * gam / (gam - 1.0)))
        rho.flat[n], u.flat[n], p.flat[n] = W
    return rho, u, p
