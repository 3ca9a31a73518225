"""Pins of the oracle's exact Riemann solver (oracle/riemann.py), the reference
the paper's Sod validation compares with (Sec. III.B, Eq. (56)).

Nothing here re-evaluates the solver's own formulas. The star states are held
to two independent sources:
  - the textbook solution of Sod's problem for gamma = 1.4, as printed to five
    significant digits in E. F. Toro, "Riemann Solvers and Numerical Methods
    for Fluid Dynamics" (3rd ed., Springer 2009), Sec. 4.3.3, Table 4.3, test 1
    (left (1, 0, 1), right (0.125, 0, 0.1));
  - the conservation laws themselves, for gamma = 1.4 and for gamma = 2 (the
    model's gas, reading c12): across the shock, the Rankine-Hugoniot jump
    conditions for mass, momentum and energy in the shock frame; across the
    rarefaction, constant entropy p / rho^gamma and the Riemann invariant
    u + 2a / (gamma - 1), with head and tail on the characteristics u - a; at
    the contact, continuous u and p. A correct star state satisfies all of
    them, and they fix it uniquely.
Inside the fan, sample_riemann is checked against the same closed-form
isentropic fan (u - a = x/t and both invariants), and away from the waves
against the star and initial states.
"""
import math

import numpy as np
import pytest

import oracle

LEFT, RIGHT = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)


def test_sod_gamma_1_4_textbook_star_state():
    st = oracle.exact_riemann(LEFT, RIGHT, gam=1.4)
    assert st["left_wave"] == "rarefaction" and st["right_wave"] == "shock"
    # printed to five significant digits: agreement within half a unit of the
    # last printed digit
    for key, printed in (("p", 0.30313), ("u", 0.92745), ("rhoL", 0.42632), ("rhoR", 0.26557)):
        assert abs(st[key] - printed) <= 5e-6, (key, st[key])


def _shock_jumps(rho0, u0, p0, rho1, u1, p1, S, gam):
    """Residuals of mass, momentum and energy flux across a shock of speed S
    (shock frame), relative to the incoming flux scales."""
    w0, w1 = u0 - S, u1 - S
    m0, m1 = rho0 * w0, rho1 * w1
    mom0, mom1 = rho0 * w0 * w0 + p0, rho1 * w1 * w1 + p1
    h0 = gam / (gam - 1.0) * p0 / rho0
    h1 = gam / (gam - 1.0) * p1 / rho1
    en0, en1 = m0 * (h0 + 0.5 * w0 * w0), m1 * (h1 + 0.5 * w1 * w1)
    return (abs(m0 - m1) / abs(m0), abs(mom0 - mom1) / abs(mom0), abs(en0 - en1) / abs(en0))


@pytest.mark.parametrize("gam", [1.4, 2.0])
def test_star_state_obeys_conservation_laws(gam):
    st = oracle.exact_riemann(LEFT, RIGHT, gam=gam)
    rL, uL, pL = LEFT
    rR, uR, pR = RIGHT
    ps, us = st["p"], st["u"]
    # the Sod data give a left rarefaction and a right shock for any gamma > 1
    assert st["left_wave"] == "rarefaction" and st["right_wave"] == "shock"
    assert pR < ps < pL and 0.0 < us
    # right shock: Rankine-Hugoniot conditions with the reported shock speed
    res = _shock_jumps(rR, uR, pR, st["rhoR"], us, ps, st["SR"], gam)
    assert max(res) < 1e-13, res
    assert st["SR"] > us  # the shock runs ahead of the contact
    # left rarefaction: isentropic, Riemann invariant, head and tail speeds
    aL = math.sqrt(gam * pL / rL)
    aS = math.sqrt(gam * ps / st["rhoL"])
    assert abs(ps / st["rhoL"] ** gam - pL / rL ** gam) < 1e-14
    inv = uL + 2.0 * aL / (gam - 1.0)
    assert abs(us + 2.0 * aS / (gam - 1.0) - inv) < 1e-13
    assert abs(st["SHL"] - (uL - aL)) < 1e-15
    assert abs(st["STL"] - (us - aS)) < 1e-13


def test_gamma_2_star_state_values():
    """The model's gas (reading c12). The values follow from the conservation
    laws above; they are held here to six decimals so that a change of the
    solver's result shows at once."""
    st = oracle.exact_riemann(LEFT, RIGHT, gam=2.0)
    for key, v in (("p", 0.285975), ("u", 0.760062), ("SR", 1.957474)):
        assert abs(st[key] - v) < 1e-6, (key, st[key])
    # gamma = 2: the textbook gamma = 1.4 state would put the shock elsewhere
    st14 = oracle.exact_riemann(LEFT, RIGHT, gam=1.4)
    assert st["SR"] - st14["SR"] > 0.2


@pytest.mark.parametrize("gam", [1.4, 2.0])
def test_sample_inside_rarefaction_fan(gam):
    st = oracle.exact_riemann(LEFT, RIGHT, gam=gam)
    rL, uL, pL = LEFT
    aL = math.sqrt(gam * pL / rL)
    t, x0 = 0.05, 0.5
    for frac in (0.2, 0.5, 0.8):
        s = st["SHL"] + frac * (st["STL"] - st["SHL"])
        rho, u, p = (float(q[0]) for q in oracle.sample_riemann(LEFT, RIGHT, [x0 + s * t], t,
                                                                  x0=x0, gam=gam))
        a = math.sqrt(gam * p / rho)
        assert abs((u - a) - s) < 1e-13  # on the characteristic x/t = u - a
        assert abs(u + 2.0 * a / (gam - 1.0) - (uL + 2.0 * aL / (gam - 1.0))) < 1e-13
        assert abs(p / rho ** gam - pL / rL ** gam) < 1e-13
        assert st["rhoL"] < rho < rL and 0.0 < u < st["u"]


@pytest.mark.parametrize("gam", [1.4, 2.0])
def test_sample_regions(gam):
    st = oracle.exact_riemann(LEFT, RIGHT, gam=gam)
    t, x0 = 0.05, 0.5
    s_pts = {
        "left": st["SHL"] - 0.1,
        "star_left": 0.5 * (st["STL"] + st["u"]),
        "star_right": 0.5 * (st["u"] + st["SR"]),
        "right": st["SR"] + 0.1,
    }
    xs = np.array([x0 + s * t for s in s_pts.values()])
    rho, u, p = oracle.sample_riemann(LEFT, RIGHT, xs, t, x0=x0, gam=gam)
    want = [LEFT, (st["rhoL"], st["u"], st["p"]), (st["rhoR"], st["u"], st["p"]), RIGHT]
    for k, w in enumerate(want):
        assert (rho[k], u[k], p[k]) == pytest.approx(w, abs=1e-15)
    # the contact: density jumps, velocity and pressure do not
    assert rho[1] != rho[2] and u[1] == u[2] and p[1] == p[2]
