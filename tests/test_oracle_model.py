"""Pins of the oracle's cell-local physics against what the paper and the
mathematics fix: the velocity set's isotropy (Sec. II.A), the weight sum rules
(Sec. II.C), the equilibrium's moment constraints (Sec. II.B) and the
conservation properties of the BGK collision."""
import json
import os
from fractions import Fraction as Fr
from itertools import product

import numpy as np
import pytest

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))
VK = tuple(GOLD["particle_speeds"]["value"])


def exact_weights(T):
    """Solve the sum rules Eqs. (40)-(43) in exact rational arithmetic for
    (F_0, F_1, F_2, F_3); independent of the closed form Eq. (44)."""
    T = Fr(T)
    v2 = [Fr(int(v)) ** 2 for v in VK]
    A = [[v ** 1 for v in v2], [v ** 2 for v in v2], [v ** 3 for v in v2]]
    b = [T / 3, Fr(4, 3) * T ** 2, 8 * T ** 3]
    # Gauss elimination on a 3x3 system of Fractions
    M = [row[:] + [bb] for row, bb in zip(A, b)]
    for c in range(3):
        piv = next(r for r in range(c, 3) if M[r][c] != 0)
        M[c], M[piv] = M[piv], M[c]
        for r in range(3):
            if r != c and M[r][c] != 0:
                fac = M[r][c] / M[c][c]
                M[r] = [x - fac * y for x, y in zip(M[r], M[c])]
    F = [M[r][3] / M[r][r] for r in range(3)]
    return [1 - 6 * sum(F)] + F


def test_velocity_table_exact(orc):
    vx, vy, vsq, shell, mx, my = orc.velocity_table(VK)
    assert vx[0] == 0 and vy[0] == 0
    for k in range(3):
        for j in range(6):
            i = 1 + 6 * k + j
            ang = (j + 1) * np.pi / 3.0
            assert vx[i] == pytest.approx(VK[k] * np.cos(ang), abs=4e-15)
            assert vy[i] == pytest.approx(VK[k] * np.sin(ang), abs=4e-15)
            assert vsq[i] == VK[k] ** 2
            assert shell[i] == k + 1
    # directions 3 and 6 lie exactly on the x axis
    assert all(vy[1 + 6 * k + 2] == 0.0 and vy[1 + 6 * k + 5] == 0.0 for k in range(3))
    # mirror partners
    for i in range(19):
        assert vx[mx[i]] == -vx[i] and vy[mx[i]] == vy[i]
        assert vx[my[i]] == vx[i] and vy[my[i]] == -vy[i]


def test_isotropy(orc):
    """Eqs. (7)-(9): rank 2 = 3 v^2 delta, rank 4 = 3/4 v^4 Delta, odd ranks
    vanish, per speed shell."""
    vx, vy, *_ = orc.velocity_table(VK)
    c2 = GOLD["isotropy_rank2_coeff"]["value"]
    c4 = GOLD["isotropy_rank4_coeff"]["value"]
    d = np.eye(2)
    for k in range(3):
        V = np.stack([vx[1 + 6 * k:7 + 6 * k], vy[1 + 6 * k:7 + 6 * k]], axis=1)
        vk = VK[k]
        for rank in (1, 3, 5):
            for idx in product(range(2), repeat=rank):
                s = np.sum(np.prod(V[:, list(idx)], axis=1))
                assert abs(s) < 1e-13 * vk ** rank
        for a, b in product(range(2), repeat=2):
            s = np.sum(V[:, a] * V[:, b])
            assert s == pytest.approx(c2 * vk ** 2 * d[a, b], abs=1e-13)
        for a, b, c, e in product(range(2), repeat=4):
            s = np.sum(V[:, a] * V[:, b] * V[:, c] * V[:, e])
            Delta = d[a, b] * d[c, e] + d[a, c] * d[b, e] + d[a, e] * d[b, c]
            assert s == pytest.approx(c4 * vk ** 4 * Delta, abs=1e-12)


@pytest.mark.parametrize("T", ["1", "4/5", "1/2", "5/4", "1/3", "3/10", "3/2"])
def test_weights_exact_rationals(orc, T):
    ex = exact_weights(Fr(T))
    got = orc.weights(float(Fr(T)), VK)
    for a, b in zip(got, ex):
        assert a == pytest.approx(float(b), abs=2e-16 * 8)


def test_weights_known_values(orc):
    # special values: F_3 vanishes at T = 1/2 and 1/3; F_0 < 0 at T = 5/4
    assert exact_weights(Fr(1)) == [Fr(1, 18), Fr(1, 9), Fr(7, 180), Fr(1, 135)]
    assert exact_weights(Fr(1, 2))[3] == 0 and exact_weights(Fr(1, 3))[3] == 0
    assert exact_weights(Fr(5, 4))[0] == Fr(-7, 48)
    assert abs(orc.weights(0.5, VK)[3]) < 1e-17


@pytest.mark.parametrize("T", np.linspace(0.2, 2.0, 13))
def test_weights_sum_rules(orc, T):
    """Eqs. (40)-(43)."""
    F = orc.weights(T, VK)
    v = np.array(VK)
    assert F[0] + 6 * F[1:].sum() == pytest.approx(1.0, abs=1e-14)
    assert np.dot(F[1:], v ** 2) == pytest.approx(T / 3, rel=1e-14)
    assert np.dot(F[1:], v ** 4) == pytest.approx(4 * T ** 2 / 3, rel=1e-14)
    assert np.dot(F[1:], v ** 6) == pytest.approx(8 * T ** 3, rel=1e-14)


def _rand_states(n, seed):
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.1, 5.0, n)
    ang = rng.uniform(0, 2 * np.pi, n)
    mag = rng.uniform(0, 0.6, n)
    T = rng.uniform(0.3, 1.5, n)
    return rho, mag * np.cos(ang), mag * np.sin(ang), T


def test_feq_moment_constraints(orc):
    """Eqs. (10)-(12), and the requirement families Eqs. (30)-(39) that they
    imply: mass, momentum, temperature, second moment P delta + rho u u and
    energy flux u (2P + rho u^2/2) of f^eq."""
    vx, vy, vsq, *_ = orc.velocity_table(VK)
    V = np.stack([vx, vy], 1)
    worst = 0.0
    for rho, ux, uy, T in zip(*_rand_states(300, 1)):
        fe = orc.feq_cell(rho, ux, uy, T, VK)
        u = np.array([ux, uy])
        P = rho * T
        got_rho = fe.sum()
        got_j = V.T @ fe
        got_T = np.sum(fe * 0.5 * np.sum((V - u) ** 2, 1)) / rho
        got_Pi = np.einsum("i,ia,ib->ab", fe, V, V)
        exp_Pi = P * np.eye(2) + rho * np.outer(u, u)
        got_q = np.einsum("i,i,ia->a", fe, 0.5 * vsq, V)
        exp_q = u * (2 * P + 0.5 * rho * u @ u)
        scale = rho * (1 + T) * 10
        for a, b in [(got_rho, rho), (got_T * rho, P)] + list(zip(got_j, rho * u)) + \
                list(zip(got_Pi.ravel(), exp_Pi.ravel())) + list(zip(got_q, exp_q)):
            worst = max(worst, abs(a - b) / scale)
    assert worst < 1e-14


def test_feq_rest_state(orc):
    """u = 0: f_i^eq = rho F_k(T) (Eq. (28) with xi = 0)."""
    for T in (0.5, 0.8, 1.0, 1.25):
        F = orc.weights(T, VK)
        fe = orc.feq_cell(2.0, 0.0, 0.0, T, VK)
        assert fe[0] == pytest.approx(2.0 * F[0], rel=1e-15, abs=1e-16)
        for k in range(3):
            assert np.allclose(fe[1 + 6 * k:7 + 6 * k], 2.0 * F[k + 1], rtol=1e-15, atol=1e-17)


def test_moments_roundtrip(orc):
    for rho, ux, uy, T in zip(*_rand_states(200, 2)):
        m = orc.moments_cell(orc.feq_cell(rho, ux, uy, T, VK), VK)
        assert m == pytest.approx([rho, ux, uy, T], rel=1e-13, abs=1e-14)


def test_collision_conserves(orc):
    """BGK relaxation toward f^eq(moments(f)) changes no conserved moment."""
    vx, vy, vsq, *_ = orc.velocity_table(VK)
    rng = np.random.default_rng(3)
    base = np.array([0.3] + [0.05] * 6 + [0.04] * 6 + [0.01] * 6)
    for _ in range(200):
        f = base * (1 + 0.4 * rng.uniform(-1, 1, 19))
        rho, ux, uy, T = orc.moments_cell(f, VK)
        d = f - orc.feq_cell(rho, ux, uy, T, VK)
        assert abs(d.sum()) < 1e-15
        assert abs(d @ vx) < 1e-14 and abs(d @ vy) < 1e-14
        assert abs(d @ (0.5 * vsq)) < 1e-14


def test_feq_partials_fd(orc):
    for rho, ux, uy, T in zip(*_rand_states(20, 4)):
        x0 = np.array([rho, ux, uy, T])
        for i in range(19):
            d = orc.feq_partials(rho, ux, uy, T, i, VK)
            for q in range(4):
                h = 1e-6 * max(1.0, abs(x0[q]))
                xp, xm = x0.copy(), x0.copy()
                xp[q] += h
                xm[q] -= h
                fd = (orc.feq_cell(*xp, VK)[i] - orc.feq_cell(*xm, VK)[i]) / (2 * h)
                assert d[q] == pytest.approx(fd, rel=1e-6, abs=1e-8)


def test_gamma_two_from_mach_numbers():
    """The paper's Mach numbers 0.5 and 0.32 (Sec. IV.A) for rho = 5 and 2 at
    P = 2.5 and |v| = 0.5 fix the sound speed sqrt(gamma P / rho) with
    gamma = 2, the value the Riemann oracle uses for the Sod check."""
    rL, rR = GOLD["khi_rho_L_R"]["value"]
    P = GOLD["khi_pressure"]["value"]
    mL, mR = GOLD["khi_mach_L_R"]["value"]
    for gam, ok in ((2.0, True), (1.4, False)):
        ML = 0.5 / np.sqrt(gam * P / rL)
        MR = 0.5 / np.sqrt(gam * P / rR)
        assert (abs(ML - mL) < 0.005 and abs(MR - mR) < 0.005) == ok
