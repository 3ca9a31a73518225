"""Pins of the oracle's WENO5 flux (Sec. III.A, Eqs. (48)-(55)) against facts
of the Jiang-Shu scheme the paper cites: exactness on quadratics for any
nonlinear weights, the optimal-weight limit, fifth-order convergence on smooth
data, the non-oscillatory choice at a jump, and the mirror image used for
negative velocities."""
import numpy as np
import pytest


def test_quadratic_exact_any_weights(orc):
    """For quadratic F every candidate reconstructs the face value exactly, so
    h_{I+1/2} - h_{I-1/2} = dx F'(x_I) whatever the weights are."""
    rng = np.random.default_rng(0)
    for _ in range(200):
        a0, a1, a2 = rng.uniform(-3, 3, 3)
        dx = rng.uniform(0.01, 1.0)
        x0 = rng.uniform(-1, 1)
        xs = x0 + dx * np.arange(-3, 4)
        F = a0 + a1 * xs + a2 * xs ** 2
        exact = dx * (a1 + 2 * a2 * x0)  # F'(x_I) dx, I at index 3
        hp = orc.weno5(*F[1:6])  # face I+1/2 uses I-2..I+2
        hm = orc.weno5(*F[0:5])  # face I-1/2 uses I-3..I+1
        scale = max(1.0, np.abs(F).max())
        assert hp - hm == pytest.approx(exact, abs=1e-13 * scale)
        # right-upwinded (mirror) stencils: face I+1/2 uses I+3..I-1
        hp = orc.weno5(*F[6:1:-1])
        hm = orc.weno5(*F[5:0:-1])
        assert hp - hm == pytest.approx(exact, abs=1e-13 * scale)


def test_linear_data_uses_optimal_weights(orc):
    """Linear data gives sigma_1 = sigma_2 = sigma_3, hence omega = delta =
    (1/10, 3/5, 3/10) and h = (2a - 13b + 47c + 27d - 3e)/60."""
    rng = np.random.default_rng(1)
    for _ in range(100):
        c0, s = rng.uniform(-2, 2, 2)
        F = c0 + s * np.arange(5)
        h = orc.weno5(*F)
        a, b, c, d, e = F
        assert h == pytest.approx((2 * a - 13 * b + 47 * c + 27 * d - 3 * e) / 60, abs=1e-14)


@pytest.mark.parametrize("amp", [1.0, 0.05, 1e-3])
def test_fifth_order_convergence(orc, amp):
    """Observed order of (h_{I+1/2}-h_{I-1/2})/dx -> F' on smooth periodic data."""
    errs = []
    Ns = [32, 64, 128, 256]
    for N in Ns:
        dx = 1.0 / N
        x = np.arange(N) * dx
        F = amp * np.sin(2 * np.pi * x) + 1.0
        for sign in (1, -1):
            h = orc.weno_periodic_line(F, sign)
            d = (h - np.roll(h, 1)) / dx
            ex = amp * 2 * np.pi * np.cos(2 * np.pi * x)
            if sign == 1:
                errs.append(np.abs(d - ex).max())
            else:
                assert np.abs(d - ex).max() < 2 * errs[-1] + 1e-12
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert orders.min() > 4.5, orders


def test_mirror_image_bitwise(orc):
    """The v < 0 flux is the v >= 0 formula on the reversed line."""
    rng = np.random.default_rng(2)
    n = 37
    F = rng.uniform(-1, 1, n)
    hm = orc.weno_periodic_line(F, -1)
    G = F[::-1].copy()
    hp = orc.weno_periodic_line(G, +1)
    for I in range(n):
        assert hm[I] == hp[(n - 2 - I) % n]


def test_odd_symmetry_bitwise(orc):
    rng = np.random.default_rng(3)
    for _ in range(100):
        s = rng.uniform(-5, 5, 5)
        assert orc.weno5(*(-s)) == -orc.weno5(*s)


def test_non_oscillatory_at_jump(orc):
    """A jump between I and I+1: the stencil that does not cross it
    (candidate 1, all on the left) receives nearly all the weight."""
    h = orc.weno5(0.0, 0.0, 0.0, 1.0, 1.0)
    assert abs(h) < 1e-10
    h = orc.weno5(1.0, 1.0, 1.0, 1.0, 0.0)  # jump between I+1 and I+2
    assert abs(h - 1.0) < 1e-10


def test_gradient_matches_fd(orc):
    rng = np.random.default_rng(4)
    for _ in range(50):
        s = rng.uniform(-2, 2, 5)
        g = orc.weno5_grad(*s)
        for k in range(5):
            h = 1e-6
            sp, sm = s.copy(), s.copy()
            sp[k] += h
            sm[k] -= h
            fd = (orc.weno5(*sp) - orc.weno5(*sm)) / (2 * h)
            assert g[k] == pytest.approx(fd, rel=1e-6, abs=1e-7)
