"""Growth-rate fit (host post-processing of the energy logs) against closed
forms: E = E0 exp(2 gamma t) gives gamma exactly, noise and samples outside
the window do not bias it, and the classical rate matches its formula at the
numbers worked out by hand."""
import math

import numpy as np
import pytest

from paper_1010_4124_amd import growth


def test_exact_exponential():
    dt, n = 1e-5, 12001
    t = np.arange(n) * dt
    for gamma in (0.3, 2.5, 7.0):
        E = 1e-9 * np.exp(2 * gamma * t)
        ke = np.stack([E * 3.0, E], axis=1)
        g, r2 = growth.growth_rate(ke, dt)
        assert abs(g - gamma) < 1e-9 * gamma and r2 > 1 - 1e-12
        g0, _ = growth.growth_rate(ke, dt, column=0)
        assert abs(g0 - gamma) < 1e-9 * gamma


def test_window_excludes_transient_and_saturation():
    dt = 1e-4
    t = np.arange(2001) * dt
    E = np.where(t < 0.02, 1.0, 1e-6 * np.exp(2 * 4.0 * t))  # transient before the window
    E = np.where(t > 0.1, 1e-6 * np.exp(2 * 4.0 * 0.1), E)   # saturation after it
    g, _ = growth.growth_rate(np.stack([E, E], 1), dt, window=(0.02, 0.1))
    assert abs(g - 4.0) < 1e-9


def test_noise_is_unbiased():
    rng = np.random.default_rng(5)
    dt = 1e-4
    t = np.arange(1001) * dt
    gs = []
    for _ in range(50):
        E = np.exp(2 * 3.0 * t + 0.01 * rng.standard_normal(t.size))
        gs.append(growth.growth_rate(np.stack([E, E], 1), dt, window=(0.0, 0.1))[0])
    assert abs(np.mean(gs) - 3.0) < 0.01


def test_rejects_bad_logs():
    with pytest.raises(ValueError):
        growth.growth_rate(np.ones((3, 2)), 1.0, window=(10, 20))
    with pytest.raises(ValueError):
        growth.growth_rate(np.zeros((100, 2)), 1e-3, window=(0.0, 0.1))


def test_classical_rate():
    # k = 2 pi / 0.512, sqrt(5 * 2) / 7 with a unit shear jump: 5.54
    assert abs(growth.classical_rate(0.512) - 2 * math.pi / 0.512 * math.sqrt(10) / 7) < 1e-12
    assert abs(growth.classical_rate(0.512) - 5.54) < 5e-3
    assert abs(growth.classical_rate(0.128) - 22.18) < 5e-3
    # symmetric in the densities, linear in the shear jump and the mode
    assert growth.classical_rate(1.0, 2, 5, 2.0, 3) == pytest.approx(6 * growth.classical_rate(1.0))


def test_linear_stage_found_between_transient_and_saturation():
    """A decaying, oscillating transient, then exponential growth at
    gamma = 6 from t = 0.12 to 0.3, then saturation: the stage search lands
    inside the growth and returns gamma."""
    dt = 1e-4
    t = np.arange(4001) * dt
    lnE = np.where(t < 0.12, -10.0 - 20.0 * t + 0.5 * np.sin(200 * t), 0.0)
    grow = -12.4 + 2 * 6.0 * (t - 0.12)
    lnE = np.where((t >= 0.12) & (t <= 0.3), grow, lnE)
    lnE = np.where(t > 0.3, -12.4 + 2 * 6.0 * 0.18, lnE)
    E = np.exp(lnE)
    g, r2, a = growth.linear_stage(np.stack([E, E], 1), dt, width=0.1)
    assert abs(g - 6.0) < 1e-9 and r2 > 1 - 1e-12 and 0.12 - 1e-9 <= a <= 0.2 + 1e-9


def test_linear_stage_reports_no_growth():
    dt = 1e-4
    t = np.arange(3001) * dt
    E = np.exp(-3.0 * t)
    g, r2, a = growth.linear_stage(np.stack([E, E], 1), dt)
    assert math.isnan(g) and r2 == 0.0 and math.isnan(a)
