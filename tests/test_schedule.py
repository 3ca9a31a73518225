"""Host logic of the checkpoint schedules (no GPU)."""
import pytest

objective = pytest.importorskip("paper_1010_4124_amd.objective")


def test_sqrt_schedule_bounds_memory():
    for N in (100, 4000, 40000):
        s = objective.Schedule.sqrt(N)
        assert 1 <= s.K2 <= s.K1 and s.K1 % s.K2 == 0
        assert s.peak_states(N) <= 4 * round(N ** (1 / 3)) + 8


def test_every_schedule():
    s = objective.Schedule.every(200)
    assert (s.K1, s.K2) == (200, 200)
    assert s.peak_states(4000) == 20 + 1 + 200 + 2
