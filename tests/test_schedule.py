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


def test_reverse_units_cover_every_step_once_last_first():
    """The overlapped gradient's work units: every step 0..N-1 reversed exactly
    once, last first, each piece inside its level-1 segment and at most K2 long."""
    KHIProblem, Schedule = objective.KHIProblem, objective.Schedule

    class P:
        pass

    for N, sch in ((60, Schedule(30, 6)), (70, Schedule(30, 6)), (45, Schedule(16, 5)),
                   (4000, Schedule.every(200)), (200, Schedule.sqrt(200)), (1, Schedule(1, 1))):
        p = P()
        p.nsteps, p.schedule = N, sch
        ck = {n: None for n in range(0, N, sch.K1)}
        units = KHIProblem._units(p, ck)
        steps = [n for (_, _, s0, s1) in units for n in range(s1 - 1, s0 - 1, -1)]
        assert steps == list(range(N - 1, -1, -1)), (N, sch)
        for c0, c1, s0, s1 in units:
            assert c0 <= s0 < s1 <= c1 and s1 - s0 <= sch.K2 and (s0 - c0) % sch.K2 == 0
            assert c0 % sch.K1 == 0 and c1 == min(c0 + sch.K1, N)
