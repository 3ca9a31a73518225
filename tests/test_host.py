"""Host-side logic, no GPU: the tuner's tie rule, the benchmark's hash-guarded
traffic figure, the seeded input recipes and the stabilisation loop (on a
problem with a known minimum)."""
import math

import numpy as np
import pytest

import bench
from paper_1010_4124_amd import inputs, stabilize, tune


# --- tuner ---------------------------------------------------------------------
def test_tie_rule_picks_lowest_index_within_band():
    # 3 is fastest; 5 is within 1.5% of it and 0 is not: 3 wins
    assert tune._pick({0: 1.02, 3: 1.0, 5: 1.005, 7: 1.2}) == 3
    # 2 is within the band of 4: the lower index wins
    assert tune._pick({4: 1.0, 2: 1.01}) == 2
    # (variant, slots) pairs order lexicographically
    assert tune._pick({(1, 0): 1.0, (0, 64): 1.01, (0, 0): 1.2}) == (0, 64)
    assert tune.TIE == pytest.approx(0.015)


def test_median_of_trials_discards_one_low_outlier():
    # variant 1's middle trial read low (a stall in its shorter call): the
    # median keeps 0 the fastest where the minimum would pick 1
    runs = {0: [1.0, 1.01, 1.02], 1: [1.3, 0.6, 1.31]}
    ms = tune._central(runs)
    assert ms == {0: 1.01, 1: 1.3} and tune._pick(ms) == 0
    assert tune._pick({k: min(v) for k, v in runs.items()}) == 1


# --- benchmark traffic figure --------------------------------------------------
def _summary(tmp_path, name, sha, kernel, traffic):
    p = tmp_path / name
    p.write_text(f"kernel: {kernel}\nsource_sha1: {sha}\n"
                 f"traffic_bytes_per_launch: {traffic}\n")


def test_traffic_needs_matching_sources_and_kernel(tmp_path):
    k1 = "lbmd::k_step<4, 18, 4, 1, false, 2> + lbmd::k_state"
    k2 = "lbmd::k_step<8, 18, 3, 1, false, 2> + lbmd::k_state"
    pat = str(tmp_path / "k_step_*_counters.md")
    assert bench.read_traffic(k1, pat) is None  # no summaries
    _summary(tmp_path, "k_step_a_counters.md", bench.source_hash(), k1, "1.25e+08")
    _summary(tmp_path, "k_step_b_counters.md", bench.source_hash(), k2, "1.5e+08")
    assert bench.read_traffic(k1, pat) == 1.25e8
    assert bench.read_traffic(k2, pat) == 1.5e8
    assert bench.read_traffic("lbmd::k_step<4, 1, 3, 1, false, 0>", pat) is None
    # counters taken on other sources do not count
    _summary(tmp_path, "k_step_b_counters.md", "0123456789abcdef", k2, "1.5e+08")
    assert bench.read_traffic(k2, pat) is None


def test_source_hash_covers_the_kernel_sources():
    import os
    h = bench.source_hash()
    assert isinstance(h, str) and len(h) >= 16 and h == bench.source_hash()
    # every file the step kernels' translation unit includes is covered
    csrc = os.path.join(bench.ROOT, "paper_1010_4124_amd", "csrc")
    names = {os.path.basename(p) for p in bench.STEP_SOURCES}
    with open(os.path.join(csrc, "lbm_forward.hip")) as fh:
        todo = [ln.split('"')[1] for ln in fh if ln.startswith('#include "')]
    seen = set()
    while todo:
        f = todo.pop()
        if f in seen:
            continue
        seen.add(f)
        assert f in names, f
        p = os.path.join(csrc, f) if f != "lbm.h" else os.path.join(bench.ROOT, "include", f)
        with open(p) as fh:
            todo += [ln.split('"')[1] for ln in fh if ln.startswith('#include "')]


# --- inputs --------------------------------------------------------------------
def test_batch_draw_is_seeded_and_in_range():
    a, b = inputs.batch_draw(2024, n=64), inputs.batch_draw(2024, n=64)
    assert a == b and len(a) == 64
    assert inputs.batch_draw(2025, n=64) != a
    for d in a:
        assert d["nx"] in (128, 192, 256, 384, 512) and d["ny"] in (128, 192, 256, 384, 512)
        assert 0.005 <= d["Dv"] <= 0.08 and 0.005 <= d["Drho"] <= 0.08
    # both widths log-uniform: their logs spread over most of the range
    lv = np.log([d["Dv"] for d in a])
    assert lv.max() - lv.min() > 0.7 * (math.log(0.08) - math.log(0.005))


def test_shear_layer_fields():
    s = inputs.khi(64, 48, Dv=0.01, Drho=0.02)
    r, ux, uy, T = s.fields()
    assert r.shape == ux.shape == uy.shape == T.shape == (48, 64)
    # mirror symmetry about y = 0 of the cell centres (to rounding of the
    # centres): ux odd, rho + mirror = rho1 + rho2
    assert np.allclose(ux[::-1], -ux, rtol=0, atol=1e-13)
    assert np.allclose(r + r[::-1], 7.0, rtol=0, atol=1e-14)
    assert np.allclose(r * T, 2.5, rtol=1e-15, atol=0)  # uniform pressure
    assert s.bc == (inputs.PERIODIC, inputs.PERIODIC, inputs.REFLECT, inputs.REFLECT)
    assert abs(uy).max() <= 1e-3 + 1e-18


def test_paper_shear_layer_fields():
    s = inputs.khi_paper(60, 20)
    r, ux, uy, T = s.fields()
    # interface normal to x: the flow along y is odd in x, the perturbation even
    assert np.allclose(uy + uy[:, ::-1], 0.0, rtol=0, atol=1e-13)
    assert np.allclose(ux, ux[:, ::-1], rtol=0, atol=1e-15)
    assert np.allclose(r + r[:, ::-1], 7.0, rtol=0, atol=1e-14)
    assert s.bc[:2] == (inputs.OUTFLOW, inputs.OUTFLOW) and s.ke_axis == 1


def test_sod_states():
    s = inputs.sod()
    r, ux, uy, T = s.fields()
    x = (np.arange(s.nx) + 0.5) * s.dx
    left = x <= 0.5
    assert np.all(r[:, left] == 1.0) and np.all(r[:, ~left] == 0.125)
    assert np.allclose((r * T)[:, left], 1.0) and np.allclose((r * T)[:, ~left], 0.1)
    assert not ux.any() and not uy.any()


def test_mode_basis_is_orthogonal():
    A, labels = inputs.mode_basis(32, 1e-3)
    G = A @ A.T
    assert np.allclose(G - np.diag(np.diag(G)), 0.0, atol=1e-12)
    assert G[0, 0] == pytest.approx(32) and np.allclose(np.diag(G)[1:-1], 16)
    assert labels[0] == ("cos", 0) and labels[-1] == ("sin", 16)


# --- stabilisation loop ---------------------------------------------------------
class _Bowl:
    """J = 1 + (ln Dv - ln 0.04)^2 + 2 (ln Drho - ln 0.03)^2: minimum at
    (0.04, 0.03), inside the default bounds."""

    def run(self, Dv, Drho, amps, keep_checkpoints=True):
        return 1.0 + (math.log(Dv / 0.04)) ** 2 + 2.0 * (math.log(Drho / 0.03)) ** 2, None

    def gradient(self, Dv, Drho, amps, ck=None):
        return (2.0 * math.log(Dv / 0.04) / Dv, 4.0 * math.log(Drho / 0.03) / Drho, None)


def test_stabilize_descends_monotonically_within_bounds():
    hist = stabilize.stabilize(_Bowl(), 0.01, 0.01, np.zeros(4), iters=12)
    J = [h["J"] for h in hist]
    assert all(b <= a for a, b in zip(J, J[1:]))
    for h in hist:
        assert 0.005 <= h["Dv"] <= 0.08 and 0.005 <= h["Drho"] <= 0.08
    assert J[-1] < 1.0 + 1e-3 * (J[0] - 1.0)
    assert hist[-1]["Dv"] == pytest.approx(0.04, rel=0.05)
    assert hist[-1]["Drho"] == pytest.approx(0.03, rel=0.05)


def test_stabilize_stops_at_a_bound():
    class Edge(_Bowl):
        # minimum beyond the upper bound in Dv: the iterate must stay on it
        def run(self, Dv, Drho, amps, keep_checkpoints=True):
            return 1.0 + (math.log(Dv / 0.5)) ** 2 + (math.log(Drho / 0.03)) ** 2, None

        def gradient(self, Dv, Drho, amps, ck=None):
            return (2.0 * math.log(Dv / 0.5) / Dv, 2.0 * math.log(Drho / 0.03) / Drho, None)

    hist = stabilize.stabilize(Edge(), 0.02, 0.01, np.zeros(4), iters=10)
    assert hist[-1]["Dv"] == pytest.approx(0.08)
    assert all(b["J"] <= a["J"] for a, b in zip(hist, hist[1:]))


def test_trace_table_groups_by_kernel_and_grid(tmp_path, capsys):
    cols = ("Kind,Kernel_Name,Start_Timestamp,End_Timestamp,Grid_Size_X\n")
    rows = ["KERNEL_DISPATCH,\"void lbmd::k_adjoint<4, 18, 1, true>(lbmd::AdjArgs)\",100,1100,2048",
            "KERNEL_DISPATCH,\"void lbmd::k_adjoint<4, 18, 1, true>(lbmd::AdjArgs)\",200,3200,2048",
            "KERNEL_DISPATCH,\"lbmd::k_adjoint<4, 18, 1, true>(lbmd::AdjArgs)\",0,8000,65536",
            "KERNEL_DISPATCH,\"lbmd::k_init(double const*)\",0,500,256"]
    d = tmp_path / "tr"
    d.mkdir()
    (d / "x_kernel_trace.csv").write_text(cols + "\n".join(rows) + "\n")
    bench.trace_table(str(d), ["k_adjoint"])
    out = capsys.readouterr().out.splitlines()
    assert len(out) == 4 and "k_init" not in "".join(out)
    assert out[2] == "| `lbmd::k_adjoint<4, 18, 1, true>` | 2048 | 2 | 2.00 | 2.00 |"
    assert out[3] == "| `lbmd::k_adjoint<4, 18, 1, true>` | 65536 | 1 | 8.00 | 8.00 |"


def test_batch_summary_from_trace_and_log(tmp_path, capsys):
    d = tmp_path / "tr"
    d.mkdir()
    k = '"lbmd::k_step_batch<4, 1, 2, 2, true, 1>(lbmd::BatchArgs)"'
    rows = [f"KERNEL_DISPATCH,{k},0,530000,1329152", f"KERNEL_DISPATCH,{k},0,534000,1329152",
            'KERNEL_DISPATCH,"lbmd::k_reduce_batch(double const*)",0,5000,16384']
    (d / "t_kernel_trace.csv").write_text("Kind,Kernel_Name,Start_Timestamp,End_Timestamp,"
                                          "Grid_Size_X\n" + "\n".join(rows) + "\n")
    log = tmp_path / "run.log"
    log.write_text('W noise\n{"batch": {"instances": 64, "cells": 5316608, "steps": 2000, '
                   '"MLUPS": 9900.0, "variant": [4, 1, 2, 2, 1, 1], "graph_chunk": 100}}\n')
    bench.summarize_batch(str(d), str(log), ["cmd"])
    out = capsys.readouterr().out
    # 532 us per step kernel; one 5 us reduction over the two steps: 2.5 per step
    assert "532.0 us for the step kernel and 2.50 us" in out
    assert "534.5 us in all, i.e. 9947 MLUPS" in out and "gave 9900 MLUPS" in out
    assert out.rstrip().endswith("    cmd")


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, bench.__file__, "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU only" in r.stderr and r.stdout == ""
