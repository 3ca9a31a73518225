"""Throughput of the D2V19 + WENO5 FDLB step on one MI355X.

A bench step is one forward-Euler time step (moments, equilibrium, WENO5
convection of all 18 moving velocities along x and y, BGK relaxation,
update) of the large shear-layer workload: 2048 x 2048 cells (about 640 MB per
19-plane state), periodic in x, reflecting walls in y, dx = dy = 1e-3,
dt = tau = 1e-5, D_v = 0.01, D_rho = 0.04. Its two states (1.28 GB) are far
larger than the 256 MB Infinity Cache, so the step streams from HBM. Inputs
are seeded synthetic fields already resident in HBM when the timed region
starts; the step variant is chosen by the autotuner before it.

Prints one JSON line. The timed run (`steps` steps after `warmup` untimed
ones) is repeated (--repeats, default 5 runs in all); `value` is the MLUPS
(million lattice-site updates per second) of the median run and `ms_per_step`
its time per step; every run is listed in `extra.forward_2048_repeats`.
`roofline` relates the step's algorithmic HBM traffic (19 FP64 values read +
19 written = 304 B per site update) to the 8 TB/s HBM3E peak over the median
run's time per step: HIP events on the stream the kernels run on bracket each
run, which holds exactly `steps` step launches (plus, for the carried-moment
variants, one moment-sums pass over the input per call, amortised over the
run). `traffic` is the measured HBM traffic per step from the committed
rocprofv3 counter summary when it was taken on the current kernel sources.
`extra` holds the other workloads: the 512 x 512 shear layer (whose two
states fit the Infinity Cache), the adjoint (reverse step alone and the full
checkpointed gradient), the 64-instance batched sweep and the paper's
transition-layer studies on its own shear layer. `cpu_baseline` is the CPU
oracle timed on a bounded sample of the main workload.

Other modes (for the rocprofv3 runs whose summaries live in profiles/):
  --pmc-run        a few steps of the main workload (with --only forward512:
                   of the 512^2 one; --only adjoint: ten 2048^2 reverse
                   steps) plus a 512 MiB device copy, for one counter pass
  --summarize ...  turn the kernel-trace and counter CSVs into the summary
  --only PART      run one of the other workloads alone (forward512, batch,
                   adjoint) and print its figures as one JSON line
  --trace-table D  per-kernel, per-grid-size durations of a rocprofv3
                   kernel trace under D, as a markdown table
  --counter-table D  the same for the counter values of one counter pass
  --summarize-adjoint / --summarize-batch  the reverse-step and batched-sweep
                   summaries from their traces, counter passes and run logs
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import re
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

BYTES_PER_LUP = 19 * 8 * 2          # forward: f^n read once, f^{n+1} written once
ADJ_BYTES_PER_LUP = 19 * 8 * 3      # adjoint: f^n and lambda^{n+1} read, lambda^n written
# adjoint given the moment sums of f^n: its 18 moving planes and the 4 sums
# read instead of all 19 planes (the rest plane enters only through the sums)
ADJ_SUMS_BYTES_PER_LUP = 18 * 8 + 4 * 8 + 19 * 8 * 2
HBM_PEAK_GBS = 8000.0
COPY_BYTES = 512 << 20              # reference copy for the counter scale factors
# counter summaries of the main workload's step, one per profiled variant
TRAFFIC_SUMMARIES = os.path.join(ROOT, "profiles", "k_step_*_khi2048_counters.md")
MAIN_N = 2048
METRIC = "MLUPS (D2V19+WENO5, FP64) fwd/adjoint/batched + % HBM roofline"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# what the profiled step kernels (k_step, k_state) are compiled from: their
# translation unit, the headers it includes and the build script's flags
STEP_SOURCES = [os.path.join(ROOT, "paper_1010_4124_amd", "csrc", f) for f in
                ("lbm_forward.hip", "lbm_device.h", "lbm_fast.h", "lbm_internal.h", "lbm_stage.h",
                 "lbm_step.h")] + [os.path.join(ROOT, "include", "lbm.h"),
                                   os.path.join(ROOT, "paper_1010_4124_amd", "build.py")]


def source_hash():
    """Hash of STEP_SOURCES: a counter summary applies only to kernels built
    from the sources it was taken on."""
    h = hashlib.sha1()
    files = sorted(STEP_SOURCES)
    for p in files:
        h.update(os.path.basename(p).encode())
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def main_setup():
    """The large shear layer: 2048^2, D_v = 0.01, D_rho = 0.04."""
    from paper_1010_4124_amd import inputs
    return inputs.khi(MAIN_N, MAIN_N, dx=1e-3, dy=1e-3, dt=1e-5, tau=1e-5, Dv=0.01, Drho=0.04)


def small_setup():
    """The single shear layer: 512^2, D_v = D_rho = 0.02."""
    from paper_1010_4124_amd import inputs
    return inputs.khi(512, 512, dx=1e-3, dy=1e-3, dt=1e-5, tau=1e-5, Dv=0.02, Drho=0.02)


def sync_time(fn):
    import torch
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    e0.record(st)
    fn()
    e1.record(st)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3, time.perf_counter() - w0


def read_traffic(kernel_name, pattern=None):
    """HBM bytes per launch from the committed counter summary of this kernel,
    or None when there is none taken on the current sources."""
    for path in sorted(glob.glob(pattern or TRAFFIC_SUMMARIES)):
        try:
            txt = open(path).read()
        except OSError:
            continue
        m_hash = re.search(r"source_sha1:\s*(\w+)", txt)
        m_kern = re.search(r"kernel:\s*(.+)", txt)
        m_traf = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", txt)
        if (m_hash and m_kern and m_traf and m_hash.group(1) == source_hash()
                and m_kern.group(1).strip() == kernel_name):
            return float(m_traf.group(1))
    return None


def step_kernel_name(variant):
    """The step's kernel(s): a state-pass variant (M = 2) launches k_state and
    then the step kernel each step; both count as the step. The fast-tile
    variants (M = 3) launch k_step_fast<R, W, D, NT>."""
    from paper_1010_4124_amd import lbm
    R, G, W, D, NT, M = lbm.lbm_step_variant_info(variant)
    nt = "true" if NT else "false"
    if M == 3:
        return f"lbmd::k_step_fast<{R}, {W}, {D}, {nt}>"
    name = f"lbmd::k_step<{R}, {G}, {W}, {D}, {nt}, {M}>"
    return name + " + lbmd::k_state" if M == 2 else name


def _is_step(name):
    return "k_step<" in name or "k_step_fast<" in name


# ---------------------------------------------------------------------------
def timed_forward(s, steps, warmup, repeats, variant=None, trial_steps=None, label=""):
    """Tune (unless `variant` is given), warm up, then time `repeats` runs of
    `steps` steps from the same initial state. Returns the context, the
    per-run times and the median run's seconds and wall time."""
    import torch
    from paper_1010_4124_amd import lbm, tune
    ctx = lbm.Context.from_setup(s)
    f0 = ctx.init(*s.fields())
    if variant is None:
        kw = {"nsteps": trial_steps} if trial_steps else {}
        t = tune.tune_context(ctx, f0, use_cache=False, **kw)
        top = sorted(t["ms"].items(), key=lambda q: q[1])[:4]
        how = "tuned; fastest ms/step " + ", ".join(
            f"{lbm.lbm_step_variant_info(int(v))}: {ms:.4f}" for v, ms in top)
    else:
        ctx.variant = variant
        how = "fixed by --variant"
    log(f"{label}: variant {ctx.variant} {lbm.lbm_step_variant_info(ctx.variant)} ({how})")
    out = ctx.empty_f()
    if warmup:
        ctx.step(f0, warmup, out=out)
    runs = [sync_time(lambda: ctx.step(f0, steps, out=out)) for _ in range(max(1, repeats))]
    rc, counts = ctx.check(out, raise_error=False)
    if rc != lbm.LBM_OK:
        raise SystemExit(f"state check after the timed run failed: code {rc}, {counts}")
    secs = [r[0] for r in runs]
    med = statistics.median(secs)
    k = secs.index(min(secs, key=lambda v: abs(v - med)))
    rep = {"runs": len(secs), "ms_per_step": [v / steps * 1e3 for v in secs],
           "median_ms_per_step": med / steps * 1e3,
           "median_MLUPS": s.nx * s.ny * steps / med / 1e6,
           "variant": list(lbm.lbm_step_variant_info(ctx.variant))}
    log(f"{label}: {rep}")
    return ctx, f0, rep, med, runs[k][1]


def bench_forward_main(args):
    s = main_setup()
    ctx, f0, rep, secs, wall = timed_forward(s, args.steps, args.warmup, args.repeats,
                                             args.variant, trial_steps=30,
                                             label=f"forward {s.nx}^2")
    return s, ctx, f0, secs, wall, secs / args.steps, rep


def bench_forward_small(args):
    s = small_setup()
    ctx, f0, rep, secs, _ = timed_forward(s, args.small_steps, 200, args.repeats,
                                          label=f"forward {s.nx}^2")
    rep["steps"] = args.small_steps
    rep["hbm_frac"] = BYTES_PER_LUP * s.nx * s.ny * args.small_steps / secs / 1e9 / HBM_PEAK_GBS
    rep["kernel"] = step_kernel_name(ctx.variant)
    del ctx, f0
    return rep


def _variants(ctx):
    from paper_1010_4124_amd import lbm
    return {"step": list(lbm.lbm_step_variant_info(ctx.variant)),
            "reverse": list(lbm.lbm_adjoint_variant_info(ctx.adj_variant))}


def tune_problem(prob):
    """Tune the forward and reverse step variants of a gradient problem on
    its own initial state (outside any timed region)."""
    import torch
    from paper_1010_4124_amd import inputs, tune
    s = prob.fields(0.02, 0.02, inputs.mode_amplitudes(prob.nx, seed=7))
    f0 = prob.ctx.init(*s.fields())
    tune.tune_context(prob.ctx, f0, use_cache=False)
    lam = torch.randn_like(f0)
    tune.tune_adjoint(prob.ctx, f0, lam, use_cache=False)
    del f0, lam


def bench_adjoint(args):
    import numpy as np
    import torch
    from paper_1010_4124_amd import inputs, lbm, objective, tune
    res = {}
    # reverse step alone at 256^2 and 2048^2
    for n, steps in ((256, 200), (2048, 20)):
        s = inputs.khi(n, n, Dv=0.02, Drho=0.02)
        ctx = lbm.Context.from_setup(s)
        f0 = ctx.init(*s.fields())
        lam = [torch.zeros_like(f0), ctx.empty_f()]
        tune.tune_adjoint(ctx, f0, torch.randn_like(f0), use_cache=False)

        def run():
            for q in range(steps):
                ctx.adjoint_step(f0, lam[q % 2], 1e-5, out=lam[(q + 1) % 2])
        run()
        secs, _ = sync_time(run)
        mlups = n * n * steps / secs / 1e6
        log(f"adjoint: reverse step {n}^2: {mlups:.0f} MLUPS")
        res[f"reverse_step_{n}"] = {"MLUPS": mlups,
                                    "variant": list(lbm.lbm_adjoint_variant_info(ctx.adj_variant)),
                                    "hbm_frac": mlups * 1e6 * ADJ_BYTES_PER_LUP / 1e9 / HBM_PEAK_GBS}
        # the same given the moment sums of f^n (lbm_adjoint_step_sums), as
        # the checkpointed gradient runs it with a fast-tile forward variant
        sums = ctx.sums(f0)

        def run_sums():
            for q in range(steps):
                ctx.adjoint_step(f0, lam[q % 2], 1e-5, out=lam[(q + 1) % 2], sums=sums)
        run_sums()
        secs, _ = sync_time(run_sums)
        mlups = n * n * steps / secs / 1e6
        res[f"reverse_step_{n}_sums"] = {
            "MLUPS": mlups, "variant": list(lbm.lbm_adjoint_variant_info(ctx.adj_variant)),
            "bytes_per_lup": ADJ_SUMS_BYTES_PER_LUP,
            "hbm_frac": mlups * 1e6 * ADJ_SUMS_BYTES_PER_LUP / 1e9 / HBM_PEAK_GBS}
        del ctx, f0, lam, sums
        torch.cuda.empty_cache()
    # full checkpointed gradient, 256^2 shear layer, 4000 steps, checkpoints every 200
    rng_amps = inputs.mode_amplitudes(256, seed=7)
    prob = objective.KHIProblem(256, 256, nsteps=args.adj_steps,
                                window=(args.adj_steps // 2, args.adj_steps),
                                schedule=objective.Schedule.every(200))
    tune_problem(prob)
    fwd_secs, _ = sync_time(lambda: prob.run(0.02, 0.02, rng_amps))
    J, ck = prob.run(0.02, 0.02, rng_amps)
    grad_secs, _ = sync_time(lambda: prob.gradient(0.02, 0.02, rng_amps, ck=ck))
    lups = 256 * 256 * args.adj_steps
    log(f"adjoint: gradient 256^2 done ({grad_secs:.1f} s)")
    res["gradient_256"] = {"steps": args.adj_steps, "checkpoint_every": 200,
                           "forward_MLUPS": lups / fwd_secs / 1e6,
                           "adjoint_MLUPS": lups / grad_secs / 1e6,
                           "variants": _variants(prob.ctx),
                           "note": "adjoint = recompute + reverse, per forward step"}
    # 2048^2, sqrt-N two-level schedule over a bounded number of steps
    n2 = args.adj_large_steps
    prob2 = objective.KHIProblem(2048, 2048, nsteps=n2, window=(n2 // 2, n2),
                                 schedule=objective.Schedule.sqrt(n2))
    tune_problem(prob2)
    log(f"adjoint: 2048^2, {n2} steps, schedule {prob2.schedule.K1} x {prob2.schedule.K2}: tuned")
    amps2 = inputs.mode_amplitudes(2048, seed=7)
    fsecs, _ = sync_time(lambda: prob2.run(0.01, 0.04, amps2, keep_checkpoints=False))
    log(f"adjoint: 2048^2 forward run {fsecs:.1f} s")
    torch.cuda.reset_peak_memory_stats()
    J2, ck2 = prob2.run(0.01, 0.04, amps2)
    log("adjoint: 2048^2 forward run with checkpoints done")
    grad2 = []
    gsecs, _ = sync_time(lambda: grad2.append(prob2.gradient(0.01, 0.04, amps2, ck=ck2)))
    gDv2, gDrho2, ga2 = grad2[0]
    l2 = 2048 * 2048 * n2
    res["gradient_2048"] = {"steps": n2, "schedule": [prob2.schedule.K1, prob2.schedule.K2],
                            "forward_MLUPS": l2 / fsecs / 1e6, "adjoint_MLUPS": l2 / gsecs / 1e6,
                            "peak_device_GB": torch.cuda.max_memory_allocated() / 1e9,
                            "finite": bool(np.isfinite([J2, gDv2, gDrho2]).all()
                                           and np.isfinite(ga2).all()),
                            "J": J2, "dJ_dDv": gDv2, "dJ_dDrho": gDrho2,
                            "variants": _variants(prob2.ctx),
                            "note": ("configuration 5 at full length" if n2 >= 40000 else
                                     f"a {n2}-step sample of configuration 5 (40000 steps: "
                                     "--only adjoint --adj-large-steps 40000)")}
    log(f"adjoint: {res}")
    del prob, prob2, ck, ck2
    torch.cuda.empty_cache()
    return res


def bench_batch(args):
    import numpy as np
    import torch
    from paper_1010_4124_amd import growth, inputs, lbm, tune
    draw = inputs.batch_draw(2024, n=64)
    setups = [inputs.khi(d["nx"], d["ny"], Dv=d["Dv"], Drho=d["Drho"]) for d in draw]
    b = lbm.Batch.from_setups(setups)
    fields = [s.fields() for s in setups]
    f0 = b.init(*[b.pack_scalars([f[q] for f in fields]) for q in range(4)])
    if args.batch_variant is None:
        tune.tune_batch(b, f0, slots=(0, 384), use_cache=False)
        b.schedule = (b.schedule[0], 100)
    else:
        b.variant = args.batch_variant
        b.schedule = (0, 100)
    out = b.empty_f()
    ke = torch.empty((b.n, args.batch_steps, 2), dtype=torch.float64, device=out.device)
    lbm.lbm_batch_step(b.handle, f0, out, 100, ke[:, :100].contiguous())  # warm: capture graph
    secs, _ = sync_time(lambda: lbm.lbm_batch_step(b.handle, f0, out, args.batch_steps, ke))
    kel = ke.cpu().numpy()
    # growth rates over the linear stage each log shows within the configured
    # run (t <= 0.1, so 0.05-long stages); instances still in the initial
    # transient have no straight rising stage (r2 < 0.99) and are not counted
    gam, below = [], 0
    for i, (d, s) in enumerate(zip(draw, setups)):
        g, r2, _ = growth.linear_stage(kel[i], s.dt, width=0.05)
        if not r2 >= 0.99:
            continue
        gam.append(g)
        below += g < growth.classical_rate(d["nx"] * s.dx)
    r = {"instances": b.n, "cells": b.cells, "steps": args.batch_steps,
         "MLUPS": b.cells * args.batch_steps / secs / 1e6,
         "variant": list(lbm.lbm_step_variant_info(b.variant)), "slots_per_xcd": b.schedule[0],
         "graph_chunk": b.schedule[1], "ke_logged": True,
         "gamma": {"fit": "linear stage of the domain-integral log, 0.05 long, r2 >= 0.99",
                   "fitted": len(gam), "median": float(np.median(gam)) if gam else None,
                   "min": float(np.min(gam)) if gam else None,
                   "max": float(np.max(gam)) if gam else None, "below_classical": int(below)}}
    log(f"batched sweep: {r}")
    return r


def bench_paper_studies():
    """The paper's own shear layer (outflow sides) as batched studies of the
    velocity- and density-layer widths: growth rates, fits, throughput."""
    from paper_1010_4124_amd import sweeps
    v = sweeps.velocity_study()
    d = sweeps.density_study()
    r = {"velocity_layer": {k: v[k] for k in ("widths", "gamma", "a", "b", "mlups", "steps")},
         "density_layer": {k: d[k] for k in ("widths", "gamma", "c", "e", "mlups", "steps")},
         "note": "widths in grid spacings; gamma from ln E_x|max over t in [0.1, 0.3]"}
    log(f"paper studies: {r}")
    return r


def cpu_baseline(setup, seconds):
    """The oracle as it stands on the GPU run's host: the first steps of the
    main workload from its initial state, on up to 16 threads (OpenMP over
    rows) and on one thread, each within a time budget."""
    import oracle
    p = oracle.OracleParams.make(setup.nx, setup.ny, setup.dx, setup.dy, setup.dt, setup.tau,
                                 setup.bc)
    f0 = oracle.init(p, *setup.fields())
    threads = min(16, os.cpu_count() or 1)

    def timed(nthreads, budget):
        f, steps, chunk = f0, 0, 1
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < budget and steps < 5000:
            f = oracle.step(p, f, chunk, nthreads=nthreads)
            steps += chunk
        return steps, time.perf_counter() - t0

    steps, dt = timed(threads, seconds)
    steps1, dt1 = timed(1, seconds / 3)
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")),
                         "")
    except OSError:
        pass
    return {"value": setup.nx * setup.ny * steps / dt / 1e6, "unit": "MLUPS", "cores": threads,
            "kind": "oracle",
            "sample": f"{setup.nx}x{setup.ny} shear layer (the main workload), its first "
                      f"{steps} steps from the same initial state, {dt:.1f} s on {threads} "
                      "threads (a rate measured on this sample, not a full-length run)",
            "single_thread_MLUPS": setup.nx * setup.ny * steps1 / dt1 / 1e6,
            "single_thread_sample": f"first {steps1} steps, {dt1:.1f} s on 1 thread",
            "host_cpus": os.cpu_count(), "cpu_model": model}


def trace_table(root, match):
    """Markdown table of a rocprofv3 kernel trace: dispatches grouped by
    kernel and grid size, with their count and mean and median durations."""
    rows = _rows(os.path.join(root, "**", "*kernel_trace.csv"))
    if not rows:
        raise SystemExit(f"no kernel trace under {root}")
    by = {}
    for r in rows:
        name = re.sub(r"^void ", "", r["Kernel_Name"]).split("(")[0]
        if match and not any(m in name for m in match):
            continue
        ns = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        by.setdefault((name, int(r["Grid_Size_X"])), []).append(ns)
    lines = ["| kernel | grid (work-items) | dispatches | mean us | median us |",
             "|---|---|---|---|---|"]
    for (name, grid), v in sorted(by.items(), key=lambda q: (q[0][0], q[0][1])):
        lines.append(f"| `{name}` | {grid} | {len(v)} | {statistics.mean(v) / 1e3:.2f} | "
                     f"{statistics.median(v) / 1e3:.2f} |")
    print("\n".join(lines))


def _table_rows(text):
    """{(kernel, grid): cells} of a markdown table printed by trace_table or
    counter_table."""
    out = {}
    for ln in text.strip().splitlines()[2:]:
        c = [x.strip() for x in ln.strip("|").split("|")]
        out[(c[0].strip("`"), int(c[1]))] = c
    return out


def _capture(fn, *a):
    import contextlib
    import io
    buf = io.StringIO()
    with contextlib.redirect_stdout(buf):
        fn(*a)
    return buf.getvalue().strip()


def _bench_line(log_path, key):
    with open(log_path) as fh:
        return json.loads(next(ln for ln in fh if ln.startswith('{"%s"' % key)))[key]


def summarize_adjoint(trace, fetch, write, log_path, commands, sq_dirs=()):
    """Markdown summary of the reverse-step profile: the kernel trace of
    `bench.py --only adjoint` and FETCH_SIZE / WRITE_SIZE passes of
    `bench.py --pmc-run --only adjoint --variant V` (ten 2048^2 reverse
    steps of variant V: its state pass, band tiles and march or tile kernel,
    then ten given the moment sums of f^n), plus any further counter passes
    of the same command (sq_dirs)."""
    tab = _capture(trace_table, trace, ["k_adj"])
    ftab = _capture(counter_table, fetch, ["k_adj", "copyBuffer"])
    wtab = _capture(counter_table, write, ["k_adj", "copyBuffer"])
    fr, wr = _table_rows(ftab), _table_rows(wtab)
    n = 2048 * 2048
    sf = COPY_BYTES / (float(fr[("__amd_rocclr_copyBuffer", 131072)][4]) * 1024)
    sw = COPY_BYTES / (float(wr[("__amd_rocclr_copyBuffer", 131072)][4]) * 1024)
    per = []
    for (name, grid), row in sorted(fr.items()):
        if "k_adj" not in name:
            continue
        w = wr.get((name, grid))
        per.append((name, float(row[4]) * 1024 * sf / n,
                    float(w[4]) * 1024 * sw / n if w else 0.0))
    # the two forms share the band and march kernels; each has its own state pass
    st_f, st_s = "lbmd::k_adj_state<false>", "lbmd::k_adj_state<true>"
    shared = [p for p in per if p[0] not in (st_f, st_s)]
    forms = []
    for label, st in (("reverse step", st_f), ("reverse step given the sums", st_s)):
        pp = shared + [p for p in per if p[0] == st]
        forms.append((label, sum(p[1] for p in pp), sum(p[2] for p in pp)))
    (_, rd, wt), (_, rds, wts) = forms
    ev = _bench_line(log_path, "adjoint")
    r2048, r256 = ev["reverse_step_2048"], ev["reverse_step_256"]
    lines = [
        "# Reverse step (discrete adjoint), shear layer at 256^2 and 2048^2: durations and HBM traffic",
        "",
        "Variants (R, G, W, PS): PS = 1 runs lbmd::k_adj_state, then lbmd::k_adjoint<R, G, W, true> "
        "over 64 x R tiles; PS = 2 runs lbmd::k_adj_state, then lbmd::k_adj_march<W> over "
        "64-column strips in chunks of R rows, with the tiles next to the walls (the tile "
        "kernel's code in band mode) in the same launch. The bench's tuner picked "
        f"{tuple(r2048['variant'])} at 2048^2 ({r2048['MLUPS']:.0f} MLUPS, "
        f"{1e6 * n / (r2048['MLUPS'] * 1e6):.0f} us per reverse step) and "
        f"{tuple(r256['variant'])} at 256^2 ({r256['MLUPS']:.0f} MLUPS); given the moment sums "
        f"of f^n, {ev['reverse_step_2048_sums']['MLUPS']:.0f} MLUPS at 2048^2 "
        f"({1e6 * n / (ev['reverse_step_2048_sums']['MLUPS'] * 1e6):.0f} us).",
        "",
        "## Kernel trace (every variant the tuner tries, both sizes, and the gradients' steps)",
        "",
        "Medians: the traced command also runs the checkpointed gradients, whose reverse steps "
        "overlap the recompute on a second stream on the 256^2 grid (not at 2048^2, a grid that "
        "fills the GPU by itself).",
        "", tab, "",
        "## Counter passes, 2048^2, ten reverse steps of the profiled variant, then ten given "
        "the moment sums of f^n",
        "", "FETCH_SIZE (KiB per dispatch):", "", ftab, "",
        "WRITE_SIZE (KiB per dispatch):", "", wtab, "",
        f"Scale factors from the 512 MiB copy in the same runs: FETCH {sf:.4f}, WRITE {sw:.4f}.",
        "",
        "| kernel | read B/cell | written B/cell |",
        "|---|---|---|",
    ] + [f"| `{nm}` | {r:.0f} | {w:.0f} |" for nm, r, w in per] + [
        f"| {lab} | {r:.0f} | {w:.0f} |" for lab, r, w in forms] + [
        "",
        f"Total {rd + wt:.0f} B per cell against the algorithmic 456 (f^n and lambda^(n+1) read "
        "once, lambda^n written once). The excess is the two-pass structure: the state pass "
        "reads f^n and lambda^(n+1) in full (304 B) and writes the four K's and the rest "
        "plane (40 B); the velocity kernels then read the 18 moving planes of both arrays again "
        "with their halo rows and strip-edge columns, plus the K's. Given the moment sums of "
        f"f^n, the state pass reads them instead of f^n: {rds + wts:.0f} B per cell in all, against "
        "the 480 that form must move (the 18 moving planes of f^n, the 4 sums, lambda^(n+1), "
        "lambda^n).",
    ]
    if sq_dirs:
        lines += ["", "## Further counter passes, 2048^2, the same ten reverse steps", ""]
        vals = {}
        for d in sq_dirs:
            lines += [_capture(counter_table, d, ["k_adj"]), ""]
            for r in _rows(os.path.join(d, "**", "*counter_collection.csv")):
                if "k_adj" in _kname(r):
                    vals.setdefault((_kname(r), int(r["Grid_Size"]), r["Counter_Name"]),
                                    []).append(float(r["Counter_Value"]))
        trows = _table_rows(tab)
        for nm, grid in sorted({(k[0], k[1]) for k in vals}):
            def get(c):
                v = vals.get((nm, grid, c))
                return statistics.mean(v) if v else None
            parts = []
            valu, waves, tr = get("SQ_INSTS_VALU"), get("SQ_WAVES"), trows.get((nm, grid))
            if tr is not None and valu is not None and waves:
                us = float(tr[4])
                issue = valu * 4 / 1024 / 2.4e3
                parts += [f"{valu / waves:.0f} VALU instructions per wave",
                          f"VALU issue {issue:.0f} us per SIMD against the traced median "
                          f"{us:.0f} us ({issue / us:.0%}; 4 cycles per wave64 instruction, "
                          "1024 SIMDs, 2.4 GHz)"]
            if get("SQ_WAIT_INST_ANY") and get("SQ_WAVE_CYCLES"):
                parts.append(f"waiting on a dependency "
                             f"{get('SQ_WAIT_INST_ANY') / get('SQ_WAVE_CYCLES'):.0%} of wave time")
            if get("SQ_LDS_BANK_CONFLICT") is not None and get("SQ_ACTIVE_INST_LDS"):
                parts.append(f"LDS bank conflicts "
                             f"{get('SQ_LDS_BANK_CONFLICT') / get('SQ_ACTIVE_INST_LDS'):.0%} of "
                             "LDS-active cycles")
            if get("TCC_HIT_sum") is not None and get("TCC_MISS_sum"):
                h, m = get("TCC_HIT_sum"), get("TCC_MISS_sum")
                parts.append(f"L2 hits {h / (h + m):.0%} of requests")
            if parts:
                lines.append(f"- `{nm}` ({grid} work-items): " + "; ".join(parts) + ".")
    lines += ["", "Commands (repository root, TMPDIR=/tmp):"] + ["    " + c for c in commands]
    print("\n".join(lines))


def summarize_batch(trace, log_path, commands):
    """Markdown summary of the batched sweep's kernel trace
    (`bench.py --only batch --batch-variant V`)."""
    tab = _capture(trace_table, trace, ["k_step_batch", "k_reduce_batch"])
    rows = _table_rows(tab)
    ev = _bench_line(log_path, "batch")
    v = ev["variant"]
    name = (f"lbmd::k_step_batch<{v[0]}, {v[1]}, {v[2]}, {v[3]}, "
            f"{'true' if v[4] else 'false'}, {v[5]}>")
    step_key = max((k for k in rows if k[0] == name), key=lambda k: int(rows[k][2]))
    red_key = next(k for k in rows if k[0] == "lbmd::k_reduce_batch")
    stp = float(rows[step_key][3])
    # one reduction launch covers the energy logs of up to 32 steps of a graph
    red = float(rows[red_key][3]) * int(rows[red_key][2]) / int(rows[step_key][2])
    cells = ev["cells"]
    lines = [
        f"# Batched step, 64-instance shear-layer sweep ({cells} cells): kernel durations",
        "",
        "The sweep's instances (seed 2024) have sizes drawn from {128, 192, 256, 384, 512}^2; one "
        "launch of lbmd::k_step_batch advances all of them by one step, and "
        "lbmd::k_reduce_batch turns the per-tile partials into the 64 energy-log entries. The "
        f"step variant is fixed to {tuple(v)}, the one the bench's tuner picks for this sweep "
        "(the tuner's own short trials run perturbed under the tracer), with one workgroup per "
        f"work item ({step_key[1]} work-items).",
        "", tab, "",
        f"Per step: {stp:.1f} us for the step kernel and {red:.2f} us for the energy "
        f"reductions ({rows[red_key][2]} launches over {rows[step_key][2]} steps), "
        f"{stp + red:.1f} us in all, i.e. {cells / (stp + red):.0f} "
        f"MLUPS; the bench's events in the same run ({ev['steps']} steps, graph chunks of "
        f"{ev['graph_chunk']}) gave {ev['MLUPS']:.0f} MLUPS.",
        "",
        "Command (repository root, TMPDIR=/tmp):",
    ] + ["    " + c for c in commands]
    print("\n".join(lines))


def counter_table(root, match):
    """Markdown table of one rocprofv3 counter pass: the mean value per
    dispatch of each counter, grouped by kernel and grid size (FETCH_SIZE
    and WRITE_SIZE in KiB)."""
    rows = _rows(os.path.join(root, "**", "*counter_collection.csv"))
    if not rows:
        raise SystemExit(f"no counter collection under {root}")
    by = {}
    for r in rows:
        name = re.sub(r"^void ", "", r["Kernel_Name"]).split("(")[0]
        if match and not any(m in name for m in match):
            continue
        key = (name, int(r["Grid_Size"]), r["Counter_Name"])
        by.setdefault(key, []).append(float(r["Counter_Value"]))
    lines = ["| kernel | grid (work-items) | counter | dispatches | mean per dispatch |",
             "|---|---|---|---|---|"]
    for (name, grid, ctr), v in sorted(by.items()):
        lines.append(f"| `{name}` | {grid} | {ctr} | {len(v)} | {statistics.mean(v):.1f} |")
    print("\n".join(lines))


# ---------------------------------------------------------------------------
def pmc_run(args):
    """A short run for one rocprofv3 counter pass: the tuned main step (with
    --only adjoint: ten 2048^2 reverse steps of variant --variant, else of
    the context's default) and a plain device copy of COPY_BYTES."""
    import torch
    from paper_1010_4124_amd import inputs, lbm, tune
    if args.only == "adjoint":
        s = inputs.khi(2048, 2048, Dv=0.01, Drho=0.04)
        ctx = lbm.Context.from_setup(s)
        f0 = ctx.init(*s.fields())
        if args.variant is not None:
            ctx.adj_variant = args.variant
        log(f"pmc run: reverse step variant {ctx.adj_variant} "
            f"{lbm.lbm_adjoint_variant_info(ctx.adj_variant)}")
        lam = [torch.randn_like(f0), ctx.empty_f()]
        for q in range(10):
            ctx.adjoint_step(f0, lam[q % 2], 1e-5, out=lam[(q + 1) % 2])
        # then ten given the moment sums of f^n (lbm_adjoint_step_sums)
        sums = ctx.sums(f0)
        for q in range(10):
            ctx.adjoint_step(f0, lam[q % 2], 1e-5, out=lam[(q + 1) % 2], sums=sums)
        del ctx, f0, lam, sums
        torch.cuda.empty_cache()
    else:
        _pmc_main(args, small_setup() if args.only == "forward512" else main_setup())
    x = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()


def _pmc_main(args, s):
    from paper_1010_4124_amd import lbm, tune
    ctx = lbm.Context.from_setup(s)
    f0 = ctx.init(*s.fields())
    if args.variant is None:
        tune.tune_context(ctx, f0, nsteps=30, use_cache=False)
    else:
        ctx.variant = args.variant
    log(f"pmc run: variant {ctx.variant} {lbm.lbm_step_variant_info(ctx.variant)}")
    out = ctx.empty_f()
    if args.warmup:
        ctx.step(f0, args.warmup, out=out)  # as in the benchmark: a warm GPU
    ctx.step(f0, args.steps, out=out)


def _rows(pattern):
    import csv
    rows = []
    for p in glob.glob(pattern, recursive=True):
        with open(p) as fh:
            rows.extend(csv.DictReader(fh))
    return rows


def _kname(r, key="Kernel_Name"):
    return re.sub(r"^void ", "", r[key]).split("(")[0]


def _last(rows, n):
    """The last n rows in dispatch order (the timed call of a --pmc-run)."""
    rows = sorted(rows, key=lambda r: int(r.get("Dispatch_Id", r.get("Correlation_Id", 0))))
    return rows[-n:]


def summarize(args):
    """Markdown summary of the kernel trace and the two counter passes of a
    --pmc-run: durations and counters of the step kernel(s) over the last
    --last dispatches (the timed call; the warm-up call comes first)."""
    trace, fetch, write = args.summarize
    n_last = args.last
    stats = _rows(os.path.join(trace, "**", "*kernel_stats.csv"))
    kt = _rows(os.path.join(trace, "**", "*kernel_trace.csv"))
    step = [r for r in stats if _is_step(r["Name"])]
    if not step:
        raise SystemExit(f"no step kernel in {trace}")
    # the tuner launches every variant a few times; the timed one dominates
    top = max(step, key=lambda r: int(r["Calls"]))
    base = re.sub(r"^void ", "", top["Name"]).split("(")[0]

    def durations(kernel):
        rows = _last([r for r in kt if _kname(r) == kernel], n_last)
        return [int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in rows]

    dur = durations(base)
    parts = [base]
    if base.endswith(", 2>"):
        sd = durations("lbmd::k_state")
        if not sd:
            raise SystemExit("state-pass variant without k_state in the trace")
        dur = [a + b for a, b in zip(dur, sd)]
        parts.append("lbmd::k_state")
    avg_ns = statistics.mean(dur)
    name = " + ".join(parts)

    def per_dispatch(root, counter):
        rows = _rows(os.path.join(root, "**", "*counter_collection.csv"))
        by = {}
        for r in rows:
            if (_is_step(r["Kernel_Name"]) or r["Kernel_Name"].startswith("lbmd::k_state(")) \
                    and r["Counter_Name"] == counter:
                by.setdefault(_kname(r), []).append(r)
        by = {k: [float(r["Counter_Value"]) for r in _last(v, n_last)] for k, v in by.items()}
        cp = [(int(r["Grid_Size"]), float(r["Counter_Value"])) for r in rows
              if "copyBuffer" in r["Kernel_Name"] and r["Counter_Name"] == counter]
        steps = {k: v for k, v in by.items() if _is_step(k)}
        if not steps or not cp:
            raise SystemExit(f"{counter}: step or copy dispatches missing in {root}")
        k = max(steps, key=lambda q: len(steps[q]))
        if k != base:
            raise SystemExit(f"{counter}: counted {k}, traced {base}")
        total = statistics.mean(by[k])
        if len(parts) > 1:
            total += statistics.mean(by["lbmd::k_state"])
        return total, max(cp)[1]

    sums = [r for r in stats if r["Name"].startswith("lbmd::k_sums(")]
    f_k, f_c = per_dispatch(fetch, "FETCH_SIZE")
    w_k, w_c = per_dispatch(write, "WRITE_SIZE")
    sf, sw = COPY_BYTES / (f_c * 1024.0), COPY_BYTES / (w_c * 1024.0)
    traffic = f_k * 1024.0 * sf + w_k * 1024.0 * sw
    cells = args.n * args.n
    algo = BYTES_PER_LUP * cells
    lines = [
        f"# Step kernel(s), {args.n} x {args.n} shear layer: duration and HBM traffic per step",
        "",
        f"kernel: {name}",
        f"source_sha1: {source_hash()}",
        f"avg_duration_ns: {avg_ns:.1f} (per step, all of its kernels, mean of the last "
        f"{len(dur)} dispatches: the timed call)",
        f"median_duration_ns: {statistics.median(dur):.1f}",
        f"calls: {top['Calls']} (warm-up and timed calls)",
        f"fetch_kib_per_dispatch: {f_k:.1f}",
        f"write_kib_per_dispatch: {w_k:.1f}",
        f"copy_fetch_kib: {f_c:.1f} (512 MiB copy; scale {sf:.4f})",
        f"copy_write_kib: {w_c:.1f} (512 MiB copy; scale {sw:.4f})",
        f"traffic_bytes_per_launch: {traffic:.6e}",
        f"algorithmic_bytes_per_launch: {algo:.6e} (304 B x {cells} cells)",
        f"traffic_per_lup: {traffic / cells:.1f} B (algorithmic 304 B)",
        f"achieved_algorithmic_GBs: {algo / avg_ns:.1f}",
        f"achieved_measured_GBs: {traffic / avg_ns:.1f}",
    ]
    if sums:
        lines.append(f"moment_sums_pass_ns: {float(sums[0]['AverageNs']):.1f} (k_sums, once per "
                     f"lbm_step call of a carried-moment variant; {sums[0]['Calls']} calls)")
    for d in args.sq or []:
        rows = _rows(os.path.join(d, "**", "*counter_collection.csv"))
        byc = {}
        for r in rows:
            if _kname(r) == base:
                byc.setdefault(r["Counter_Name"], []).append(r)
        by = {c: [float(r["Counter_Value"]) for r in _last(v, n_last)] for c, v in byc.items()}
        if not by:
            raise SystemExit(f"no {base} dispatches in {d}")
        lines += ["", f"SQ counters ({d.rstrip('/').split('/')[-1]}), mean per dispatch of {base}:", ""]
        lines += [f"    {c}: {statistics.mean(v):.1f}" for c, v in sorted(by.items())]
        if "SQ_INSTS_VALU" in by and "SQ_WAVES" in by:
            valu = statistics.mean(by["SQ_INSTS_VALU"])
            lines.append(f"    VALU instructions per wave: {valu / statistics.mean(by['SQ_WAVES']):.0f}; "
                         f"per site update (64 lanes): {valu * 64 / cells:.0f}")
            lines.append(f"    VALU issue share (4 cycles per wave64 instruction, 1024 SIMDs, "
                         f"2.4 GHz, over the traced duration): "
                         f"{valu * 4 / 1024 / (avg_ns * 2.4):.2f}")
    lines += ["", "Commands (repository root, TMPDIR=/tmp):"]
    lines += ["    " + c for c in args.commands] if args.commands else []
    print("\n".join(lines))


# ---------------------------------------------------------------------------
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--repeats", type=int, default=5,
                    help="timed runs of the main workload; the median is the reported value")
    ap.add_argument("--variant", type=int, default=None,
                    help="step variant of the main workload (default: autotuned)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--small-steps", type=int, default=2000,
                    help="timed steps per run of the 512^2 shear layer in extra")
    ap.add_argument("--adj-steps", type=int, default=4000)
    ap.add_argument("--adj-large-steps", type=int, default=200)
    ap.add_argument("--batch-steps", type=int, default=10000)
    ap.add_argument("--batch-variant", type=int, default=None,
                    help="step variant of the batched sweep (default: autotuned)")
    ap.add_argument("--pmc-run", action="store_true")
    ap.add_argument("--summarize", nargs=3, metavar=("TRACE", "FETCH", "WRITE"))
    ap.add_argument("--commands", nargs="*")
    ap.add_argument("--sq", nargs="*", help="SQ counter-pass directories for --summarize")
    ap.add_argument("--n", type=int, default=MAIN_N,
                    help="--summarize: the side of the profiled grid (2048, or 512 for forward512)")
    ap.add_argument("--last", type=int, default=20,
                    help="--summarize: dispatches of the timed call (its last ones)")
    ap.add_argument("--only", choices=("forward512", "batch", "adjoint"))
    ap.add_argument("--trace-table", metavar="TRACE")
    ap.add_argument("--counter-table", metavar="PMC")
    ap.add_argument("--match", nargs="*", default=[])
    ap.add_argument("--summarize-adjoint", nargs=4, metavar=("TRACE", "FETCH", "WRITE", "LOG"))
    ap.add_argument("--summarize-batch", nargs=2, metavar=("TRACE", "LOG"))
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: one GPU only; --gpus {args.gpus} is not supported. The step shards by "
              "row slabs with a 3-row halo exchange; that path is designed, not built.",
              file=sys.stderr)
        sys.exit(2)
    if args.summarize:
        summarize(args)
        return
    if args.trace_table:
        trace_table(args.trace_table, args.match)
        return
    if args.counter_table:
        counter_table(args.counter_table, args.match)
        return
    if args.summarize_adjoint:
        summarize_adjoint(*args.summarize_adjoint, args.commands or [], args.sq or [])
        return
    if args.summarize_batch:
        summarize_batch(*args.summarize_batch, args.commands or [])
        return

    import torch
    torch.cuda.set_device(0)
    if args.pmc_run:
        pmc_run(args)
        return
    if args.only:
        part = {"forward512": bench_forward_small, "batch": bench_batch,
                "adjoint": bench_adjoint}[args.only]
        print(json.dumps({args.only: part(args)}), flush=True)
        return

    s, ctx, f0, secs, wall, avg, rep = bench_forward_main(args)
    lups = s.nx * s.ny * args.steps
    mlups = lups / secs / 1e6
    kname = step_kernel_name(ctx.variant)
    algo = BYTES_PER_LUP * s.nx * s.ny
    achieved = algo / avg / 1e9
    traffic = read_traffic(kname)
    del ctx, f0
    torch.cuda.empty_cache()

    extra = {"forward_2048_repeats": rep}
    if not args.no_extra:
        extra["forward_512"] = bench_forward_small(args)
        torch.cuda.empty_cache()
        extra["batched_sweep"] = bench_batch(args)
        extra["paper_studies"] = bench_paper_studies()
        extra["adjoint"] = bench_adjoint(args)

    out = {
        "metric": METRIC,
        "value": mlups,
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": secs / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"large shear layer (KHI) {s.nx}x{s.ny}, periodic x, reflecting "
                               "walls in y, dx=dy=1e-3, dt=tau=1e-5, D_v=0.01, D_rho=0.04, "
                               "forward step (median of the timed runs)",
                   "nx": s.nx, "ny": s.ny, "steps": args.steps, "repeats": rep["runs"],
                   "wall_s": wall},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": kname, "avg_launch_us": avg * 1e6,
                     "algorithmic_bytes_per_launch": algo},
        "extra": extra,
    }
    if not args.no_cpu:
        log("cpu baseline ...")
        out["cpu_baseline"] = cpu_baseline(main_setup(), args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
