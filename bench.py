"""Throughput of the D2V19 + WENO5 FDLB step on one MI355X.

A bench step is one forward-Euler time step (moments, equilibrium, WENO5
convection of all 18 moving velocities along x and y, BGK relaxation,
update) of the single shear-layer workload: 512 x 512 cells, periodic in x,
reflecting walls in y, dx = dy = 1e-3, dt = tau = 1e-5, D_v = D_rho = 0.02,
20000 steps. Inputs are seeded synthetic fields already resident in HBM when
the timed region starts.

Prints one JSON line. `value` is MLUPS (million lattice-site updates per
second) of that run; `roofline` relates the step kernel's algorithmic HBM
traffic (19 FP64 values read + 19 written = 304 B per site update) to the
8 TB/s HBM3E peak; `cpu_baseline` is the CPU oracle timed on a bounded sample
of the same workload on this host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

BYTES_PER_LUP = 19 * 8 * 2
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def time_forward(ctx, f0, steps, warmup):
    import torch
    fa = ctx.empty_f()
    if warmup:
        ctx.step(f0, warmup, out=fa)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    ctx.step(f0, steps, out=fa)
    e1.record(st)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3, fa


def cpu_baseline(setup, nsteps):
    import oracle
    p = oracle.OracleParams.make(setup.nx, setup.ny, setup.dx, setup.dy, setup.dt, setup.tau,
                                 setup.bc)
    f0 = oracle.init(p, *setup.fields())
    threads = min(16, os.cpu_count() or 1)
    t = time.perf_counter()
    oracle.step(p, f0, nsteps, nthreads=threads)
    dt = time.perf_counter() - t
    return {"value": setup.nx * setup.ny * nsteps / dt / 1e6, "unit": "MLUPS", "cores": threads,
            "kind": "oracle",
            "sample": f"{setup.nx}x{setup.ny} shear layer, {nsteps} steps from the same "
                      f"initial state ({dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--cpu-steps", type=int, default=30)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--large-steps", type=int, default=200)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only; --gpus {args.gpus} is not supported "
              "(the step is designed to shard by row slabs, see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1010_4124_amd import inputs, lbm
    torch.cuda.set_device(0)

    setup = inputs.khi(512, 512, dx=1e-3, dy=1e-3, dt=1e-5, tau=1e-5, Dv=0.02, Drho=0.02)
    ctx = lbm.Context.from_setup(setup)
    f0 = ctx.init(*setup.fields())
    log(f"forward 512^2: warmup {args.warmup}, timed {args.steps} steps, variant "
        f"{lbm.lbm_step_variant_info(ctx.variant)}")
    secs, f_end = time_forward(ctx, f0, args.steps, args.warmup)
    lups = setup.nx * setup.ny * args.steps
    mlups = lups / secs / 1e6
    ms_step = secs / args.steps * 1e3
    achieved = BYTES_PER_LUP * lups / secs / 1e9
    log(f"forward 512^2: {mlups:.1f} MLUPS, {ms_step * 1e3:.2f} us/step")
    rho = ctx.moments(f_end)[0]
    if not torch.isfinite(rho).all():
        raise SystemExit("non-finite state after the timed run")

    extra = {}
    # the 2048^2 shear layer: HBM-resident working set (2 x 637 MB)
    big = inputs.khi(2048, 2048, dx=1e-3, dy=1e-3, dt=1e-5, tau=1e-5, Dv=0.01, Drho=0.04)
    bctx = lbm.Context.from_setup(big)
    bf0 = bctx.init(*big.fields())
    bsecs, _ = time_forward(bctx, bf0, args.large_steps, 10)
    blups = big.nx * big.ny * args.large_steps
    extra["forward_2048"] = {
        "MLUPS": blups / bsecs / 1e6, "steps": args.large_steps,
        "us_per_step": bsecs / args.large_steps * 1e6,
        "hbm_frac": BYTES_PER_LUP * blups / bsecs / 1e9 / HBM_PEAK_GBS,
    }
    log(f"forward 2048^2: {extra['forward_2048']}")
    del bctx, bf0
    torch.cuda.empty_cache()

    out = {
        "metric": "MLUPS (D2V19+WENO5, FP64) fwd/adjoint/batched + % HBM roofline",
        "value": mlups,
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "single shear layer (KHI) 512x512, periodic x, reflecting y, "
                               "dx=dy=1e-3, dt=tau=1e-5, D_v=D_rho=0.02, forward step",
                   "nx": 512, "ny": 512, "steps": args.steps},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None},
        "extra": extra,
    }
    if not args.no_cpu:
        log("cpu baseline ...")
        small = inputs.khi(512, 512, dx=1e-3, dy=1e-3, dt=1e-5, tau=1e-5, Dv=0.02, Drho=0.02)
        out["cpu_baseline"] = cpu_baseline(small, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
