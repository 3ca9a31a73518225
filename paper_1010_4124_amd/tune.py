"""Step-kernel autotuner with an on-disk cache.

The timing itself is native (lbm_tune_step / lbm_batch_tune time each
variant with HIP events); this module picks what to time, remembers the
winner per device and problem shape in a JSON file, and reapplies it.

Cache file: $LBM_TUNE_CACHE, else ~/.cache/lbm_hip/tune.json. A key names
the device, the kind of problem (single grid or batch), its shape and
boundary rules; a batch key covers every instance's shape.
"""
from __future__ import annotations

import hashlib
import json
import os
import statistics

import torch

from . import lbm


def cache_path():
    return os.environ.get("LBM_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "lbm_hip", "tune.json"))


def _load():
    try:
        with open(cache_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(db):
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as fh:
            json.dump(db, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass  # a read-only home only loses the cache


def _device():
    return torch.cuda.get_device_name(torch.cuda.current_device()).replace("|", "/")


def context_key(ctx):
    p = ctx.params
    return f"{_device()}|grid|{ctx.nx}x{ctx.ny}|bc{tuple(p.bc)}"


def batch_key(b):
    sig = ";".join(f"{nx}x{ny}:{tuple(p.bc)}" for (nx, ny), p in zip(b.shapes, b.params))
    return f"{_device()}|batch|n{b.n}|{hashlib.sha1(sig.encode()).hexdigest()[:16]}"


# Variants within this fraction of the fastest count as ties; the lowest
# index among them wins, so that repeated tuning of one shape is stable.
TIE = 0.015


def _pick(ms):
    best = min(ms.values())
    return min(k for k, v in ms.items() if v <= best * (1.0 + TIE))


def _central(runs):
    """Per-step time of each key from its repeated trials: the median. The
    step and batch tuners time a step as the difference of two calls, so a
    stall in the shorter call makes a trial read low; the median of three
    trials discards one such outlier, where the minimum would keep it."""
    return {k: statistics.median(v) for k, v in runs.items()}


def tune_context(ctx, f, nsteps=None, reps=3, use_cache=True):
    """Select the fastest step variant for ctx; f is a representative state.
    Each variant is timed `reps` times over nsteps and 2 nsteps steps
    (default: about 5e7 site updates) and keeps the median of its per-step
    times.
    Returns {"variant": v, "ms": {variant: ms per step}, "cached": bool}."""
    key = context_key(ctx)
    db = _load() if use_cache else {}
    n = lbm.lbm_step_variant_count()
    if key in db and 0 <= db[key]["variant"] < n:
        ctx.variant = db[key]["variant"]
        return dict(db[key], cached=True)
    tmp = ctx.empty_f()
    if nsteps is None:
        nsteps = max(3, min(200, int(5e7 / (ctx.nx * ctx.ny))))
    runs = {}
    for _ in range(max(1, reps)):
        for k, v in lbm.lbm_tune_step(ctx.handle, ctx.nx, ctx.ny, f, tmp, nsteps).items():
            runs.setdefault(k, []).append(v)
    ms = _central(runs)
    ctx.variant = _pick(ms)
    rec = {"variant": ctx.variant, "ms": {str(k): v for k, v in ms.items()}}
    if use_cache:
        db = _load()
        db[key] = rec
        _store(db)
    return dict(rec, cached=False)


def tune_batch(b, f, nsteps=None, slots=(0,), reps=3, use_cache=True):
    """Select the fastest (variant, persistent slots per XCD) for batch b,
    with the same repetition and tie rule as tune_context."""
    key = batch_key(b)
    db = _load() if use_cache else {}
    n = lbm.lbm_step_variant_count()
    if key in db and 0 <= db[key]["variant"] < n:
        b.variant = db[key]["variant"]
        b.schedule = (db[key]["slots"], b.schedule[1])
        return dict(db[key], cached=True)
    tmp = b.empty_f()
    if nsteps is None:
        nsteps = max(3, min(200, int(5e7 / b.cells)))
    runs = {}
    for _ in range(max(1, reps)):
        for k, v in lbm.lbm_batch_tune(b.handle, f, tmp, nsteps, slots=slots).items():
            runs.setdefault(k, []).append(v)
    ms = _central(runs)
    v, q = _pick(ms)
    b.variant = v
    b.schedule = (q, b.schedule[1])
    rec = {"variant": b.variant, "slots": b.schedule[0],
           "ms": {f"{v},{q}": t for (v, q), t in ms.items()}}
    if use_cache:
        db = _load()
        db[key] = rec
        _store(db)
    return dict(rec, cached=False)


def tune_adjoint(ctx, f, lam, nsteps=None, reps=2, use_cache=True):
    """Select the fastest reverse-step variant for ctx (f, lam: representative
    f^n and lambda^{n+1}); same repetition and tie rule as tune_context."""
    key = context_key(ctx) + "|adjoint"
    db = _load() if use_cache else {}
    n = lbm.lbm_adjoint_variant_count()
    if key in db and 0 <= db[key]["variant"] < n:
        ctx.adj_variant = db[key]["variant"]
        return dict(db[key], cached=True)
    tmp = ctx.empty_f()
    if nsteps is None:
        nsteps = max(2, min(100, int(2e7 / (ctx.nx * ctx.ny))))
    ms = {}
    for _ in range(max(1, reps)):
        for k, v in lbm.lbm_tune_adjoint(ctx.handle, ctx.nx, ctx.ny, f, lam, tmp, nsteps).items():
            ms[k] = min(ms.get(k, v), v)
    ctx.adj_variant = _pick(ms)
    rec = {"variant": ctx.adj_variant, "ms": {str(k): v for k, v in ms.items()}}
    if use_cache:
        db = _load()
        db[key] = rec
        _store(db)
    return dict(rec, cached=False)
