"""Autotuner: times every variant natively, selects the fastest and caches
the choice per device and shape; results change only by rounding."""
import json

import pytest
import torch

from paper_1010_4124_amd import inputs, lbm, tune

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _env(tmp_path, monkeypatch):
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    torch.cuda.set_device(0)
    monkeypatch.setenv("LBM_TUNE_CACHE", str(tmp_path / "tune.json"))


def test_tune_context_selects_fastest_and_caches():
    s = inputs.khi(192, 96, Dv=0.02, Drho=0.02, pert=1e-2)
    ctx = lbm.Context.from_setup(s)
    f0 = ctx.init(*s.fields())
    ref = ctx.step(f0, 3)
    r = tune.tune_context(ctx, f0, nsteps=5)
    n = lbm.lbm_step_variant_count()
    assert not r["cached"] and len(r["ms"]) == n
    assert all(v > 0 for v in r["ms"].values())
    best = min(r["ms"].values())
    ties = [int(k) for k, v in r["ms"].items() if v <= best * (1 + tune.TIE)]
    assert ctx.variant == min(ties) == r["variant"]
    # variants group the WENO face arithmetic by tile height: same result up
    # to rounding
    got = ctx.step(f0, 3)
    assert float((got - ref).abs().max() / ref.abs().max()) < 1e-14
    db = json.load(open(tune.cache_path()))
    assert tune.context_key(ctx) in db
    ctx.variant = (r["variant"] + 1) % n
    r2 = tune.tune_context(ctx, f0)
    assert r2["cached"] and ctx.variant == r["variant"]


def test_tune_batch_selects_pair():
    setups = [inputs.khi(128, 64, Dv=0.02, Drho=0.01), inputs.khi(64, 128, Dv=0.01, Drho=0.02)]
    b = lbm.Batch.from_setups(setups)
    fields = [s.fields() for s in setups]
    f0 = b.init(*[b.pack_scalars([f[q] for f in fields]) for q in range(4)])
    ref = b.step(f0, 2)
    r = tune.tune_batch(b, f0, nsteps=3, slots=(0, 64))
    assert len(r["ms"]) == 2 * lbm.lbm_step_variant_count()
    best = min(r["ms"].values())
    ties = [tuple(int(x) for x in k.split(",")) for k, v in r["ms"].items()
            if v <= best * (1 + tune.TIE)]
    assert (b.variant, b.schedule[0]) == min(ties)
    got = b.step(f0, 2)
    assert float((got - ref).abs().max() / ref.abs().max()) < 1e-14
    r2 = tune.tune_batch(b, f0)
    assert r2["cached"]


def test_tune_adjoint_selects_fastest():
    s = inputs.khi(128, 96, Dv=0.02, Drho=0.02, pert=1e-2)
    ctx = lbm.Context.from_setup(s)
    f0 = ctx.init(*s.fields())
    lam = torch.randn_like(f0)
    ref = ctx.adjoint_step(f0, lam, 1e-5)
    r = tune.tune_adjoint(ctx, f0, lam, nsteps=2)
    n = lbm.lbm_adjoint_variant_count()
    assert len(r["ms"]) == n and all(v > 0 for v in r["ms"].values())
    best = min(r["ms"].values())
    ties = [int(k) for k, v in r["ms"].items() if v <= best * (1 + tune.TIE)]
    assert ctx.adj_variant == min(ties)
    got = ctx.adjoint_step(f0, lam, 1e-5)
    assert float((got - ref).abs().max() / ref.abs().max()) < 1e-13
    assert tune.tune_adjoint(ctx, f0, lam)["cached"]
