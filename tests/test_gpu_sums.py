"""Carried moment sums: lbm_sums, lbm_step_sums and lbm_adjoint_step_sums.

- lbm_sums against the oracle's moments (Eq. (10)): rho, rho u and
  rho T + rho |u|^2 / 2, to 1e-14 of each sum's scale.
- lbm_step_sums for every step variant on every boundary kind (grids with
  boundary tiles and ragged tails): f_out equal to lbm_step's bit for bit,
  two carried steps equal to lbm_step(nsteps = 2) bit for bit, and sums_out
  equal to lbm_sums(f_out) bit for bit for the fast-tile variants (mode 3)
  and the variants that do not carry sums, to 1e-14 for the others.
- lbm_adjoint_step_sums for every reverse variant: equal to lbm_adjoint_step
  bit for bit given lbm_sums(f_n), and within the adjoint parity bar of the
  oracle.
- The checkpointed gradient with a fast-tile forward variant (which carries
  the sums through the recompute and the reverse steps) against the CPU
  pipeline built from the oracle, and overlapped = sequential bit for bit.
- Argument errors."""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle
from paper_1010_4124_amd import inputs, lbm
from paper_1010_4124_amd.objective import KHIProblem, Schedule

pytestmark = pytest.mark.gpu
P, F, R, O = 0, 1, 2, 3
SIDES = [(1.1, 0.05, 0.0, 0.9), (0.8, -0.05, 0.02, 1.05), (1.0, 0.0, 0.05, 1.0),
         (0.9, 0.1, -0.05, 0.85)]
CASES = [((67, 45), (P, P, P, P)), ((130, 37), (R, R, F, F)), ((70, 41), (F, F, P, P)),
         ((69, 43), (R, R, R, R)), ((200, 50), (O, O, P, P)), ((5, 6), (P, P, R, R))]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    torch.cuda.set_device(0)


def _setup(nx, ny, bc, seed=1):
    p = oracle.OracleParams.make(nx, ny, 2e-2, 2.5e-2, 4e-4, 6e-4, bc, side_state=SIDES)
    f = oracle.init(p, *inputs.random_fields(nx, ny, seed, smooth=False))
    f = f * (1.0 + 0.05 * inputs.random_like((19, ny, nx), seed + 1))
    ctx = lbm.Context(nx, ny, 2e-2, 2.5e-2, 4e-4, 6e-4, bc, side_state=SIDES)
    return p, f, ctx


@pytest.mark.parametrize("shape,bc", CASES)
def test_sums_match_oracle_moments(shape, bc):
    nx, ny = shape
    p, f, ctx = _setup(nx, ny, bc)
    got = ctx.sums(torch.from_numpy(f).cuda()).cpu().numpy()
    rho, ux, uy, T = oracle.moments(p, f)
    ref = (rho, rho * ux, rho * uy, rho * T + 0.5 * rho * (ux * ux + uy * uy))
    for q in range(4):
        scale = max(np.abs(ref[q]).max(), np.abs(rho).max() * 1e-3)
        err = float(np.abs(got[q] - ref[q]).max() / scale)
        assert err < 1e-14, (q, err)


@pytest.mark.parametrize("shape,bc", CASES)
def test_step_sums_is_the_step(shape, bc):
    nx, ny = shape
    _, f, ctx = _setup(nx, ny, bc)
    fg = torch.from_numpy(f).cuda()
    for v in range(lbm.lbm_step_variant_count()):
        info = lbm.lbm_step_variant_info(v)
        ctx.variant = v
        ref1 = ctx.step(fg, 1)
        ref2 = ctx.step(fg, 2)
        s0 = ctx.sums(fg)
        f1, s1 = ctx.step_sums(fg, s0)
        f2, s2 = ctx.step_sums(f1, s1)
        f1n, s1n = ctx.step_sums(fg, None)
        assert torch.equal(f1, ref1), info
        assert torch.equal(f1n, ref1) and torch.equal(s1n, s1), info
        assert torch.equal(f2, ref2), info
        exact = ctx.sums(f1)
        if info[5] in (0, 2, 3):
            assert torch.equal(s1, exact), info
        else:
            err = float((s1 - exact).abs().max() / exact.abs().max())
            assert err < 1e-14, (info, err)
        print(f"step_sums {shape} {bc} variant {info}: ok", flush=True)


@pytest.mark.parametrize("shape,bc", [c for c in CASES if O not in c[1]])
def test_adjoint_step_sums_is_the_adjoint_step(shape, bc):
    nx, ny = shape
    p, f, ctx = _setup(nx, ny, bc)
    lam = inputs.random_like(f.shape, 3)
    ref = oracle.adjoint_step(p, f, lam, 0.7)
    fg, lg = torch.from_numpy(f).cuda(), torch.from_numpy(lam).cuda()
    sg = ctx.sums(fg)
    for v in range(lbm.lbm_adjoint_variant_count()):
        ctx.adj_variant = v
        a = ctx.adjoint_step(fg, lg, 0.7)
        b = ctx.adjoint_step(fg, lg, 0.7, sums=sg)
        assert torch.equal(a, b), lbm.lbm_adjoint_variant_info(v)
        err = float(np.abs(b.cpu().numpy() - ref).max() / np.abs(ref).max())
        assert err < 1e-12, (v, err)


def _fast_variant():
    return next(v for v in range(lbm.lbm_step_variant_count())
                if lbm.lbm_step_variant_info(v) == (4, 1, 2, 1, 1, 3))


def test_gradient_with_carried_sums_matches_oracle_pipeline():
    """The checkpointed gradient with the fast-tile forward variant (moment
    sums carried through the recompute into the reverse steps) against the
    CPU pipeline built from the oracle alone (the bars of the default-variant
    test)."""
    from test_gpu_objective import oracle_gradient
    prob = KHIProblem(64, 48, dx=1e-3, dy=1e-3, dt=1e-5, tau=1e-5, nsteps=40, window=(10, 40),
                      schedule=Schedule(16, 4))
    prob.ctx.variant = _fast_variant()
    Dv, Drho = 0.006, 0.009
    amps = inputs.mode_amplitudes(64, seed=3, base=1e-2)
    J, ck = prob.run(Dv, Drho, amps)
    gDv, gDrho, ga = prob.gradient(Dv, Drho, amps, ck)
    Jo, oDv, oDrho, oa = oracle_gradient(prob, Dv, Drho, amps)
    assert J == pytest.approx(Jo, rel=1e-12)
    assert gDv == pytest.approx(oDv, rel=1e-10)
    assert gDrho == pytest.approx(oDrho, rel=1e-10)
    assert np.abs(ga - oa).max() < 1e-10 * np.abs(oa).max()


@pytest.mark.parametrize("nsteps,sch", [(60, Schedule(30, 6)), (45, Schedule(16, 5))])
def test_gradient_with_carried_sums_schedules_and_overlap(nsteps, sch):
    """With carried sums, overlapped = sequential bit for bit, and the same
    as a single-level schedule bit for bit (the sums are lbm_sums's)."""
    amps = inputs.mode_amplitudes(64, seed=5, base=1e-2)
    res = []
    for s in (sch, Schedule.every(nsteps)):
        prob = KHIProblem(64, 40, nsteps=nsteps, window=(nsteps // 3, nsteps), schedule=s)
        prob.ctx.variant = _fast_variant()
        _, ck = prob.run(0.008, 0.01, amps)
        a = prob.gradient(0.008, 0.01, amps, ck, overlap=False)
        b = prob.gradient(0.008, 0.01, amps, ck, overlap=True)
        assert a[0] == b[0] and a[1] == b[1] and np.array_equal(a[2], b[2])
        res.append(a)
    assert res[0][0] == res[1][0] and res[0][1] == res[1][1]
    assert np.array_equal(res[0][2], res[1][2])


def test_sums_argument_errors():
    nx, ny = 67, 45
    _, f, ctx = _setup(nx, ny, (P, P, R, R))
    fg = torch.from_numpy(f).cuda()
    lam = torch.zeros_like(fg)
    out = torch.empty_like(fg)
    L = lbm.lib()
    ptr = lambda t: C.c_void_p(t.data_ptr())  # noqa: E731
    # no sums for the sums form of the reverse step
    assert L.lbm_adjoint_step_sums(ctx.handle, ptr(fg), None, ptr(lam), 0.0, ptr(out),
                                   None) == lbm.LBM_EINVAL
    # sums_out inside f_in; f_out on f_in; a null sums_out
    s = ctx.sums(fg)
    assert L.lbm_step_sums(ctx.handle, ptr(fg), ptr(s), ptr(out), ptr(fg), None) == lbm.LBM_EINVAL
    assert L.lbm_step_sums(ctx.handle, ptr(fg), ptr(s), ptr(fg), ptr(s), None) == lbm.LBM_EINVAL
    assert L.lbm_step_sums(ctx.handle, ptr(fg), ptr(s), ptr(out), None, None) == lbm.LBM_EINVAL
    # sums on f
    assert L.lbm_sums(ctx.handle, ptr(fg), ptr(fg), None) == lbm.LBM_EINVAL
    # the reverse step's output on the sums
    big = torch.empty_like(fg)
    assert L.lbm_adjoint_step_sums(ctx.handle, ptr(fg), ptr(big), ptr(lam), 0.0, ptr(big),
                                   None) == lbm.LBM_EINVAL
