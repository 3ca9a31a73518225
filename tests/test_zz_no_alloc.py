"""lbm_kinetic_y_noalloc (the entry point that allocates nothing) against
lbm_kinetic_y through the C-ABI: two calls in a row on different grids, the
second smaller, each identical to the context entry point's result (same
kernels, same summation order), plus the size limit."""
import pytest
import torch

from paper_1010_4124_amd import inputs, lbm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    torch.cuda.set_device(0)


def _state(s, nsteps):
    ctx = lbm.Context.from_setup(s)
    f = ctx.init(*s.fields())
    return ctx, ctx.step(f, nsteps) if nsteps else f


def test_noalloc_matches_context_entry_point_twice():
    cases = [inputs.khi(1030, 517, Dv=0.01, Drho=0.02), inputs.khi(96, 40, Dv=0.01, Drho=0.01)]
    for s, nsteps in zip(cases, (20, 7)):
        ctx, f = _state(s, nsteps)
        ref = ctx.kinetic_y(f)
        got = torch.full((2,), float("nan"), dtype=torch.float64, device=f.device)
        lbm.lbm_kinetic_y_noalloc(ctx.params, f, got)
        torch.cuda.synchronize()
        print(f"{s.nx}x{s.ny}: noalloc {got.tolist()} context {ref.tolist()}", flush=True)
        assert torch.equal(got, ref)


def test_noalloc_x_axis_and_limit():
    s = inputs.khi_paper(120, 64)
    ctx, f = _state(s, 5)
    got = torch.empty(2, dtype=torch.float64, device=f.device)
    lbm.lbm_kinetic_y_noalloc(ctx.params, f, got)
    assert torch.equal(got, ctx.kinetic_y(f))
    # one cell over the limit: refused on the host before any launch (the
    # small buffers passed are never touched)
    import ctypes as C
    big = lbm.LbmParams.make(4097, 4096, 1e-3, 1e-3, 1e-5, 1e-5)
    rc = lbm.lib().lbm_kinetic_y_noalloc(C.byref(big), C.c_void_p(f.data_ptr()),
                                         C.c_void_p(got.data_ptr()), None)
    assert rc == lbm.LBM_EINVAL
    assert "fixed scratch" in lbm.lib().lbm_last_error().decode()
