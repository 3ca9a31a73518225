"""The C-ABI library loads and exports every function include/lbm.h declares
(no compute call: these run without a GPU)."""
import os

import pytest

from paper_1010_4124_amd import lbm


def test_library_built():
    assert os.path.exists(lbm.LIB_PATH), "run __graft_entry__.build() first"


def test_exports_every_declared_symbol():
    names = lbm.header_functions()
    assert "lbm_step" in names and "lbm_init" in names and "lbm_moments" in names
    L = lbm.lib()
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_version_and_variants_without_gpu():
    L = lbm.lib()
    assert b"gfx950" in L.lbm_version()
    n = lbm.lbm_step_variant_count()
    assert n >= 2
    for v in range(n):
        R, G, W, D, NT, M = lbm.lbm_step_variant_info(v)
        assert R in (1, 2, 4, 8) and G in (1, 2, 3, 6, 9, 18) and W >= 1 and D in (1, 2)
        assert NT in (0, 1) and M in (0, 1, 2, 3) and 18 % G == 0
    with pytest.raises(lbm.LbmError):
        lbm.lbm_step_variant_info(n)
    na = lbm.lbm_adjoint_variant_count()
    assert na >= 2
    for v in range(na):
        R, G, W, PS = lbm.lbm_adjoint_variant_info(v)
        assert 18 % G == 0 and W >= 1 and PS in (0, 1, 2)
        # tile rows, or the rows of a marched chunk (a multiple of 4)
        assert R in (2, 4, 8) if PS < 2 else (R % 4 == 0 and G == 18)
    with pytest.raises(lbm.LbmError):
        lbm.lbm_adjoint_variant_info(na)


def test_create_rejects_bad_params_without_gpu():
    """Parameter validation happens before any device work."""
    import ctypes as C
    L = lbm.lib()
    bad = [
        lbm.LbmParams.make(0, 4, 1e-3, 1e-3, 1e-5, 1e-5),
        lbm.LbmParams.make(8, 8, 1e-3, 1e-3, -1e-5, 1e-5),
        lbm.LbmParams.make(8, 8, 1e-3, 1e-3, 1e-5, 0.0),
        lbm.LbmParams.make(8, 8, 1e-3, 1e-3, 1e-5, 1e-5, vk=(1, 1, 3)),
        lbm.LbmParams.make(2, 8, 1e-3, 1e-3, 1e-5, 1e-5, bc=(2, 2, 0, 0)),
        lbm.LbmParams.make(8, 8, 1e-3, 1e-3, 1e-5, 1e-5, bc=(0, 2, 0, 0)),
        lbm.LbmParams.make(8, 8, 1e-3, 1e-3, 1e-5, 1e-5, bc=(1, 1, 0, 0)),  # side rho = 0
    ]
    for p in bad:
        h = C.c_void_p()
        assert L.lbm_create(C.byref(p), C.byref(h)) == lbm.LBM_EINVAL
        assert L.lbm_last_error()
    for p in (lbm.LbmParams.make(8, 8, 1e-3, 1e-3, 1e-5, 1e-5, ke_axis=2),
              lbm.LbmParams.make(8, 8, 1e-3, 1e-3, 1e-5, 1e-5, bc=(3, 3, 0, 0), ke_axis=-1)):
        h = C.c_void_p()
        assert L.lbm_create(C.byref(p), C.byref(h)) == lbm.LBM_EINVAL
    for bad_scheme in (-1, 3):
        p = lbm.LbmParams.make(8, 8, 1e-3, 1e-3, 1e-5, 1e-5, scheme=bad_scheme)
        assert L.lbm_create(C.byref(p), C.byref(h)) == lbm.LBM_EINVAL


def test_batch_create_rejects_bad_instances_without_gpu():
    """Batch validation (instances, shared vk and eps, offsets) happens before
    any device work."""
    import ctypes as C
    L = lbm.lib()

    def create(ps, offs=None):
        arr = (lbm.LbmParams * len(ps))(*ps)
        o = None if offs is None else (C.c_int64 * len(ps))(*offs)
        h = C.c_void_p()
        return L.lbm_batch_create(arr, len(ps), o, C.byref(h))

    good = lbm.LbmParams.make(8, 8, 1e-3, 1e-3, 1e-5, 1e-5)
    other_vk = lbm.LbmParams.make(8, 8, 1e-3, 1e-3, 1e-5, 1e-5, vk=(1.0, 2.0, 3.5))
    other_eps = lbm.LbmParams.make(8, 8, 1e-3, 1e-3, 1e-5, 1e-5, eps=1e-7)
    bad = lbm.LbmParams.make(8, 8, 1e-3, 1e-3, 1e-5, 0.0)
    bad_axis = lbm.LbmParams.make(8, 8, 1e-3, 1e-3, 1e-5, 1e-5, ke_axis=3)
    h = C.c_void_p()
    assert L.lbm_batch_create(None, 1, None, C.byref(h)) == lbm.LBM_EINVAL
    assert create([good, other_vk]) == lbm.LBM_EINVAL
    assert create([good, other_eps]) == lbm.LBM_EINVAL
    assert create([good, bad]) == lbm.LBM_EINVAL
    assert create([good, bad_axis]) == lbm.LBM_EINVAL
    # the batched step is WENO5's only
    assert create([good, lbm.LbmParams.make(8, 8, 1e-3, 1e-3, 1e-5, 1e-5,
                                            scheme=lbm.UPWIND1)]) == lbm.LBM_EUNSUPPORTED
    assert b"WENO5" in L.lbm_last_error()
    n = 19 * 64
    assert create([good, good], [0, n - 1]) == lbm.LBM_EINVAL     # overlapping blocks
    assert create([good, good], [n, 0 + 5]) == lbm.LBM_EINVAL     # overlapping, reversed
    assert create([good, good], [-1, n]) == lbm.LBM_EINVAL        # negative offset
    assert b"overlap" in L.lbm_last_error()


def test_sums_entry_points_reject_null_arguments_without_gpu():
    """lbm_sums, lbm_step_sums and lbm_adjoint_step_sums check their
    arguments before any device work."""
    L = lbm.lib()
    assert L.lbm_sums(None, None, None, None) == lbm.LBM_EINVAL
    assert L.lbm_step_sums(None, None, None, None, None, None) == lbm.LBM_EINVAL
    assert L.lbm_adjoint_step_sums(None, None, None, None, 0.0, None, None) == lbm.LBM_EINVAL
    assert b"null" in L.lbm_last_error()
