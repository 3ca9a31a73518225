"""ctypes binding of liblbm_hip.so (the C-ABI of include/lbm.h).

Argument marshalling only: torch tensors supply device pointers and the
current HIP stream; every step of the computation runs in the library's HIP
kernels. The binding refuses to run without the built library and without a
GPU: there is no CPU fallback.

Functions carry the C entry points' names (``lbm_create``, ``lbm_init``,
``lbm_step``, ...); ``Context`` is a small owner of an ``lbm_ctx*``.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm_hip.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "lbm.h")

NV = 19
PERIODIC, FIXED_EQ, REFLECT, OUTFLOW = 0, 1, 2, 3
WENO5, UPWIND1, UPWIND2 = 0, 1, 2  # lbm_params.scheme
LBM_OK, LBM_EINVAL, LBM_EUNSUPPORTED, LBM_EHIP, LBM_ENOMEM = 0, -1, -2, -3, -4
LBM_ENONFINITE, LBM_ENONPHYS = -5, -6


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"liblbm_hip error {code}: {msg}")
        self.code = code


class LbmParams(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("bc", C.c_int32 * 4),
        ("dx", C.c_double), ("dy", C.c_double), ("dt", C.c_double), ("tau", C.c_double),
        ("vk", C.c_double * 3), ("weno_eps", C.c_double),
        ("side_state", (C.c_double * 4) * 4),
        ("ke_axis", C.c_int32), ("scheme", C.c_int32),
    ]

    @classmethod
    def make(cls, nx, ny, dx, dy, dt, tau, bc=(PERIODIC,) * 4, vk=(1.0, 2.0, 3.0), eps=1e-6,
             side_state=None, ke_axis=0, scheme=WENO5):
        p = cls()
        p.ke_axis = int(ke_axis)
        p.scheme = int(scheme)
        p.nx, p.ny = int(nx), int(ny)
        for s in range(4):
            p.bc[s] = int(bc[s])
        p.dx, p.dy, p.dt, p.tau = float(dx), float(dy), float(dt), float(tau)
        for k in range(3):
            p.vk[k] = float(vk[k])
        p.weno_eps = float(eps)
        if side_state is not None:
            for s in range(4):
                if side_state[s] is not None:
                    for q in range(4):
                        p.side_state[s][q] = float(side_state[s][q])
        return p


_lib = None
_P = C.c_void_p
_I = C.c_int32


def header_functions(path=HEADER):
    """Names of the functions include/lbm.h declares."""
    txt = open(path).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z0-9_]+)\s*\(", txt)))


def lib():
    """Load liblbm_hip.so (built by paper_1010_4124_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() "
                           "(the HIP library is the only compute path)")
    L = C.CDLL(LIB_PATH)
    sig = {
        "lbm_create": (C.c_int, [C.POINTER(LbmParams), C.POINTER(C.c_void_p)]),
        "lbm_destroy": (None, [_P]),
        "lbm_init": (C.c_int, [_P, _P, _P, _P, _P, _P, _P]),
        "lbm_step": (C.c_int, [_P, _P, _P, _I, _P, _P]),
        "lbm_moments": (C.c_int, [_P, _P, _P, _P, _P, _P, _P]),
        "lbm_sums": (C.c_int, [_P, _P, _P, _P]),
        "lbm_step_sums": (C.c_int, [_P, _P, _P, _P, _P, _P]),
        "lbm_kinetic_y": (C.c_int, [_P, _P, _P, _P]),
        "lbm_check_state": (C.c_int, [_P, _P, C.POINTER(C.c_int64), _P]),
        "lbm_kinetic_y_noalloc": (C.c_int, [C.POINTER(LbmParams), _P, _P, _P]),
        "lbm_step_variant_count": (C.c_int, []),
        "lbm_step_variant_info": (C.c_int, [_I, C.POINTER(_I)]),
        "lbm_set_step_variant": (C.c_int, [_P, _I]),
        "lbm_get_step_variant": (C.c_int, [_P, C.POINTER(_I)]),
        "lbm_adjoint_step": (C.c_int, [_P, _P, _P, C.c_double, _P, _P]),
        "lbm_adjoint_step_sums": (C.c_int, [_P, _P, _P, _P, C.c_double, _P, _P]),
        "lbm_init_vjp": (C.c_int, [_P] + [_P] * 9 + [_P]),
        "lbm_sep_project": (C.c_int, [_P, _P, _P, _I, _P, _P, _P]),
        "lbm_batch_create": (C.c_int, [C.POINTER(LbmParams), _I, C.POINTER(C.c_int64),
                                       C.POINTER(C.c_void_p)]),
        "lbm_batch_destroy": (None, [_P]),
        "lbm_batch_info": (C.c_int, [_P, C.POINTER(C.c_int64)]),
        "lbm_batch_init": (C.c_int, [_P, _P, _P, _P, _P, _P, _P]),
        "lbm_batch_moments": (C.c_int, [_P, _P, _P, _P, _P, _P, _P]),
        "lbm_batch_step": (C.c_int, [_P, _P, _P, _I, _P, _P]),
        "lbm_batch_set_step_variant": (C.c_int, [_P, _I]),
        "lbm_batch_get_step_variant": (C.c_int, [_P, C.POINTER(_I)]),
        "lbm_batch_set_schedule": (C.c_int, [_P, _I, _I]),
        "lbm_batch_get_schedule": (C.c_int, [_P, C.POINTER(_I)]),
        "lbm_tune_step": (C.c_int, [_P, _P, _P, _I, C.POINTER(_I), _I, C.POINTER(C.c_double), _P]),
        "lbm_adjoint_variant_count": (C.c_int, []),
        "lbm_adjoint_variant_info": (C.c_int, [_I, C.POINTER(_I)]),
        "lbm_set_adjoint_variant": (C.c_int, [_P, _I]),
        "lbm_get_adjoint_variant": (C.c_int, [_P, C.POINTER(_I)]),
        "lbm_tune_adjoint": (C.c_int, [_P, _P, _P, _P, _I, C.POINTER(_I), _I,
                                       C.POINTER(C.c_double), _P]),
        "lbm_batch_tune": (C.c_int, [_P, _P, _P, _I, C.POINTER(_I), _I, C.POINTER(_I), _I,
                                     C.POINTER(C.c_double), _P]),
        "lbm_last_error": (C.c_char_p, []),
        "lbm_version": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name, None)
        if fn is None:
            continue
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _check(rc):
    if rc != LBM_OK:
        raise LbmError(rc, lib().lbm_last_error().decode())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t, shape=None, what="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{what} must be float64")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{what} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return C.c_void_p(t.data_ptr())


def _require_gpu():
    if not torch.cuda.is_available():
        raise RuntimeError("liblbm_hip needs a HIP GPU; no CPU fallback exists")


# --- thin wrappers carrying the C names -----------------------------------
def lbm_create(params: LbmParams):
    _require_gpu()
    h = C.c_void_p()
    _check(lib().lbm_create(C.byref(params), C.byref(h)))
    return h


def lbm_destroy(h):
    if h:
        lib().lbm_destroy(h)


def lbm_init(h, nx, ny, rho, ux, uy, T, f_out, stream=None):
    s = (ny, nx)
    _check(lib().lbm_init(h, _ptr(rho, s, "rho"), _ptr(ux, s, "ux"), _ptr(uy, s, "uy"),
                          _ptr(T, s, "T"), _ptr(f_out, (NV, ny, nx), "f_out"), _stream(stream)))


def lbm_step(h, nx, ny, f_in, f_out, nsteps=1, ke_log=None, stream=None):
    if ke_log is not None:
        _ptr(ke_log, (int(nsteps), 2), "ke_log")
    _check(lib().lbm_step(h, _ptr(f_in, (NV, ny, nx), "f_in"), _ptr(f_out, (NV, ny, nx), "f_out"),
                          int(nsteps), _ptr(ke_log), _stream(stream)))


def lbm_sums(h, nx, ny, f, sums, stream=None):
    _check(lib().lbm_sums(h, _ptr(f, (NV, ny, nx), "f"), _ptr(sums, (4, ny, nx), "sums"),
                          _stream(stream)))


def lbm_step_sums(h, nx, ny, f_in, sums_in, f_out, sums_out, stream=None):
    s4 = (4, ny, nx)
    _check(lib().lbm_step_sums(h, _ptr(f_in, (NV, ny, nx), "f_in"),
                               None if sums_in is None else _ptr(sums_in, s4, "sums_in"),
                               _ptr(f_out, (NV, ny, nx), "f_out"), _ptr(sums_out, s4, "sums_out"),
                               _stream(stream)))


def lbm_moments(h, nx, ny, f, rho, ux, uy, T, stream=None):
    s = (ny, nx)
    _check(lib().lbm_moments(h, _ptr(f, (NV, ny, nx), "f"), _ptr(rho, s, "rho"), _ptr(ux, s, "ux"),
                             _ptr(uy, s, "uy"), _ptr(T, s, "T"), _stream(stream)))


def lbm_kinetic_y(h, nx, ny, f, out2, stream=None):
    _check(lib().lbm_kinetic_y(h, _ptr(f, (NV, ny, nx), "f"), _ptr(out2, (2,), "out2"),
                               _stream(stream)))


def lbm_kinetic_y_noalloc(params, f, out2, stream=None):
    """lbm_kinetic_y from parameters alone (no context), allocating nothing."""
    nx, ny = int(params.nx), int(params.ny)
    _check(lib().lbm_kinetic_y_noalloc(C.byref(params), _ptr(f, (NV, ny, nx), "f"),
                                       _ptr(out2, (2,), "out2"), _stream(stream)))


def lbm_check_state(h, nx, ny, f, stream=None, raise_error=True):
    """(return code, (non-finite cells, non-physical cells, first non-finite
    cell, first non-physical cell)); with raise_error a non-zero code raises
    LbmError (whose .code is LBM_ENONFINITE or LBM_ENONPHYS)."""
    out = (C.c_int64 * 4)()
    rc = lib().lbm_check_state(h, _ptr(f, (NV, ny, nx), "f"), out, _stream(stream))
    if raise_error:
        _check(rc)
    return rc, tuple(int(x) for x in out)


def lbm_adjoint_step(h, nx, ny, f_n, lam_np1, w, lam_n, stream=None):
    s = (NV, ny, nx)
    _check(lib().lbm_adjoint_step(h, _ptr(f_n, s, "f_n"), _ptr(lam_np1, s, "lam_np1"), float(w),
                                  _ptr(lam_n, s, "lam_n"), _stream(stream)))


def lbm_adjoint_step_sums(h, nx, ny, f_n, sums_n, lam_np1, w, lam_n, stream=None):
    s = (NV, ny, nx)
    _check(lib().lbm_adjoint_step_sums(h, _ptr(f_n, s, "f_n"), _ptr(sums_n, (4, ny, nx), "sums_n"),
                                       _ptr(lam_np1, s, "lam_np1"), float(w),
                                       _ptr(lam_n, s, "lam_n"), _stream(stream)))


def lbm_init_vjp(h, nx, ny, rho, ux, uy, T, lam0, g_rho, g_ux, g_uy, g_T, stream=None):
    s = (ny, nx)
    _check(lib().lbm_init_vjp(h, _ptr(rho, s, "rho"), _ptr(ux, s, "ux"), _ptr(uy, s, "uy"),
                              _ptr(T, s, "T"), _ptr(lam0, (NV, ny, nx), "lam0"),
                              _ptr(g_rho, s, "g_rho"), _ptr(g_ux, s, "g_ux"),
                              _ptr(g_uy, s, "g_uy"), _ptr(g_T, s, "g_T"), _stream(stream)))


def lbm_sep_project(h, nx, ny, g, A, B, out, stream=None):
    M = int(A.shape[0])
    _check(lib().lbm_sep_project(h, _ptr(g, (ny, nx), "g"), _ptr(A, (M, nx), "A"), M,
                                 _ptr(B, (ny,), "B"), _ptr(out, (M,), "out"), _stream(stream)))


def lbm_step_variant_count():
    return int(lib().lbm_step_variant_count())


def lbm_step_variant_info(v):
    """(rows per lane R, waves per tile G, waves-per-SIMD target W, planes in
    flight D, non-temporal stores NT, carried moments M)."""
    info = (_I * 6)()
    _check(lib().lbm_step_variant_info(int(v), info))
    return tuple(int(x) for x in info)


def lbm_set_step_variant(h, v):
    _check(lib().lbm_set_step_variant(h, int(v)))


def lbm_get_step_variant(h):
    v = _I()
    _check(lib().lbm_get_step_variant(h, C.byref(v)))
    return v.value


def lbm_adjoint_variant_count():
    return int(lib().lbm_adjoint_variant_count())


def lbm_adjoint_variant_info(v):
    """(rows per lane R, velocity groups G, waves-per-SIMD target W, state pass PS)."""
    info = (_I * 4)()
    _check(lib().lbm_adjoint_variant_info(int(v), info))
    return tuple(int(x) for x in info)


def lbm_set_adjoint_variant(h, v):
    _check(lib().lbm_set_adjoint_variant(h, int(v)))


def lbm_get_adjoint_variant(h):
    v = _I()
    _check(lib().lbm_get_adjoint_variant(h, C.byref(v)))
    return v.value


def lbm_tune_adjoint(h, nx, ny, f_n, lam_np1, lam_tmp, nsteps=5, variants=None, stream=None):
    """Times the reverse-step variants; returns {variant: ms per call} and
    leaves the fastest selected."""
    vs = list(range(lbm_adjoint_variant_count())) if variants is None else [int(v) for v in variants]
    ms = (C.c_double * len(vs))()
    s = (NV, ny, nx)
    _check(lib().lbm_tune_adjoint(h, _ptr(f_n, s, "f_n"), _ptr(lam_np1, s, "lam_np1"),
                                  _ptr(lam_tmp, s, "lam_tmp"), int(nsteps), (_I * len(vs))(*vs),
                                  len(vs), ms, _stream(stream)))
    return {v: ms[j] for j, v in enumerate(vs)}


def lbm_tune_step(h, nx, ny, f_in, f_tmp, nsteps=20, variants=None, stream=None):
    """Times the variants on this grid; returns {variant: ms per step} and
    leaves the fastest selected."""
    vs = list(range(lbm_step_variant_count())) if variants is None else [int(v) for v in variants]
    ms = (C.c_double * len(vs))()
    s = (NV, ny, nx)
    _check(lib().lbm_tune_step(h, _ptr(f_in, s, "f_in"), _ptr(f_tmp, s, "f_tmp"), int(nsteps),
                               (_I * len(vs))(*vs), len(vs), ms, _stream(stream)))
    return {v: ms[j] for j, v in enumerate(vs)}


# --- batches -------------------------------------------------------------------
def lbm_batch_create(params, f_offset=None):
    """params: sequence of LbmParams; f_offset: None or int sequence."""
    _require_gpu()
    n = len(params)
    arr = (LbmParams * n)(*params)
    offs = None if f_offset is None else (C.c_int64 * n)(*[int(o) for o in f_offset])
    h = C.c_void_p()
    _check(lib().lbm_batch_create(arr, n, offs, C.byref(h)))
    return h


def lbm_batch_destroy(h):
    if h:
        lib().lbm_batch_destroy(h)


def lbm_batch_info(h):
    """(n, field extent, total cells, work items per launch)."""
    out = (C.c_int64 * 4)()
    _check(lib().lbm_batch_info(h, out))
    return tuple(int(x) for x in out)


def _flat(t, n, what):
    if t is not None and t.dim() != 1:
        raise ValueError(f"{what} must be 1-d")
    return _ptr(t, (n,), what)


def lbm_batch_init(h, rho, ux, uy, T, f_out, stream=None):
    _, ext, cells, _ = lbm_batch_info(h)
    _check(lib().lbm_batch_init(h, _flat(rho, cells, "rho"), _flat(ux, cells, "ux"),
                                _flat(uy, cells, "uy"), _flat(T, cells, "T"),
                                _flat(f_out, ext, "f_out"), _stream(stream)))


def lbm_batch_moments(h, f, rho, ux, uy, T, stream=None):
    _, ext, cells, _ = lbm_batch_info(h)
    _check(lib().lbm_batch_moments(h, _flat(f, ext, "f"), _flat(rho, cells, "rho"),
                                   _flat(ux, cells, "ux"), _flat(uy, cells, "uy"),
                                   _flat(T, cells, "T"), _stream(stream)))


def lbm_batch_step(h, f_in, f_out, nsteps=1, ke_log=None, stream=None):
    n, ext, _, _ = lbm_batch_info(h)
    if ke_log is not None:
        _ptr(ke_log, (n, int(nsteps), 2), "ke_log")
    _check(lib().lbm_batch_step(h, _flat(f_in, ext, "f_in"), _flat(f_out, ext, "f_out"),
                                int(nsteps), _ptr(ke_log), _stream(stream)))


def lbm_batch_set_step_variant(h, v):
    _check(lib().lbm_batch_set_step_variant(h, int(v)))


def lbm_batch_get_step_variant(h):
    v = _I()
    _check(lib().lbm_batch_get_step_variant(h, C.byref(v)))
    return v.value


def lbm_batch_set_schedule(h, slots_per_xcd=0, graph_chunk=0):
    _check(lib().lbm_batch_set_schedule(h, int(slots_per_xcd), int(graph_chunk)))


def lbm_batch_get_schedule(h):
    out = (_I * 2)()
    _check(lib().lbm_batch_get_schedule(h, out))
    return int(out[0]), int(out[1])


def lbm_batch_tune(h, f_in, f_tmp, nsteps=10, variants=None, slots=None, stream=None):
    """Times (variant, slots) pairs; returns {(variant, slots): ms per step}
    and leaves the fastest selected."""
    _, ext, _, _ = lbm_batch_info(h)
    vs = list(range(lbm_step_variant_count())) if variants is None else [int(v) for v in variants]
    cur = lbm_batch_get_schedule(h)[0]
    ss = [cur] if slots is None else [int(x) for x in slots]
    ms = (C.c_double * (len(vs) * len(ss)))()
    _check(lib().lbm_batch_tune(h, _flat(f_in, ext, "f_in"), _flat(f_tmp, ext, "f_tmp"),
                                int(nsteps), (_I * len(vs))(*vs), len(vs), (_I * len(ss))(*ss),
                                len(ss), ms, _stream(stream)))
    return {(v, q): ms[j * len(ss) + k] for j, v in enumerate(vs) for k, q in enumerate(ss)}


class Batch:
    """Owns one lbm_batch* over instances given as LbmParams or Setups.

    Batch distribution fields are flat float64 tensors of ``extent`` elements
    (instance i's [19][ny][nx] block at ``offsets[i]``); batch scalar fields
    are flat tensors of ``cells`` elements packing the instances in order."""

    def __init__(self, params, f_offset=None):
        self.params = list(params)
        self.handle = lbm_batch_create(self.params, f_offset)
        self.n, self.extent, self.cells, _ = lbm_batch_info(self.handle)
        self.shapes = [(int(p.nx), int(p.ny)) for p in self.params]
        if f_offset is None:
            f_offset, o = [], 0
            for nx, ny in self.shapes:
                f_offset.append(o)
                o += NV * nx * ny
        self.offsets = [int(o) for o in f_offset]
        self.cell_offsets, c = [], 0
        for nx, ny in self.shapes:
            self.cell_offsets.append(c)
            c += nx * ny
        self.device = torch.device("cuda", torch.cuda.current_device())

    @classmethod
    def from_setups(cls, setups, f_offset=None):
        return cls([LbmParams.make(s.nx, s.ny, s.dx, s.dy, s.dt, s.tau, s.bc,
                                   side_state=s.side_state, ke_axis=getattr(s, "ke_axis", 0),
                                   scheme=getattr(s, "scheme", WENO5))
                    for s in setups], f_offset)

    def close(self):
        if getattr(self, "handle", None):
            lbm_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def empty_f(self):
        return torch.empty(self.extent, dtype=torch.float64, device=self.device)

    def empty_scalar(self):
        return torch.empty(self.cells, dtype=torch.float64, device=self.device)

    def view(self, f, i):
        """Instance i's (19, ny, nx) view of a batch field."""
        nx, ny = self.shapes[i]
        o = self.offsets[i]
        return f[o:o + NV * nx * ny].view(NV, ny, nx)

    def scalar_view(self, a, i):
        nx, ny = self.shapes[i]
        o = self.cell_offsets[i]
        return a[o:o + nx * ny].view(ny, nx)

    def pack_scalars(self, planes):
        """Concatenate per-instance (ny, nx) planes into one batch scalar field."""
        return torch.cat([torch.as_tensor(p, dtype=torch.float64).reshape(-1) for p in planes]).to(
            self.device).contiguous()

    def init(self, rho, ux, uy, T, out=None):
        out = self.empty_f() if out is None else out
        lbm_batch_init(self.handle, rho, ux, uy, T, out)
        return out

    def step(self, f, nsteps=1, out=None, ke_log=False):
        out = self.empty_f() if out is None else out
        ke = (torch.empty((self.n, int(nsteps), 2), dtype=torch.float64, device=self.device)
              if ke_log else None)
        lbm_batch_step(self.handle, f, out, nsteps, ke)
        return (out, ke) if ke_log else out

    def moments(self, f):
        outs = [self.empty_scalar() for _ in range(4)]
        lbm_batch_moments(self.handle, f, *outs)
        return tuple(outs)

    @property
    def variant(self):
        return lbm_batch_get_step_variant(self.handle)

    @variant.setter
    def variant(self, v):
        lbm_batch_set_step_variant(self.handle, v)

    @property
    def schedule(self):
        """(persistent workgroups per XCD or 0, graph chunk or 0)."""
        return lbm_batch_get_schedule(self.handle)

    @schedule.setter
    def schedule(self, sc):
        lbm_batch_set_schedule(self.handle, *sc)


# --- convenience owner -------------------------------------------------------
class Context:
    """Owns one lbm_ctx* for a grid and its parameters."""

    def __init__(self, nx, ny, dx, dy, dt, tau, bc=(PERIODIC,) * 4, vk=(1.0, 2.0, 3.0),
                 eps=1e-6, side_state=None, ke_axis=0, scheme=WENO5):
        self.params = LbmParams.make(nx, ny, dx, dy, dt, tau, bc, vk, eps, side_state, ke_axis,
                                     scheme)
        self.nx, self.ny = int(nx), int(ny)
        self.handle = lbm_create(self.params)
        self.device = torch.device("cuda", torch.cuda.current_device())

    @classmethod
    def from_setup(cls, s, **kw):
        return cls(s.nx, s.ny, s.dx, s.dy, s.dt, s.tau, s.bc, side_state=s.side_state,
                   ke_axis=getattr(s, "ke_axis", 0), scheme=getattr(s, "scheme", WENO5), **kw)

    def close(self):
        if getattr(self, "handle", None):
            lbm_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # allocation helpers (device memory comes from torch)
    def empty_f(self):
        return torch.empty((NV, self.ny, self.nx), dtype=torch.float64, device=self.device)

    def empty_plane(self):
        return torch.empty((self.ny, self.nx), dtype=torch.float64, device=self.device)

    def _dev(self, a):
        if isinstance(a, torch.Tensor):
            return a.to(device=self.device, dtype=torch.float64).contiguous()
        return torch.as_tensor(a, dtype=torch.float64, device=self.device).contiguous()

    def init(self, rho, ux, uy, T, out=None):
        out = self.empty_f() if out is None else out
        lbm_init(self.handle, self.nx, self.ny, *(self._dev(x) for x in (rho, ux, uy, T)), out)
        return out

    def step(self, f, nsteps=1, out=None, ke_log=False):
        out = self.empty_f() if out is None else out
        ke = torch.empty((int(nsteps), 2), dtype=torch.float64, device=self.device) if ke_log else None
        lbm_step(self.handle, self.nx, self.ny, f, out, nsteps, ke)
        return (out, ke) if ke_log else out

    def moments(self, f):
        outs = [self.empty_plane() for _ in range(4)]
        lbm_moments(self.handle, self.nx, self.ny, f, *outs)
        return tuple(outs)

    def empty_sums(self):
        return torch.empty((4, self.ny, self.nx), dtype=torch.float64, device=self.device)

    def sums(self, f, out=None):
        """lbm_sums: the moment sums (rho, j_x, j_y, E) of f, [4][ny][nx]."""
        out = self.empty_sums() if out is None else out
        lbm_sums(self.handle, self.nx, self.ny, f, out)
        return out

    def step_sums(self, f, sums=None, out=None, sums_out=None):
        """lbm_step_sums: one step from f (whose moment sums are `sums`, or
        None) -> (f_out, the moment sums of f_out)."""
        out = self.empty_f() if out is None else out
        sums_out = self.empty_sums() if sums_out is None else sums_out
        lbm_step_sums(self.handle, self.nx, self.ny, f, sums, out, sums_out)
        return out, sums_out

    def carries_sums(self):
        """True when the step variant carries the moment sums (modes 1, 3)."""
        return lbm_step_variant_info(self.variant)[5] in (1, 3)

    def kinetic_y(self, f):
        out = torch.empty(2, dtype=torch.float64, device=self.device)
        lbm_kinetic_y(self.handle, self.nx, self.ny, f, out)
        return out

    def check(self, f, raise_error=True):
        """lbm_check_state of f: (code, counts)."""
        return lbm_check_state(self.handle, self.nx, self.ny, f, raise_error=raise_error)

    def adjoint_step(self, f_n, lam_np1, w=0.0, out=None, sums=None):
        """lbm_adjoint_step, or lbm_adjoint_step_sums when the moment sums of
        f_n are given."""
        out = self.empty_f() if out is None else out
        if sums is None:
            lbm_adjoint_step(self.handle, self.nx, self.ny, f_n, lam_np1, w, out)
        else:
            lbm_adjoint_step_sums(self.handle, self.nx, self.ny, f_n, sums, lam_np1, w, out)
        return out

    def init_vjp(self, rho, ux, uy, T, lam0):
        outs = [self.empty_plane() for _ in range(4)]
        lbm_init_vjp(self.handle, self.nx, self.ny, *(self._dev(x) for x in (rho, ux, uy, T)),
                     lam0, *outs)
        return tuple(outs)

    def sep_project(self, g, A, B):
        A = self._dev(A)
        out = torch.empty(A.shape[0], dtype=torch.float64, device=self.device)
        lbm_sep_project(self.handle, self.nx, self.ny, g, A, self._dev(B), out)
        return out

    @property
    def variant(self):
        return lbm_get_step_variant(self.handle)

    @variant.setter
    def variant(self, v):
        lbm_set_step_variant(self.handle, v)

    @property
    def adj_variant(self):
        return lbm_get_adjoint_variant(self.handle)

    @adj_variant.setter
    def adj_variant(self, v):
        lbm_set_adjoint_variant(self.handle, v)
