"""ctypes binding of the plain C oracle (``lbm_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
benchmark's CPU-baseline leg, never by the GPU library.

Layout of every field: ``float64[19, ny, nx]`` (x fastest); scalar planes are
``float64[ny, nx]``. Boundary codes: 0 periodic, 1 fixed equilibrium
(Sec. III.B, Eq. (57)), 2 reflecting wall, 3 outflow (Sec. IV.A,
Eqs. (63)-(64)). Sides are ordered x-lo, x-hi, y-lo, y-hi.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import sysconfig

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.c")
LIB = os.path.join(HERE, "liblbm_oracle.so")

PERIODIC, FIXED_EQ, REFLECT, OUTFLOW = 0, 1, 2, 3
NV = 19

__all__ = [
    "OracleParams", "build_oracle", "lib", "lib_contracted", "velocity_table", "weights", "feq_cell",
    "moments_cell", "weno5", "weno5_grad", "weno_periodic_line", "scheme_periodic_line",
    "init", "moments", "state_check",
    "step", "kinetic_y", "kinetic_y_grad", "adjoint_step", "init_vjp", "feq_partials",
    "PERIODIC", "FIXED_EQ", "REFLECT", "OUTFLOW", "NV",
]


# The same source built with fused multiply-adds allowed (-mfma
# -ffp-contract=fast): every expression then rounds once per fused pair
# instead of once per operation. Its arithmetic is the oracle's; it exists to
# measure how far two legal roundings of the same scheme drift apart over a
# long run (the rounding-accumulation reading of the long-run parity bar).
LIB_FMA = os.path.join(HERE, "liblbm_oracle_fma.so")


def build_oracle(force: bool = False, contract: bool = False) -> str:
    """Compile the oracle with gcc: -O2, no FMA contraction, no fast-math
    (contract=True: the FMA-contracted build, LIB_FMA)."""
    out = LIB_FMA if contract else LIB
    if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(SRC):
        return out
    tmp = out + ".tmp%d" % os.getpid()
    fp = ["-mfma", "-ffp-contract=fast"] if contract else ["-ffp-contract=off"]
    cmd = ["gcc", "-O2", *fp, "-fno-fast-math", "-fopenmp", "-fPIC",
           "-shared", "-std=c11", "-Wall", "-Wno-unused-function", SRC, "-o", tmp, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


class OracleParams(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("bc", C.c_int32 * 4),
        ("dx", C.c_double), ("dy", C.c_double), ("dt", C.c_double), ("tau", C.c_double),
        ("vk", C.c_double * 3), ("eps", C.c_double),
        ("side_state", (C.c_double * 4) * 4),
        ("scheme", C.c_int32), ("pad", C.c_int32),
    ]

    @classmethod
    def make(cls, nx, ny, dx, dy, dt, tau, bc=(PERIODIC,) * 4, vk=(1.0, 2.0, 3.0),
             eps=1e-6, side_state=None, scheme=0):
        p = cls()
        p.scheme = int(scheme)  # 0 WENO5, 1 first-order, 2 second-order upwind
        p.nx, p.ny = int(nx), int(ny)
        for s in range(4):
            p.bc[s] = int(bc[s])
        p.dx, p.dy, p.dt, p.tau = float(dx), float(dy), float(dt), float(tau)
        for k in range(3):
            p.vk[k] = float(vk[k])
        p.eps = float(eps)
        if side_state is not None:
            for s in range(4):
                if side_state[s] is not None:
                    for q in range(4):
                        p.side_state[s][q] = float(side_state[s][q])
        return p


_lib = None
_lib_fma = None


def lib_contracted():
    """The FMA-contracted build (LIB_FMA), with the same entry points."""
    global _lib_fma
    if _lib_fma is None:
        _lib_fma = _bind(C.CDLL(build_oracle(contract=True)))
    return _lib_fma


def lib():
    global _lib
    if _lib is None:
        _lib = _bind(C.CDLL(build_oracle()))
    return _lib


def _bind(L):
    """Declare the entry points' signatures on a loaded oracle build."""
    d = C.c_double
    pd = C.POINTER(C.c_double)
    pi = C.POINTER(C.c_int32)
    pp = C.POINTER(OracleParams)
    L.orc_velocity_table.argtypes = [pd, pd, pd, pd, pi, pi, pi]
    L.orc_weights.argtypes = [d, pd, pd]
    L.orc_weights.restype = None
    L.orc_feq_cell.argtypes = [d, d, d, d, pd, pd]
    L.orc_feq_cell.restype = None
    L.orc_moments_cell.argtypes = [pd, pd, pd]
    L.orc_moments_cell.restype = None
    L.orc_weno5.argtypes = [d, d, d, d, d, d]
    L.orc_weno5.restype = d
    L.orc_weno5_grad.argtypes = [d, d, d, d, d, d, pd]
    L.orc_weno5_grad.restype = None
    L.orc_weno_periodic_line.argtypes = [pd, C.c_int, C.c_int, d, pd]
    L.orc_weno_periodic_line.restype = None
    L.orc_scheme_periodic_line.argtypes = [pd, C.c_int, C.c_int, C.c_int, d, pd]
    L.orc_scheme_periodic_line.restype = None
    L.orc_init.argtypes = [pp, pd, pd, pd, pd, pd]
    L.orc_moments.argtypes = [pp, pd, pd, pd, pd, pd]
    L.orc_step.argtypes = [pp, pd, pd, C.c_int, C.c_int]
    L.orc_kinetic_y.argtypes = [pp, pd, pd]
    L.orc_kinetic_y_grad.argtypes = [pp, pd, pd]
    L.orc_adjoint_step.argtypes = [pp, pd, pd, d, pd]
    L.orc_init_vjp.argtypes = [pp, pd, pd, pd, pd, pd, pd, pd, pd, pd]
    L.orc_feq_partials.argtypes = [d, d, d, d, pd, C.c_int, pd]
    L.orc_feq_partials.restype = None
    return L


def _p(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _vk(vk):
    return np.ascontiguousarray(vk, dtype=np.float64)


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


def velocity_table(vk=(1.0, 2.0, 3.0)):
    """(vx, vy, |v|^2, shell, x-mirror, y-mirror) for the 19 velocities."""
    L = lib()
    vx, vy, vsq = np.zeros(NV), np.zeros(NV), np.zeros(NV)
    shell, mx, my = (np.zeros(NV, np.int32) for _ in range(3))
    pi = C.POINTER(C.c_int32)
    L.orc_velocity_table(_p(_vk(vk)), _p(vx), _p(vy), _p(vsq), shell.ctypes.data_as(pi),
                         mx.ctypes.data_as(pi), my.ctypes.data_as(pi))
    return vx, vy, vsq, shell, mx, my


def weights(T, vk=(1.0, 2.0, 3.0)):
    """(F_0, F_1, F_2, F_3) at temperature T."""
    F = np.zeros(4)
    lib().orc_weights(float(T), _p(_vk(vk)), _p(F))
    return F


def feq_cell(rho, ux, uy, T, vk=(1.0, 2.0, 3.0)):
    out = np.zeros(NV)
    lib().orc_feq_cell(float(rho), float(ux), float(uy), float(T), _p(_vk(vk)), _p(out))
    return out


def feq_partials(rho, ux, uy, T, i, vk=(1.0, 2.0, 3.0)):
    out = np.zeros(4)
    lib().orc_feq_partials(float(rho), float(ux), float(uy), float(T), _p(_vk(vk)), int(i),
                           _p(out))
    return out


def moments_cell(f, vk=(1.0, 2.0, 3.0)):
    """(rho, ux, uy, T) of one cell's 19 values."""
    f = _f64(f)
    out = np.zeros(4)
    lib().orc_moments_cell(_p(f), _p(_vk(vk)), _p(out))
    return out


def weno5(a, b, c, d, e, eps=1e-6):
    return lib().orc_weno5(float(a), float(b), float(c), float(d), float(e), float(eps))


def weno5_grad(a, b, c, d, e, eps=1e-6):
    g = np.zeros(5)
    lib().orc_weno5_grad(float(a), float(b), float(c), float(d), float(e), float(eps), _p(g))
    return g


def weno_periodic_line(F, sign=1, eps=1e-6):
    """Face fluxes h[I] at I+1/2 of a periodic line."""
    F = _f64(F)
    h = np.zeros_like(F)
    lib().orc_weno_periodic_line(_p(F), F.size, int(sign), float(eps), _p(h))
    return h


def scheme_periodic_line(F, sign=1, scheme=0, eps=1e-6):
    """Face fluxes h[I] at I+1/2 of a periodic line with scheme 0 (WENO5),
    1 (first-order upwind) or 2 (second-order upwind)."""
    F = _f64(F)
    h = np.zeros_like(F)
    lib().orc_scheme_periodic_line(_p(F), F.size, int(sign), int(scheme), float(eps), _p(h))
    return h


def init(params, rho, ux, uy, T):
    ny, nx = params.ny, params.nx
    f = np.zeros((NV, ny, nx))
    a = [_f64(x).reshape(ny, nx) for x in (rho, ux, uy, T)]
    _check(lib().orc_init(C.byref(params), *[_p(x) for x in a], _p(f)), "init")
    return f


def moments(params, f):
    ny, nx = params.ny, params.nx
    f = _f64(f)
    out = [np.zeros((ny, nx)) for _ in range(4)]
    _check(lib().orc_moments(C.byref(params), _p(f), *[_p(x) for x in out]), "moments")
    return tuple(out)


def state_check(params, f):
    """Classify the cells of f as the state check does: non-finite if one of
    its 19 values or its moments (Eq. (10)) is not finite, non-physical if all
    are finite but rho <= 0 or T <= 0. Returns (non-finite cells,
    non-physical cells, first non-finite cell index y*nx + x or -1, first
    non-physical cell or -1)."""
    f = _f64(f)
    with np.errstate(all="ignore"):
        rho, ux, uy, T = moments(params, f)
        fin = np.isfinite(f).all(axis=0)
        for q in (rho, ux, uy, T):
            fin &= np.isfinite(q)
        bad = ~fin
        unphys = fin & ~((rho > 0.0) & (T > 0.0))
    first = [int(np.flatnonzero(m.ravel())[0]) if m.any() else -1 for m in (bad, unphys)]
    return int(bad.sum()), int(unphys.sum()), first[0], first[1]


def step(params, f, nsteps=1, nthreads=1, contracted=False):
    """nsteps forward steps; contracted=True runs the FMA-contracted build."""
    f = _f64(f)
    out = np.zeros_like(f)
    L = lib_contracted() if contracted else lib()
    _check(L.orc_step(C.byref(params), _p(f), _p(out), int(nsteps), int(nthreads)), "step")
    return out


def kinetic_y(params, f):
    """(sum of rho uy^2/2 dx dy, max of rho uy^2/2)."""
    f = _f64(f)
    out = np.zeros(2)
    _check(lib().orc_kinetic_y(C.byref(params), _p(f), _p(out)), "kinetic_y")
    return out


def kinetic_y_grad(params, f):
    f = _f64(f)
    out = np.zeros_like(f)
    _check(lib().orc_kinetic_y_grad(C.byref(params), _p(f), _p(out)), "kinetic_y_grad")
    return out


def adjoint_step(params, f_n, lam_np1, w=0.0):
    f_n = _f64(f_n)
    lam_np1 = _f64(lam_np1)
    out = np.zeros_like(f_n)
    _check(lib().orc_adjoint_step(C.byref(params), _p(f_n), _p(lam_np1), float(w), _p(out)),
           "adjoint_step")
    return out


def init_vjp(params, rho, ux, uy, T, lam0):
    ny, nx = params.ny, params.nx
    a = [_f64(x).reshape(ny, nx) for x in (rho, ux, uy, T)]
    lam0 = _f64(lam0)
    out = [np.zeros((ny, nx)) for _ in range(4)]
    _check(lib().orc_init_vjp(C.byref(params), *[_p(x) for x in a], _p(lam0),
                              *[_p(x) for x in out]), "init_vjp")
    return tuple(out)
