"""Seeded synthetic inputs for the D2V19 FDLB step.

This module holds only workload recipes (initial macroscopic fields, seeded
draws, perturbation bases and their parameter tangents). It contains none of
the lattice-Boltzmann arithmetic and imports neither the GPU library nor the
CPU oracle, so both sides can be fed from it.

Fields are returned as float64 planes of shape (ny, nx), x fastest. Cell
centres are x_i = (i + 1/2) dx and, for the shear-layer runs,
y_j = (j + 1/2) dy - L_y / 2, so the interface lies between rows ny/2 - 1 and
ny/2.

The shear-layer profiles follow Sec. IV.A, Eqs. (59)-(61) of the paper
(tanh transition layers of widths D_v and D_rho at uniform pressure), turned
so that the interface normal is y, with a seeded transverse-velocity
perturbation in place of Eq. (62).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

PERIODIC, FIXED_EQ, REFLECT, OUTFLOW = 0, 1, 2, 3


@dataclass
class Setup:
    nx: int
    ny: int
    dx: float
    dy: float
    dt: float
    tau: float
    bc: tuple
    rho: np.ndarray
    ux: np.ndarray
    uy: np.ndarray
    T: np.ndarray
    side_state: tuple = (None, None, None, None)
    meta: dict = field(default_factory=dict)
    ke_axis: int = 0  # velocity component of the energy diagnostic: 0 u_y, 1 u_x
    scheme: int = 0   # convection flux: 0 WENO5, 1 first-order upwind, 2 second-order upwind

    def fields(self):
        return self.rho, self.ux, self.uy, self.T


# --------------------------------------------------------------------------
# Sod shock tube (Sec. III.B): left (rho, u, p) = (1, 0, 1), right
# (0.125, 0, 0.1), i.e. T = p / rho = 1 and 0.8; jump at x = 0.5; periodic
# in y; fixed-equilibrium ghosts in x (Eq. (57)).
# --------------------------------------------------------------------------
def sod(nx=400, ny=4, dx=2.5e-3, dy=2.5e-3, dt=1e-5, tau=2e-5, x0=0.5):
    x = (np.arange(nx) + 0.5) * dx
    left = x <= x0
    rho1 = np.where(left, 1.0, 0.125)
    T1 = np.where(left, 1.0, 0.8)
    rho = np.tile(rho1, (ny, 1))
    T = np.tile(T1, (ny, 1))
    z = np.zeros((ny, nx))
    sides = ((1.0, 0.0, 0.0, 1.0), (0.125, 0.0, 0.0, 0.8), None, None)
    return Setup(nx, ny, dx, dy, dt, tau, (FIXED_EQ, FIXED_EQ, PERIODIC, PERIODIC),
                 rho, z.copy(), z.copy(), T, sides,
                 {"workload": "sod", "left": (1.0, 0.0, 1.0), "right": (0.125, 0.0, 0.1), "x0": x0})


# --------------------------------------------------------------------------
# Shear layer (Kelvin-Helmholtz) runs
# --------------------------------------------------------------------------
def khi_coords(nx, ny, dx, dy):
    x = (np.arange(nx) + 0.5) * dx
    y = (np.arange(ny) + 0.5) * dy - 0.5 * ny * dy
    return x, y


def mode_basis(nx, dx):
    """Real Fourier basis on the nx cell centres: cos(2 pi m x / L) for
    m = 0 .. nx/2 - 1 followed by sin(2 pi m x / L) for m = 1 .. nx/2.
    Returns (A[nmodes, nx], labels). nx must be even."""
    if nx % 2:
        raise ValueError("mode basis needs an even nx")
    L = nx * dx
    x = (np.arange(nx) + 0.5) * dx
    rows, labels = [], []
    for m in range(nx // 2):
        rows.append(np.cos(2.0 * np.pi * m * x / L))
        labels.append(("cos", m))
    for m in range(1, nx // 2 + 1):
        rows.append(np.sin(2.0 * np.pi * m * x / L))
        labels.append(("sin", m))
    return np.array(rows), labels


def mode_amplitudes(nx, seed, base=1e-3):
    """Seeded amplitudes of the mode basis: the sin m=1 mode carries `base`
    (the single-mode perturbation), every other mode base * z / max(m, 1)
    with z ~ N(0, 1); none is zero."""
    _, labels = mode_basis(nx, 1.0)
    rng = np.random.default_rng(seed)
    z = rng.standard_normal(len(labels))
    a = np.empty(len(labels))
    for n, (kind, m) in enumerate(labels):
        a[n] = base if (kind == "sin" and m == 1) else base * z[n] / max(m, 1)
    a[a == 0.0] = base * 1e-3
    return a


def khi(nx=512, ny=512, dx=1e-3, dy=1e-3, dt=1e-5, tau=1e-5, Dv=0.02, Drho=0.02,
        rho1=5.0, rho2=2.0, u0=0.5, p0=2.5, amps=None, pert=1e-3, yw=0.02):
    """Shear layer periodic in x with reflecting walls in y.

    rho(y) = (rho1 + rho2)/2 - (rho1 - rho2)/2 tanh(y / Drho),
    ux(y)  = u0 tanh(y / Dv), uniform p0 so T = p0 / rho,
    uy     = g(y) * sum_m a_m phi_m(x) with g(y) = exp(-(y / yw)^2);
    without `amps` the perturbation is pert * sin(2 pi x / L_x) g(y).
    """
    x, y = khi_coords(nx, ny, dx, dy)
    rho1d = 0.5 * (rho1 + rho2) - 0.5 * (rho1 - rho2) * np.tanh(y / Drho)
    ux1d = u0 * np.tanh(y / Dv)
    gy = np.exp(-(y / yw) ** 2)
    if amps is None:
        px = pert * np.sin(2.0 * np.pi * x / (nx * dx))
    else:
        A, _ = mode_basis(nx, dx)
        px = np.asarray(amps, dtype=np.float64) @ A
    rho = np.repeat(rho1d[:, None], nx, axis=1)
    ux = np.repeat(ux1d[:, None], nx, axis=1)
    uy = gy[:, None] * px[None, :]
    T = p0 / rho
    return Setup(nx, ny, dx, dy, dt, tau, (PERIODIC, PERIODIC, REFLECT, REFLECT),
                 rho, ux, np.ascontiguousarray(uy), T, (None,) * 4,
                 {"workload": "khi", "Dv": Dv, "Drho": Drho, "rho1": rho1, "rho2": rho2,
                  "u0": u0, "p0": p0, "yw": yw})


def khi_paper(nx=600, ny=200, dx=1e-3, dy=1e-3, dt=1e-5, tau=1e-5, Dv=4e-3, Drho=8e-3,
              rhoL=5.0, rhoR=2.0, vL=0.5, vR=-0.5, p0=2.5, u0=0.02, k=10 * np.pi):
    """The paper's own shear layer (Sec. IV.A, Eqs. (59)-(62)): interface
    normal to x at x = 0 (x_i = (i + 1/2) dx - L_x / 2), flow along y,
    periodic in y, outflow sides in x (Eqs. (63)-(64)).

    rho(x) = (rhoL + rhoR)/2 - (rhoL - rhoR)/2 tanh(x / Drho),
    v(x)   = (vL + vR)/2 - (vL - vR)/2 tanh(x / Dv),     uniform p0 (T = p0 / rho),
    u      = u0 sin(k y) exp(-k |x|)    (Eq. (62) read with |x|: the printed
                                         exp(-k x) grows without bound for x < 0).
    The growth diagnostic is rho u_x^2 / 2 (ke_axis = 1). The paper's widths
    4, 8, ... are grid spacings: Dv = 4 dx by default."""
    x = (np.arange(nx) + 0.5) * dx - 0.5 * nx * dx
    y = (np.arange(ny) + 0.5) * dy
    rho1d = 0.5 * (rhoL + rhoR) - 0.5 * (rhoL - rhoR) * np.tanh(x / Drho)
    v1d = 0.5 * (vL + vR) - 0.5 * (vL - vR) * np.tanh(x / Dv)
    rho = np.tile(rho1d, (ny, 1))
    uy = np.tile(v1d, (ny, 1))
    ux = u0 * np.sin(k * y)[:, None] * np.exp(-k * np.abs(x))[None, :]
    T = p0 / rho
    return Setup(nx, ny, dx, dy, dt, tau, (OUTFLOW, OUTFLOW, PERIODIC, PERIODIC), rho, ux, uy, T,
                 meta=dict(Dv=Dv, Drho=Drho, rhoL=rhoL, rhoR=rhoR, vL=vL, vR=vR, p0=p0, u0=u0,
                           k=k), ke_axis=1)


def khi_tangents(nx, ny, dx, dy, Dv, Drho, rho1=5.0, rho2=2.0, u0=0.5, p0=2.5, yw=0.02):
    """Derivatives of the shear-layer initial fields with respect to the
    layer widths and the mode amplitudes, in separable form:

      d rho / d Drho = r(y),   d T / d Drho = t(y),   d ux / d Dv = v(y),
      d uy  / d a_m  = A[m, x] g(y).

    Returns dict(r, t, v, g, A) of 1-D profiles and the mode matrix."""
    x, y = khi_coords(nx, ny, dx, dy)
    sech2 = lambda s: 1.0 / np.cosh(s) ** 2  # noqa: E731
    rho1d = 0.5 * (rho1 + rho2) - 0.5 * (rho1 - rho2) * np.tanh(y / Drho)
    r = -0.5 * (rho1 - rho2) * sech2(y / Drho) * (-y / Drho ** 2)
    t = -p0 / rho1d ** 2 * r
    v = u0 * sech2(y / Dv) * (-y / Dv ** 2)
    g = np.exp(-(y / yw) ** 2)
    A, _ = mode_basis(nx, dx) if nx % 2 == 0 else (None, None)
    return {"r": r, "t": t, "v": v, "g": g, "A": A}


def batch_draw(seed, n=64, sizes=(128, 192, 256, 384, 512), dmin=0.005, dmax=0.08):
    """Seeded draw of n shear-layer instances: (nx, ny) drawn independently
    from `sizes`, D_v and D_rho log-uniform in [dmin, dmax]."""
    rng = np.random.default_rng(seed)
    nx = rng.choice(sizes, size=n)
    ny = rng.choice(sizes, size=n)
    lo, hi = np.log(dmin), np.log(dmax)
    Dv = np.exp(rng.uniform(lo, hi, size=n))
    Drho = np.exp(rng.uniform(lo, hi, size=n))
    return [dict(nx=int(a), ny=int(b), Dv=float(c), Drho=float(d))
            for a, b, c, d in zip(nx, ny, Dv, Drho)]


# --------------------------------------------------------------------------
# Generic seeded fields for parity and invariant tests
# --------------------------------------------------------------------------
def _smooth_noise(rng, nx, ny, nmodes=4):
    x = np.arange(nx) / nx
    y = np.arange(ny) / ny
    out = np.zeros((ny, nx))
    for _ in range(nmodes):
        kx, ky = rng.integers(0, 4, size=2)
        ph = rng.uniform(0, 2 * np.pi)
        out += rng.uniform(-1, 1) * np.cos(2 * np.pi * (kx * x[None, :] + ky * y[:, None]) + ph)
    return out / nmodes


def random_fields(nx, ny, seed, rho=(0.5, 2.0), u=0.3, T=(0.5, 1.2), smooth=True):
    """Seeded (rho, ux, uy, T) planes, smooth (periodic) or white noise."""
    rng = np.random.default_rng(seed)
    if smooth:
        n = [_smooth_noise(rng, nx, ny) for _ in range(4)]
        s = [0.5 * (v + 1.0) for v in n]  # in [0, 1]
    else:
        s = [rng.uniform(0.0, 1.0, size=(ny, nx)) for _ in range(4)]
    r = rho[0] + (rho[1] - rho[0]) * s[0]
    ux = u * (2.0 * s[1] - 1.0)
    uy = u * (2.0 * s[2] - 1.0)
    Tt = T[0] + (T[1] - T[0]) * s[3]
    return r, ux, uy, Tt


# Arbitrary positive base populations (not the model's weights): used to
# build non-equilibrium distributions directly, independent of any f^eq.
_BASE = np.array([0.30] + [0.05] * 6 + [0.04] * 6 + [0.01] * 6)


def random_f(nx, ny, seed, amp=0.2, smooth=False):
    """Seeded positive 19-plane distribution, far from equilibrium."""
    rng = np.random.default_rng(seed)
    f = np.empty((19, ny, nx))
    for i in range(19):
        noise = _smooth_noise(rng, nx, ny) if smooth else rng.uniform(-1.0, 1.0, (ny, nx))
        f[i] = _BASE[i] * (1.0 + amp * noise)
    return f


def random_like(shape, seed, scale=1.0):
    """Seeded N(0, scale^2) array (adjoint seeds, perturbation directions)."""
    return scale * np.random.default_rng(seed).standard_normal(shape)
