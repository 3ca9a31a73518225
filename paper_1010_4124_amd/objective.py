"""Differentiable shear-layer objective on top of the C-ABI.

J(D_v, D_rho, a) = dt * sum_{n=n0}^{n1} E_y(f^n),   E_y = sum_cells rho u_y^2 / 2 dx dy,

where f^0 = f^eq of the shear-layer initial fields (tanh layers of widths D_v
and D_rho, uniform pressure, transverse velocity sum_m a_m phi_m(x) g(y)) and
f^{n+1} is one forward-Euler FDLB step of f^n. E_y is the transverse kinetic
energy whose linear-phase growth measures the Kelvin-Helmholtz growth rate
(the paper's Sec. IV diagnostic with the interface normal along y).

The gradient is the discrete adjoint: lambda^N = w_N dE_y/df^N, then
lambda^n = (dS/df^n)^T lambda^{n+1} + w_n dE_y/df^n (lbm_adjoint_step),
lambda^0 -> dJ/d(rho, ux, uy, T) (lbm_init_vjp) -> dJ/dparameters through the
separable tangents of the initial fields (lbm_sep_project). States are
recomputed from checkpoints: every K1 steps (level 1), and inside a level-1
segment every K2 steps (level 2); only the K2 states of the sub-segment being
reversed are held at once. Every arithmetic step runs in the HIP library;
this module orchestrates calls and owns device buffers.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

from . import inputs, lbm


@dataclass
class Schedule:
    """Checkpoint schedule: level-1 interval K1, level-2 interval K2 (K2 <= K1)."""
    K1: int
    K2: int

    @classmethod
    def every(cls, K):
        return cls(int(K), int(K))

    @classmethod
    def sqrt(cls, nsteps):
        """Two-level schedule with about N^(1/3) states per level."""
        K2 = max(1, int(round(nsteps ** (1.0 / 3.0))))
        K1 = max(K2, int(round(nsteps ** (2.0 / 3.0))))
        K1 = K2 * max(1, K1 // K2)
        return cls(K1, K2)

    def peak_states(self, nsteps, overlap=False):
        """Live 19-plane states of a gradient: level-1 and level-2
        checkpoints, one piece's states, lambda and its partner; the
        overlapped gradient adds one more piece and one more set of level-2
        checkpoints. (With a fast-tile step variant each piece state also
        keeps its 4 moment-sum planes.)"""
        seq = math.ceil(nsteps / self.K1) + math.ceil(self.K1 / self.K2) + self.K2 + 2
        return seq + (math.ceil(self.K1 / self.K2) + self.K2 if overlap else 0)


class KHIProblem:
    """A shear-layer run: grid, physics, step count and objective window."""

    def __init__(self, nx, ny, dx=1e-3, dy=1e-3, dt=1e-5, tau=1e-5, nsteps=4000, window=(2000, 4000),
                 rho1=5.0, rho2=2.0, u0=0.5, p0=2.5, yw=0.02, schedule=None, variant=None):
        self.nx, self.ny, self.dx, self.dy, self.dt, self.tau = nx, ny, dx, dy, dt, tau
        self.nsteps = int(nsteps)
        self.n0, self.n1 = int(window[0]), int(window[1])
        if not (0 <= self.n0 <= self.n1 <= self.nsteps):
            raise ValueError("window must satisfy 0 <= n0 <= n1 <= nsteps")
        self.phys = dict(rho1=rho1, rho2=rho2, u0=u0, p0=p0, yw=yw)
        self.schedule = schedule or Schedule.every(min(200, max(1, self.nsteps)))
        self.bc = (inputs.PERIODIC, inputs.PERIODIC, inputs.REFLECT, inputs.REFLECT)
        self.ctx = lbm.Context(nx, ny, dx, dy, dt, tau, self.bc)
        self._ctx2 = None  # the recompute context of the overlapped gradient
        if variant is not None:
            self.ctx.variant = variant

    def weight(self, n):
        return self.dt if self.n0 <= n <= self.n1 else 0.0

    def fields(self, Dv, Drho, amps):
        return inputs.khi(self.nx, self.ny, self.dx, self.dy, self.dt, self.tau, Dv=float(Dv),
                          Drho=float(Drho), amps=np.asarray(amps, dtype=np.float64), **self.phys)

    # -- forward ---------------------------------------------------------------
    def run(self, Dv, Drho, amps, keep_checkpoints=True):
        """J and the level-1 checkpoints {n: f^n}."""
        s = self.fields(Dv, Drho, amps)
        ctx = self.ctx
        f = ctx.init(*s.fields())
        K1 = self.schedule.K1
        ck = {}
        J = 0.0
        n = 0
        buf = ctx.empty_f()
        while n < self.nsteps:
            if keep_checkpoints and n % K1 == 0:
                ck[n] = f.clone()
            m = min(K1 - n % K1, self.nsteps - n)
            f_next, ke = ctx.step(f, m, out=buf, ke_log=True)
            ke = ke[:, 0].cpu().numpy()
            for q in range(m):
                J += self.weight(n + q) * ke[q]
            buf, f = f, f_next
            n += m
        J += self.weight(self.nsteps) * float(ctx.kinetic_y(f)[0])
        return J, ck

    # -- backward --------------------------------------------------------------
    def _units(self, ck):
        """The reverse sweep's work units in the order it takes them:
        (c0, c1, s0, s1) = level-1 segment [c0, c1) and its level-2 piece
        [s0, s1), last first."""
        N, K1, K2 = self.nsteps, self.schedule.K1, self.schedule.K2
        out = []
        for c0 in sorted(ck, reverse=True):
            c1 = min(c0 + K1, N)
            for s0 in reversed(range(c0, c1, K2)):
                out.append((c0, c1, s0, min(s0 + K2, c1)))
        return out

    def _recompute(self, ctx, ck, units):
        """States f^s0 .. f^(s1-1) of each unit in turn, recomputed from the
        level-1 checkpoints (and, per level-1 segment, its level-2
        checkpoints every K2 steps) on ctx, with their moment sums when the
        step variant is a fast-tile one (mode 3): its single steps then carry
        the sums from step to step instead of forming them from f each call,
        and the reverse steps read them instead of f's 19 planes a second
        time (the sums are lbm_sums's bit for bit, so the gradient is the
        same either way). Yields (states, sums or None)."""
        K2 = self.schedule.K2
        seg, sub = None, {}
        for c0, c1, s0, s1 in units:
            if c0 != seg:
                seg, f, sub = c0, ck[c0], {c0: ck[c0]}
                for n in range(c0 + K2, c1, K2):
                    f = ctx.step(f, K2)
                    sub[n] = f
            states = [sub.pop(s0)]
            if lbm.lbm_step_variant_info(ctx.variant)[5] == 3:
                sums = [ctx.sums(states[0])]
                for _ in range(s0 + 1, s1):
                    f, m = ctx.step_sums(states[-1], sums[-1])
                    states.append(f)
                    sums.append(m)
            else:
                sums = None
                for _ in range(s0 + 1, s1):
                    states.append(ctx.step(states[-1], 1))
            yield states, sums

    # grids from this many cells on fill the GPU alone: no overlapped recompute
    OVERLAP_MAX_CELLS = 1 << 20

    def gradient(self, Dv, Drho, amps, ck=None, scale=1.0, overlap=None):
        """(dJ/dD_v, dJ/dD_rho, dJ/da) by the discrete adjoint.

        overlap: recompute the next unit's states on a second context and
        stream while the current unit's reverse steps run (the two are
        independent), so that grids too small to fill the GPU alone share it;
        at most one more unit's states and one more segment's level-2
        checkpoints are alive. The result is the same bit for bit. None (the
        default): overlap below OVERLAP_MAX_CELLS cells only. On larger grids
        the overlap gains little, and the states it frees on one stream after
        use on the other are not reused by torch's caching allocator soon
        enough: at 2048^2 x 4000 steps it reserved 250 GB for 45 GB in use,
        and a 40000-step gradient ran out of room and slowed down."""
        if overlap is None:
            overlap = self.nx * self.ny < self.OVERLAP_MAX_CELLS
        if ck is None:
            _, ck = self.run(Dv, Drho, amps)
        ctx = self.ctx
        N = self.nsteps
        zero = torch.zeros((19, self.ny, self.nx), dtype=torch.float64, device=ctx.device)
        # lambda^N = w_N dE_y/df^N: the adjoint step with a zero seed
        fN = self._advance(ck[max(ck)], max(ck), N)
        lam = ctx.adjoint_step(fN, zero, scale * self.weight(N))
        del fN
        lam_next = ctx.empty_f()
        units = self._units(ck)

        def reverse(unit, states, sums):
            _, _, s0, s1 = unit
            nonlocal lam, lam_next
            for n in range(s1 - 1, s0 - 1, -1):
                ctx.adjoint_step(states[n - s0], lam, scale * self.weight(n), out=lam_next,
                                 sums=None if sums is None else sums[n - s0])
                lam, lam_next = lam_next, lam

        if not overlap:
            for unit, (states, sums) in zip(units, self._recompute(ctx, ck, units)):
                reverse(unit, states, sums)
                del states, sums
        else:
            main = torch.cuda.current_stream()
            side = torch.cuda.Stream()  # default priority
            if self._ctx2 is None:
                self._ctx2 = lbm.Context(self.nx, self.ny, self.dx, self.dy, self.dt, self.tau,
                                         self.bc)
            self._ctx2.variant = ctx.variant
            side.wait_stream(main)  # the checkpoints are complete
            for f in ck.values():
                f.record_stream(side)
            gen = self._recompute(self._ctx2, ck, units)

            def produce():
                with torch.cuda.stream(side):
                    states = next(gen, None)
                    done = torch.cuda.Event()
                    done.record(side)
                return states, done

            ahead = produce()
            for i, unit in enumerate(units):
                ((states, sums), done), ahead = ahead, None
                if i + 1 < len(units):
                    ahead = produce()  # queued on the side stream before this unit's reverse steps
                main.wait_event(done)
                for t in states + (sums or []):
                    t.record_stream(main)
                reverse(unit, states, sums)
                del states, sums
            main.wait_stream(side)
        s = self.fields(Dv, Drho, amps)
        g_rho, g_ux, g_uy, g_T = ctx.init_vjp(*s.fields(), lam)
        t = inputs.khi_tangents(self.nx, self.ny, self.dx, self.dy, float(Dv), float(Drho),
                                **{k: self.phys[k] for k in ("rho1", "rho2", "u0", "p0", "yw")})
        ones = np.ones((1, self.nx))
        dDv = ctx.sep_project(g_ux, ones, t["v"])[0]
        dDrho = ctx.sep_project(g_rho, ones, t["r"])[0] + ctx.sep_project(g_T, ones, t["t"])[0]
        da = ctx.sep_project(g_uy, t["A"], t["g"])
        return float(dDv), float(dDrho), da.cpu().numpy()

    def _advance(self, f, n_from, n_to):
        return f if n_to == n_from else self.ctx.step(f, n_to - n_from)


class KHIObjective(torch.autograd.Function):
    """J = KHIObjective.apply(D_v, D_rho, amps, problem): differentiable in the
    two layer widths (0-d tensors) and the mode amplitudes (1-d tensor)."""

    @staticmethod
    def forward(fctx, Dv, Drho, amps, problem):
        vals = (float(Dv), float(Drho), amps.detach().cpu().numpy())
        J, ck = problem.run(*vals)
        fctx.problem, fctx.vals, fctx.ck = problem, vals, ck
        return torch.tensor(J, dtype=torch.float64)

    @staticmethod
    def backward(fctx, gJ):
        gDv, gDrho, ga = fctx.problem.gradient(*fctx.vals, ck=fctx.ck, scale=float(gJ))
        fctx.ck = None
        return (torch.tensor(gDv, dtype=torch.float64), torch.tensor(gDrho, dtype=torch.float64),
                torch.from_numpy(ga), None)
