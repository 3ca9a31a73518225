// lbm_fast.h -- one forward-Euler D2V19 FDLB step (Eq. (47) of
// arXiv:1010.4124) of a fast tile with carried moment sums: the device body
// of the M = 3 step variants.
//
// A fast tile (fast_tile in lbm_stage.h) has its rows and its 3-cell halo
// inside the grid, or its halo columns one period away around a periodic x
// axis, so its staging needs no boundary logic. One wavefront advances one
// 64 x R tile through all 18 moving velocities, as the M = 1 kernel does,
// and evaluates the same expressions in the same order (its results are
// those of the M = 1 variant with the same R, W, D, NT, bit for bit); what
// differs is the schedule of a plane:
//   - the lane holds its own column of the staged rows in registers (one row
//     load per row), so the y pass runs from those registers, before the x
//     pass and while the staged image is written to LDS; the x pass is the
//     only LDS round trip left;
//   - the direction of each velocity of a speed shell is a compile-time
//     constant, so each plane's code has its upwind orientation and y-flux
//     presence fixed, with no branch on the sign of v;
//   - the plane index is made opaque to loop strength reduction
//     (readfirstlane), which otherwise keeps one set of output and input
//     pointers per direction alive across the shell loop and spills them.
// The tiles that are not fast, in bands around the rectangle of fast tiles,
// take the M = 1 tile body in the same launch.
#pragma once

#include <type_traits>

#include "lbm_device.h"
#include "lbm_stage.h"
#include "lbm_step.h"

namespace lbmd {

template <int R>
struct FastStage {
    static constexpr int ROWS = R + 2 * HALO;  // staged rows per lane
    static constexpr int NPRE = ROWS + 1;      // + one halo-column value
    static constexpr int PAD = ROWS * PITCH;
    static constexpr int NPAD = 64 - 2 * HALO * R > 0 ? 64 - 2 * HALO * R : 1;
    static constexpr int SLOTS = PAD + NPAD;
    static constexpr int LDS = SLOTS + R * XPITCH;  // staged image + x flux differences
};

// Step of fast tile `tile` (row-major index): carried sums in m_in, out,
// energy partials of the tile into ke_dst (if not null). D planes are in
// flight ahead of the one being computed (1 or 2). With own_sums the tile
// forms the moment sums of its cells from f itself (m_in is not read), with
// the expressions and order of the sums pass (k_sums), so its results are
// the same bit for bit.
template <int R, int D, bool NT>
__device__ __forceinline__ void fast_tile_work(const StepGrid& a, const Consts& k, int tile,
                                               double* ke_dst, double* lds,
                                               const double* __restrict__ m_in,
                                               double* __restrict__ m_out, bool own_sums = false)
{
    using S = FastStage<R>;
    static_assert(D == 1 || D == 2, "one or two planes in flight");
    const int lane = threadIdx.x & 63;
    const int ty = tile / a.tiles_x, tx = tile - ty * a.tiles_x;
    const int x0 = tx * TX, y0 = ty * R;
    const int nx = a.nx;
    const int64_t plane = (int64_t)nx * a.ny;
    const int gx = x0 + lane;
    double* s_pl = lds;
    double* s_dx = lds + S::SLOTS;
    // halo lanes: the 3 columns on each side of the R centre rows; the value
    // is taken one period away around a periodic x axis (fast_tile)
    const bool hl = lane < 2 * HALO * R;
    const int hr = hl ? lane / (2 * HALO) : 0, hc = lane - 2 * HALO * (lane / (2 * HALO));
    const int hlx = hl ? (hc < HALO ? hc - HALO : hc + 64 - HALO) : 0;
    const int hoff = hr * nx + wrap_once(x0 + hlx, nx);
    const int hslot = hl ? (hr + HALO) * PITCH + hlx + HALO : S::PAD + (lane - 2 * HALO * R);

    // the rows of plane i at the lane's column that its faces use, and its
    // halo value. p[r] is row y0 - 3 + r. The upwind stencils of the R cells
    // reach rows y0-3 .. y0+R+1 when v_y > 0 and y0-2 .. y0+R+2 when
    // v_y < 0 (SY, the sign of v_y); with v_y = 0 there are no y faces, and
    // the x pass reads the R centre rows only
    auto load = [&](auto sy, int i_in, double(&p)[S::NPRE]) {
        constexpr int SY = decltype(sy)::value;
        constexpr int R0 = SY > 0 ? 0 : SY < 0 ? 1 : HALO;
        constexpr int R1 = SY > 0 ? S::ROWS - 1 : SY < 0 ? S::ROWS : HALO + R;
        const int i = __builtin_amdgcn_readfirstlane(i_in);
        const double* base = a.fin + i * plane + (int64_t)(y0 - HALO) * nx + x0;
        // a raised wave priority while the plane's loads are issued, so that
        // they are not held back behind the other waves' arithmetic
        __builtin_amdgcn_s_setprio(1);
        p[S::ROWS] = (a.fin + i * plane + (int64_t)y0 * nx)[(unsigned)hoff];
#pragma unroll
        for (int r = R0; r < R1; ++r) p[r] = (base + (int64_t)r * nx)[(unsigned)lane];
        __builtin_amdgcn_s_setprio(0);
    };
    // the sign of v_y of direction d, as a type
    auto yrows = [](auto dc) {
        return std::integral_constant<int, dir_sin_sign(decltype(dc)::value)>{};
    };

    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using I3 = std::integral_constant<int, 3>;
    using I4 = std::integral_constant<int, 4>;
    using I5 = std::integral_constant<int, 5>;
    // ---- phase 1: cell state from the carried sums; rest particle; energy
    // The carried sums and the rest particle are read by this tile only:
    // non-temporal loads keep them from displacing halo rows in L2. The
    // first plane(s) are requested right after them, so that their latency
    // overlaps phase 1's.
    double ms[5][R];
    if (own_sums) {
#pragma unroll
        for (int m = 0; m < R; ++m) ms[0][m] = ms[1][m] = ms[2][m] = ms[3][m] = 0.0;
#pragma unroll
        for (int i = 0; i < NV; ++i) {
#pragma unroll
            for (int m = 0; m < R; ++m) {
                const double fi = a.fin[i * plane + (int64_t)(y0 + m) * nx + gx];
                if (i == 0) ms[4][m] = fi;
                ms[0][m] += fi;
                ms[1][m] = __builtin_fma(fi, k.vx[i], ms[1][m]);
                ms[2][m] = __builtin_fma(fi, k.vy[i], ms[2][m]);
                ms[3][m] = __builtin_fma(fi, k.hv2[i], ms[3][m]);
            }
        }
    } else {
#pragma unroll
        for (int m = 0; m < R; ++m) {
            const int64_t c = (int64_t)(y0 + m) * nx + gx;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                ms[q][m] = __builtin_nontemporal_load(&m_in[q * plane + c]);
            ms[4][m] = __builtin_nontemporal_load(&a.fin[c]);
        }
    }
    double pa[S::NPRE], pb[S::NPRE];
    load(yrows(I0{}), 1, pa);
    if constexpr (D == 2) load(yrows(I1{}), 2, pb);

    double rho[R], Tm[R], uxt[R], uyt[R];  // rho[] holds dt/tau rho
    // 1 - |u|^2/2T of each cell, and (dt/tau) rho F_k(T) of the shell being
    // advanced: the same expressions the M = 1 kernel evaluates per plane,
    // evaluated once per cell and once per cell and shell
    double t0c[R], Ash[R];
    Sums<R> acc;
    double ke_s = 0.0, ke_m = 0.0;
#pragma unroll
    for (int m = 0; m < R; ++m) {
        const double r = ms[0][m], jx = ms[1][m], jy = ms[2][m], E = ms[3][m], f0 = ms[4][m];
        const CellEq q = cell_eq_from_sums(r, jx, jy, E);
        rho[m] = a.ct * q.rho;
        Tm[m] = q.T;
        uxt[m] = q.uxt;
        uyt[m] = q.uyt;
        t0c[m] = __builtin_fma(-0.5 * q.T, __builtin_fma(q.uxt, q.uxt, q.uyt * q.uyt), 1.0);
        const double un = (a.ke_axis ? jx : jy) / r;
        const double e = 0.5 * r * un * un;
        ke_s += e;
        ke_m = fmax(ke_m, e);
        // rest particle: no convection, f^eq_0 = rho F_0 (1 - u^2/2T)
        const double F0 =
            1.0 - 6.0 * (weight_c(k, 0, q.T) + weight_c(k, 1, q.T) + weight_c(k, 2, q.T));
        const double fe = q.rho * F0 * q.t0;
        const double fn = __builtin_fma(-a.ct, f0 - fe, f0);
        (a.fout + (int64_t)(y0 + m) * nx + x0)[(unsigned)lane] = fn;
        acc.r[m] = fn;  // v_0 = 0: the rest particle adds to rho only
        acc.jx[m] = acc.jy[m] = acc.E[m] = 0.0;
    }
    if (ke_dst) {
        ke_s = wave_sum(ke_s);
        ke_m = wave_max(ke_m);
        if (lane == 0) {
            ke_dst[0] = ke_s;
            ke_dst[1] = ke_m;
        }
    }
    const double omct = 1.0 - a.ct;

    // plane of direction d (compile time) in shell s (run time), staged rows
    // in p; with D = 1, p is refilled with plane `next` once its rows are
    // staged and copied for the y pass
    auto do_plane = [&](auto dc, int s, double(&p)[S::NPRE], int next) {
        constexpr int d = decltype(dc)::value;
        constexpr bool NEGX = dir_cos(d) < 0.0;
        constexpr int SY = dir_sin_sign(d);
        __builtin_amdgcn_sched_barrier(0);
        const int i = __builtin_amdgcn_readfirstlane(1 + 6 * s + d);
        const double vx = k.vx[i], vy = k.vy[i];
        const double cxv = a.cx * vx, cyv = a.cy * vy;
        // the staged image for the x pass (its R centre rows are all it reads)
#pragma unroll
        for (int r = HALO; r < HALO + R; ++r) s_pl[r * PITCH + lane + HALO] = p[r];
        s_pl[hslot] = p[S::ROWS];
        // y pass from the registers (y_pass's samples, in the same order)
        double dhy[R], fc[R];
#pragma unroll
        for (int m = 0; m < R; ++m) {
            fc[m] = p[m + HALO];
            dhy[m] = 0.0;
        }
        // the y pass works on a copy of the rows, so that the next plane's
        // loads (D = 1) are issued into p before it rather than after it
        double P[SY != 0 ? R + 5 : 1];
        if constexpr (SY != 0) {
#pragma unroll
            for (int j = 0; j < R + 5; ++j) P[j] = SY < 0 ? p[R + 5 - j] : p[j];
        }
        if constexpr (D == 1) {
            // after the last plane of the last shell there is nothing to load
            if (d < 5 || next < NV) load(yrows(std::integral_constant<int, (d + 1) % 6>{}), next, p);
        }
        if constexpr (SY != 0)
            weno_strip<R, (SY < 0)>(P, k.epsy[i], [&](int m, double dd) { dhy[m] = dd; });
        __syncthreads();
        x_pass<R, NEGX>(s_pl, s_dx, lane, k.epsx[i]);
        __syncthreads();
        // f' = (1 - ct) f + (ct rho F_k) poly(eta) - cx dh^x - cy dh^y, as
        // the M = 1 kernel evaluates it
        double* base = a.fout + i * plane + (int64_t)y0 * nx + x0;
        const double hv = k.hv2[i];
#pragma unroll
        for (int m = 0; m < R; ++m) {
            const double dhx = s_dx[m * XPITCH + lane];
            const double eta = __builtin_fma(vx, uxt[m], vy * uyt[m]);
            double fn = __builtin_fma(omct, fc[m], Ash[m] * feq_poly(eta, t0c[m]));
            fn = __builtin_fma(-cxv, dhx, fn);
            fn = __builtin_fma(-cyv, dhy[m], fn);
            acc.r[m] += fn;
            acc.jx[m] = __builtin_fma(fn, vx, acc.jx[m]);
            acc.jy[m] = __builtin_fma(fn, vy, acc.jy[m]);
            acc.E[m] = __builtin_fma(fn, hv, acc.E[m]);
            double* dst = base + (int64_t)m * nx;
            if (NT)
                __builtin_nontemporal_store(fn, &dst[(unsigned)lane]);
            else
                dst[(unsigned)lane] = fn;
        }
        __builtin_amdgcn_sched_barrier(0);
    };

    // ---- phase 2: the 18 moving velocities, shell by shell
#pragma unroll 1
    for (int s = 0; s < 3; ++s) {
        const int b1 = 1 + 6 * s;
#pragma unroll
        for (int m = 0; m < R; ++m) Ash[m] = rho[m] * weight_c(k, s, Tm[m]);
        if constexpr (D == 1) {
            do_plane(I0{}, s, pa, b1 + 1);
            do_plane(I1{}, s, pa, b1 + 2);
            do_plane(I2{}, s, pa, b1 + 3);
            do_plane(I3{}, s, pa, b1 + 4);
            do_plane(I4{}, s, pa, b1 + 5);
            do_plane(I5{}, s, pa, b1 + 6);
        } else {
            do_plane(I0{}, s, pa, 0);
            load(yrows(I2{}), b1 + 2, pa);
            do_plane(I1{}, s, pb, 0);
            load(yrows(I3{}), b1 + 3, pb);
            do_plane(I2{}, s, pa, 0);
            load(yrows(I4{}), b1 + 4, pa);
            do_plane(I3{}, s, pb, 0);
            load(yrows(I5{}), b1 + 5, pb);
            do_plane(I4{}, s, pa, 0);
            // the next shell's first two planes (past the last shell: plane
            // 18 again, unused)
            load(yrows(I0{}), min(b1 + 6, NV - 1), pa);
            do_plane(I5{}, s, pb, 0);
            load(yrows(I1{}), min(b1 + 7, NV - 1), pb);
        }
    }

    // ---- phase 3: the moment sums of f^{n+1} for the next step
#pragma unroll
    for (int m = 0; m < R; ++m) {
        const int64_t c = (int64_t)(y0 + m) * nx + gx;
        m_out[c] = acc.r[m];
        m_out[plane + c] = acc.jx[m];
        m_out[2 * plane + c] = acc.jy[m];
        m_out[3 * plane + c] = acc.E[m];
    }
}

// Rectangle of fast tiles of a grid with 64 x R tiles: tile columns
// [c0, c1) and tile rows [r0, r1), the tiles for which fast_tile holds
// (its x and y conditions are independent). Empty: c0 = c1 = 0 and
// r0 = r1 = tiles_y.
struct FastRect {
    int c0, c1, r0, r1;
};

__host__ __device__ inline FastRect fast_rect(int nx, int ny, int bc_xlo, int R)
{
    FastRect f;
    const int tiles_y = (ny + R - 1) / R;
    if (bc_xlo == PERIODIC) {
        f.c0 = 0;
        f.c1 = nx >= HALO ? nx / TX : 0;
    } else {
        // x0 = 64 c >= 3 and 64 c + 64 + 3 <= nx
        f.c0 = 1;
        f.c1 = nx >= TX + HALO ? (nx - TX - HALO) / TX + 1 : 0;
    }
    // y0 = R t >= 3 and R t + R + 3 <= ny
    f.r0 = (HALO + R - 1) / R;
    f.r1 = ny >= R + HALO ? (ny - R - HALO) / R + 1 : 0;
    if (f.c1 <= f.c0 || f.r1 <= f.r0) {
        f.c0 = f.c1 = 0;
        f.r0 = f.r1 = tiles_y;
    }
    return f;
}

// Tile (row-major index) of work item w of the bands around a FastRect:
// the rows above it, the rows below it, then row by row the columns to its
// left and right. band_count gives the number of work items.
__host__ __device__ inline int band_count(const FastRect& f, int tiles_x, int tiles_y)
{
    return f.r0 * tiles_x + (tiles_y - f.r1) * tiles_x +
           (f.r1 - f.r0) * (f.c0 + tiles_x - f.c1);
}

__device__ __forceinline__ int band_tile(int w, const FastRect& f, int tiles_x, int tiles_y)
{
    const int top = f.r0 * tiles_x;
    if (w < top) return w;
    w -= top;
    const int bot = (tiles_y - f.r1) * tiles_x;
    if (w < bot) return f.r1 * tiles_x + w;
    w -= bot;
    const int lw = f.c0, per = max(1, f.c0 + tiles_x - f.c1);
    const int r = w / per, c = w - r * per;
    return (f.r0 + r) * tiles_x + (c < lw ? c : f.c1 + (c - lw));
}

}  // namespace lbmd
