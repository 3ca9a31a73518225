// lbm_step.h -- body of one forward-Euler D2V19 FDLB step (Eq. (47) of
// arXiv:1010.4124) for one 64 x R tile, shared by the single-grid kernel
// (lbm_forward.hip) and the batched kernel (lbm_batch.hip).
//
// A work item is one tile and one of G groups of the 18 moving velocities;
// each lane owns a column strip of R cells.
//
//   phase 1  every lane loads the 19 values of its R cells, forms the moments
//            of Eq. (10) and keeps u/T, 1-u^2/2T and rho F_k(T) in
//            registers. Group 0 also relaxes and stores the rest particle and
//            reduces the tile's transverse kinetic energy.
//   phase 2  for each velocity i of the group:
//            - plane f_i of the tile plus a 3-cell cross-shaped halo (ghosts
//              from the boundary rule) is staged in LDS; the next plane is
//              already in flight into registers (software pipeline);
//            - x pass: lanes re-map to row strips of R cells and compute the
//              R+1 WENO faces of their strip once, sharing first and second
//              differences between faces; flux differences go to LDS;
//            - y pass (v_iy != 0): lanes compute the R+1 faces of their column
//              strip in registers;
//            - each lane combines convection, BGK relaxation toward f^eq and
//              the Euler update and stores f_i^{n+1} (coalesced along x).
//
// A tile's G work items repeat phase 1 (the 19 centre values come from L2);
// G > 1 multiplies the number of workgroups on small grids.
#pragma once

#include "lbm_device.h"
#include "lbm_stage.h"

namespace lbmd {

constexpr int TX = 64;
constexpr int PITCH = 71;   // LDS row pitch of a staged plane (odd: no bank conflicts)
constexpr int XPITCH = 65;  // LDS row pitch of the x flux differences

template <int R>
using Stage = StageG<R, HALO, PITCH>;

// One grid as seen by a step: states, shape, boundary rules and the ratios
// dt/dx, dt/dy, dt/tau.
struct StepGrid {
    const double* __restrict__ fin;
    double* __restrict__ fout;
    int nx, ny;
    int bc[4];
    int tiles_x;
    double cx, cy, ct;
};

__device__ __forceinline__ GridBC grid_bc(const StepGrid& s)
{
    return GridBC{s.nx, s.ny, {s.bc[0], s.bc[1], s.bc[2], s.bc[3]}};
}

// x pass: lane -> (row r = lane % R, strip s = lane / R); the flux
// differences go to s_dx.
template <int R, bool NEG>
__device__ __forceinline__ void x_pass(const double* s_pl, double* s_dx, int lane, double v,
                                       double eps)
{
    const int r = lane % R, s = lane / R;
    const double* b = s_pl + (r + HALO) * PITCH + s * R;
    double P[R + 5];
#pragma unroll
    for (int k = 0; k < R + 5; ++k) P[k] = v * (NEG ? b[R + 5 - k] : b[k]);
    double* out = s_dx + r * XPITCH + s * R;
    weno_strip<R, NEG>(P, eps, [&](int m, double d) { out[m] = d; });
}

// y pass: lane = column; calls upd(m, f_m, dh^y_m) for each cell of the strip
// as soon as its two faces are known.
template <int R, bool NEG, class Upd>
__device__ __forceinline__ void y_pass(const double* s_pl, int lane, double v, double eps, Upd&& upd)
{
    const double* col = s_pl + lane + HALO;
    double P[R + 5];
#pragma unroll
    for (int k = 0; k < R + 5; ++k) P[k] = v * (NEG ? col[(R + 5 - k) * PITCH] : col[k * PITCH]);
    // the centre value of cell m is re-read from LDS when the cell completes
    weno_strip<R, NEG>(P, eps, [&](int m, double d) { upd(m, col[(m + HALO) * PITCH], d); });
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Phase 2 of one tile: this group's moving velocities. Instantiated once for
// interior tiles and once for boundary tiles, so that each loop is straight
// line code and the compiler tracks its outstanding loads and stores exactly.
// DEPTH planes are in flight ahead of the one being computed; every load is
// issued unconditionally (past the group's last plane the last plane is
// re-read) and consumed after the current plane's stores, so waiting for a
// staged plane never waits for stores.
template <int R, int G, bool BND, int DEPTH, bool NT, class SE>
__device__ __forceinline__ void plane_loop(const StepGrid& a, const Consts& k, SE se,
                                           int grp, int x0, int y0, int lane, const TileMapG& t,
                                           int64_t plane, double* s_pl, double* s_dx,
                                           const double (&rho)[R], const double (&Tm)[R],
                                           const double (&uxt)[R], const double (&uyt)[R],
                                           const double (&t0)[R])
{
    constexpr int NPL = 18 / G;  // moving velocities per group
    static_assert(DEPTH == 1 || NPL % 2 == 0, "two-deep pipeline needs an even plane count");
    const int gx = x0 + lane;
    const int i0 = 1 + grp * NPL, iend = i0 + NPL;
    double A[R];  // (dt/tau) rho F_k(T) of the current speed shell
    int kcur = -1;
    const double omct = 1.0 - a.ct;
    const GridBC g = grid_bc(a);

    // f' = f - cx dh^x - cy dh^y - ct (f - f^eq)
    //    = (1 - ct) f + (ct rho F_k) poly(eta) - cx dh^x - cy dh^y
    auto compute = [&](int i) {
        const int ks = (i - 1) / 6;
        if (ks != kcur) {
            kcur = ks;
#pragma unroll
            for (int m = 0; m < R; ++m) A[m] = (a.ct * rho[m]) * weight_c(k, ks, Tm[m]);
        }
        const double vx = k.vx[i], vy = k.vy[i], eps = k.eps;
        if (vx < 0.0)
            x_pass<R, true>(s_pl, s_dx, lane, vx, eps);
        else
            x_pass<R, false>(s_pl, s_dx, lane, vx, eps);
        __syncthreads();
        double* base = a.fout + i * plane + (int64_t)y0 * a.nx + x0;
        auto upd = [&](int m, double fcm, double dhy) {
            const double dhx = s_dx[m * XPITCH + lane];
            const double eta = __builtin_fma(vx, uxt[m], vy * uyt[m]);
            double fn = __builtin_fma(omct, fcm, A[m] * feq_poly(eta, t0[m]));
            fn = __builtin_fma(-a.cx, dhx, fn);
            fn = __builtin_fma(-a.cy, dhy, fn);
            double* dst = base + (int64_t)m * a.nx;
            if (!BND || (gx < a.nx && y0 + m < a.ny)) {
                if (NT)
                    __builtin_nontemporal_store(fn, &dst[(unsigned)lane]);
                else
                    dst[(unsigned)lane] = fn;
            }
        };
        if (vy > 0.0) {
            y_pass<R, false>(s_pl, lane, vy, eps, upd);
        } else if (vy < 0.0) {
            y_pass<R, true>(s_pl, lane, vy, eps, upd);
        } else {
#pragma unroll
            for (int m = 0; m < R; ++m) upd(m, s_pl[(m + HALO) * PITCH + lane + HALO], 0.0);
        }
    };

    double pa[Stage<R>::NPRE], pb[Stage<R>::NPRE];
    stage_load_g<R, HALO, PITCH, BND, false>(a.fin, g, k, i0, x0, y0, lane, t, plane, pa);
    stage_store_g<R, HALO, PITCH, BND, false>(g, k, se, i0, y0, lane, t, s_pl, pa);
    __syncthreads();
    if (DEPTH == 2) stage_load_g<R, HALO, PITCH, BND, false>(a.fin, g, k, i0 + 1 < iend ? i0 + 1 : i0, x0, y0, lane, t, plane, pb);
#pragma unroll 1
    for (int i = i0; i < iend; i += DEPTH) {
        if (DEPTH == 1) {
            stage_load_g<R, HALO, PITCH, BND, false>(a.fin, g, k, i + 1 < iend ? i + 1 : i, x0, y0, lane, t, plane, pa);
            compute(i);
            stage_store_g<R, HALO, PITCH, BND, false>(g, k, se, i + 1 < iend ? i + 1 : i, y0, lane, t, s_pl, pa);
            __syncthreads();
        } else {
            stage_load_g<R, HALO, PITCH, BND, false>(a.fin, g, k, i + 2 < iend ? i + 2 : i, x0, y0, lane, t, plane, pa);
            compute(i);
            stage_store_g<R, HALO, PITCH, BND, false>(g, k, se, i + 1, y0, lane, t, s_pl, pb);
            __syncthreads();
            stage_load_g<R, HALO, PITCH, BND, false>(a.fin, g, k, i + 3 < iend ? i + 3 : i, x0, y0, lane, t, plane, pb);
            compute(i + 1);
            stage_store_g<R, HALO, PITCH, BND, false>(g, k, se, i + 2 < iend ? i + 2 : i, y0, lane, t, s_pl, pa);
            __syncthreads();
        }
    }
}

// One work item (tile, group) of a step. ke_dst, if not null, receives the
// tile's (sum, max) of rho u_y^2 / 2 (group 0 only).
template <int R, int G, int DEPTH, bool NT, class SE>
__device__ __forceinline__ void step_work(const StepGrid& a, const Consts& k, SE se, int tile,
                                          int grp, double* ke_dst, double* s_pl, double* s_dx)
{
    const int lane = threadIdx.x;
    const int ty = tile / a.tiles_x, tx = tile - ty * a.tiles_x;
    const int x0 = tx * TX, y0 = ty * R;
    const int64_t plane = (int64_t)a.nx * a.ny;
    const bool interior =
        x0 >= HALO && x0 + TX + HALO <= a.nx && y0 >= HALO && y0 + R + HALO <= a.ny;
    const int gx = x0 + lane;

    // ---- phase 1: moments, equilibrium data, rest particle, diagnostics ----
    double rho[R], Tm[R], uxt[R], uyt[R], t0[R];
    double ke_s = 0.0, ke_m = 0.0;
#pragma unroll
    for (int m = 0; m < R; ++m) {
        const int gy = y0 + m;
        const bool act = gx < a.nx && gy < a.ny;
        double r = 1.0, jx = 0.0, jy = 0.0, E = 1.0, fz = 0.0;
        if (act) {
            const double* p = a.fin + (int64_t)gy * a.nx + x0;
            r = 0.0;
            E = 0.0;
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                const double fi = (p + i * plane)[(unsigned)lane];
                if (i == 0) fz = fi;
                r += fi;
                jx = __builtin_fma(fi, k.vx[i], jx);
                jy = __builtin_fma(fi, k.vy[i], jy);
                E = __builtin_fma(fi, k.hv2[i], E);
            }
        }
        const CellEq c = cell_eq_from_sums(r, jx, jy, E);
        rho[m] = c.rho;
        Tm[m] = c.T;
        uxt[m] = c.uxt;
        uyt[m] = c.uyt;
        t0[m] = c.t0;
        if (act && grp == 0) {
            const double uy = jy / r;
            const double e = 0.5 * r * uy * uy;
            ke_s += e;
            ke_m = fmax(ke_m, e);
            // rest particle: no convection, f^eq_0 = rho F_0 (1 - u^2/2T)
            const double F0 =
                1.0 - 6.0 * (weight_c(k, 0, c.T) + weight_c(k, 1, c.T) + weight_c(k, 2, c.T));
            const double fe = c.rho * F0 * c.t0;
            (a.fout + (int64_t)gy * a.nx + x0)[(unsigned)lane] = __builtin_fma(-a.ct, fz - fe, fz);
        }
    }
    if (ke_dst && grp == 0) {
        ke_s = wave_sum(ke_s);
        ke_m = wave_max(ke_m);
        if (lane == 0) {
            ke_dst[0] = ke_s;
            ke_dst[1] = ke_m;
        }
    }

    // ---- phase 2 ----
    const TileMapG t = tile_map_g<R, HALO, false>(grid_bc(a), x0, y0, lane, !interior);
    if (interior)
        plane_loop<R, G, false, DEPTH, NT>(a, k, se, grp, x0, y0, lane, t, plane, s_pl, s_dx, rho,
                                           Tm, uxt, uyt, t0);
    else
        plane_loop<R, G, true, DEPTH, NT>(a, k, se, grp, x0, y0, lane, t, plane, s_pl, s_dx, rho,
                                          Tm, uxt, uyt, t0);
}

// Step kernel variants: rows per lane R, velocity groups G, the
// wavefronts-per-SIMD target W that bounds the register budget, planes in
// flight D and non-temporal stores NT. Both the single-grid and the batched
// kernel are instantiated for every entry, in this order.
// Variants that the 128-register budget of W = 4 forces to spill are left
// out: two such builds gave wrong results on a 5 x 3 grid with fixed x sides.
#define LBM_STEP_VARIANTS(X)                                                                     \
    X(4, 1, 3, 1, 0) X(4, 3, 3, 1, 0) X(8, 2, 2, 1, 0) X(8, 1, 2, 1, 0) X(2, 3, 4, 1, 0)         \
    X(4, 1, 3, 2, 0) X(4, 3, 3, 2, 0) X(8, 1, 2, 2, 0) X(8, 2, 2, 1, 1) X(4, 1, 3, 2, 1)         \
    X(8, 1, 3, 1, 0)

}  // namespace lbmd
