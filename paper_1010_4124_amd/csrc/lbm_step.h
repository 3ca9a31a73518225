// lbm_step.h -- body of one forward-Euler D2V19 FDLB step (Eq. (47) of
// arXiv:1010.4124) for one 64 x R tile, shared by the single-grid kernel
// (lbm_forward.hip) and the batched kernel (lbm_batch.hip).
//
// The 18 moving velocities are split into G groups. Without carried moments
// (M = 0) each group of a tile is a separate one-wavefront workgroup that
// forms the tile's moments itself; with carried moments (M = 1) the G groups
// are the wavefronts of one workgroup, each with its own LDS region. Each
// lane owns a column strip of R cells.
//
//   phase 1  the moments of Eq. (10) of the tile's cells: summed over the 19
//            planes (M = 0), or read back from the sums rho, j, E that the
//            previous step wrote (M = 1). Every lane keeps u/T, 1-u^2/2T and
//            rho, T of its cells in registers. Group 0 also relaxes and
//            stores the rest particle and reduces the tile's transverse
//            kinetic energy.
//   phase 2  for each velocity i of the wave's group:
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
//   phase 3  (carried moments) the waves' partial sums of rho, j, E over the
//            f^{n+1} values they stored are added up in a fixed order and
//            written for the next step.
#pragma once

#include <type_traits>

#include "lbm_device.h"
#include "lbm_stage.h"

namespace lbmd {

constexpr int TX = 64;
constexpr int PITCH = 71;   // LDS row pitch of a staged plane (odd: no bank conflicts)
constexpr int XPITCH = 65;  // LDS row pitch of the x flux differences

template <int R>
using Stage = StageG<R, HALO, PITCH>;

// One grid as seen by a step: states, shape, boundary rules (with the outflow
// ghost arrays), the ratios dt/dx, dt/dy, dt/tau and the velocity component
// of the energy diagnostic (0: u_y, 1: u_x).
struct StepGrid {
    const double* __restrict__ fin;
    double* __restrict__ fout;
    int nx, ny;
    int bc[4];
    int tiles_x;
    int ke_axis;
    double cx, cy, ct;
    const double* gb[4];
};

__device__ __forceinline__ GridBC grid_bc(const StepGrid& s)
{
    return GridBC{s.nx, s.ny, {s.bc[0], s.bc[1], s.bc[2], s.bc[3]},
                  {s.gb[0], s.gb[1], s.gb[2], s.gb[3]}};
}

// x pass: lane -> (row r = lane % R, strip s = lane / R); the flux
// differences of f (WENO on f with eps / v_x^2: weno_faces) go to s_dx.
template <int R, bool NEG>
__device__ __forceinline__ void x_pass(const double* s_pl, double* s_dx, int lane, double eps)
{
    const int r = lane % R, s = lane / R;
    const double* b = s_pl + (r + HALO) * PITCH + s * R;
    double P[R + 5];
#pragma unroll
    for (int k = 0; k < R + 5; ++k) P[k] = NEG ? b[R + 5 - k] : b[k];
    double* out = s_dx + r * XPITCH + s * R;
    weno_strip<R, NEG>(P, eps, [&](int m, double d) { out[m] = d; });
}

// y pass: lane = column; calls upd(m, f_m, dh^y_m) for each cell of the strip
// as soon as its two faces are known (flux differences of f, as in x_pass).
template <int R, bool NEG, class Upd>
__device__ __forceinline__ void y_pass(const double* s_pl, int lane, double eps, Upd&& upd)
{
    const double* col = s_pl + lane + HALO;
    double P[R + 5];
#pragma unroll
    for (int k = 0; k < R + 5; ++k) P[k] = NEG ? col[(R + 5 - k) * PITCH] : col[k * PITCH];
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

// Outflow ghost arrays of a grid (null: not an outflow side) and its shape.
struct Ghosts {
    double* g[4];
    int nx, ny;
};

// f^eq of cell state q into position p of the ghost array g of a side of
// length len (g[i * len + p]), evaluated as outflow_point evaluates it.
__device__ __forceinline__ void ghost_from_state(double* g, int len, int p, const CellEq& q,
                                                 const Consts& k)
{
    const double F1 = weight_c(k, 0, q.T), F2 = weight_c(k, 1, q.T), F3 = weight_c(k, 2, q.T);
    g[p] = q.rho * (1.0 - 6.0 * (F1 + F2 + F3)) * q.t0;
#pragma unroll
    for (int i = 1; i < NV; ++i) {
        const double A = q.rho * (i < 7 ? F1 : i < 13 ? F2 : F3);
        const double eta = __builtin_fma(k.vx[i], q.uxt, k.vy[i] * q.uyt);
        g[(int64_t)i * len + p] = A * feq_poly(eta, q.t0);
    }
}

// Block `blk` of the state pass, one thread per cell c = blk * 256 + thread
// of a grid of n cells: the moments of Eq. (10) summed over the 19 planes in
// the order phase 1 uses, the cell state (dt/tau rho, T, u/T, v/T) for the
// step kernel, the rest particle's update (no convection: f_0' = f_0 -
// dt/tau (f_0 - rho F_0 (1 - u^2/2T))) and, if part is not null, the block's
// (sum, max) of rho u_n^2 / 2 in part[2 blk], part[2 blk + 1]. Cells on an
// outflow side (gh.g[side] not null) also write their ghost values, as the
// outflow kernel would from the same f (Eqs. (63)-(64)). sr: 8 doubles of
// workgroup LDS; every thread of the block must call this.
__device__ __forceinline__ void state_block(const double* __restrict__ f,
                                            double* __restrict__ fout, double* __restrict__ st,
                                            int64_t n, double ct, int ke_axis,
                                            double* __restrict__ part, const Consts& k,
                                            int64_t blk, double* sr, const Ghosts& gh)
{
    const int64_t c = blk * 256 + threadIdx.x;
    double e = 0.0;
    if (c < n) {
        double r = 0.0, jx = 0.0, jy = 0.0, E = 0.0;
        const double f0 = f[c];
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const double fi = f[i * n + c];
            r += fi;
            jx = __builtin_fma(fi, k.vx[i], jx);
            jy = __builtin_fma(fi, k.vy[i], jy);
            E = __builtin_fma(fi, k.hv2[i], E);
        }
        const CellEq q = cell_eq_from_sums(r, jx, jy, E);
        const double F0 =
            1.0 - 6.0 * (weight_c(k, 0, q.T) + weight_c(k, 1, q.T) + weight_c(k, 2, q.T));
        const double fe = q.rho * F0 * q.t0;
        fout[c] = __builtin_fma(-ct, f0 - fe, f0);
        st[c] = ct * q.rho;
        st[n + c] = q.T;
        st[2 * n + c] = q.uxt;
        st[3 * n + c] = q.uyt;
        const double un = (ke_axis ? jx : jy) / r;
        e = 0.5 * r * un * un;
        if (gh.g[0] || gh.g[1] || gh.g[2] || gh.g[3]) {
            const int y = (int)(c / gh.nx), x = (int)(c - (int64_t)y * gh.nx);
            if (gh.g[0] && x == 0) ghost_from_state(gh.g[0], gh.ny, y, q, k);
            if (gh.g[1] && x == gh.nx - 1) ghost_from_state(gh.g[1], gh.ny, y, q, k);
            if (gh.g[2] && y == 0) ghost_from_state(gh.g[2], gh.nx, x, q, k);
            if (gh.g[3] && y == gh.ny - 1) ghost_from_state(gh.g[3], gh.nx, x, q, k);
        }
    }
    if (!part) return;
    const double s = wave_sum(e), mx = wave_max(e);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sr[2 * w] = s;
        sr[2 * w + 1] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        part[2 * blk] = sr[0] + sr[2] + sr[4] + sr[6];
        part[2 * blk + 1] = fmax(fmax(sr[1], sr[3]), fmax(sr[5], sr[7]));
    }
}

// Outflow ghosts (Sec. IV.A, Eqs. (63)-(64)) at position p of side `side` of
// an nx x ny grid: f^eq of the moments of the nearest interior cell, into
// g[i][p] (side length ny for x sides, nx for y sides; p beyond it: nothing).
__device__ __forceinline__ void outflow_point(const double* __restrict__ f, int nx, int ny,
                                              double* g, int side, int p, const Consts& k)
{
    const int len = side < 2 ? ny : nx;
    if (p >= len) return;
    const int x = side == 0 ? 0 : side == 1 ? nx - 1 : p;
    const int y = side < 2 ? p : (side == 2 ? 0 : ny - 1);
    const int64_t n = (int64_t)nx * ny, c = (int64_t)y * nx + x;
    double r = 0.0, jx = 0.0, jy = 0.0, E = 0.0;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        const double fi = f[i * n + c];
        r += fi;
        jx = __builtin_fma(fi, k.vx[i], jx);
        jy = __builtin_fma(fi, k.vy[i], jy);
        E = __builtin_fma(fi, k.hv2[i], E);
    }
    ghost_from_state(g, len, p, cell_eq_from_sums(r, jx, jy, E), k);
}

// Per-wave LDS region: the staged plane, the x flux differences, and (reused,
// carried-moment mode only) the exchange of the 4 x R moment sums of the
// wave's lanes.
template <int R, int MODE>
struct WaveLds {
    static constexpr int DX = Stage<R>::SLOTS;
    static constexpr int WORK = Stage<R>::SLOTS + R * XPITCH;
    static constexpr int XCH = MODE == 1 ? 4 * R * 64 : 0;
    static constexpr int SIZE = WORK > XCH ? WORK : XCH;
};

// How phase 1 obtains the tile's moments.
enum {
    PH_SUMS = 0,   // sum the 19 planes of f^n
    PH_CARRY = 1,  // read the sums rho, j, E the previous step wrote
    PH_STATE = 2,  // read the cell state (dt/tau rho, T, u/T, v/T) a state pass wrote
    PH_FAST = 3,   // carried sums as PH_CARRY; fast tiles by the kernel of lbm_fast.h
};

// Waves per workgroup of a variant: the G groups are waves of one workgroup
// only with carried moments.
template <int G, int MODE>
struct Waves {
    static constexpr int N = MODE == PH_CARRY ? G : 1;
};

// Orders one wave's LDS accesses between the staging, x-pass and y-pass of a
// plane. A one-wave workgroup uses the workgroup barrier; in a multi-wave
// workgroup each wave works in its own LDS region, LDS operations of a wave
// execute in issue order, and a wave-scope fence keeps the compiler from
// moving them across.
template <int G>
__device__ __forceinline__ void plane_sync()
{
    if constexpr (G == 1) {
        __syncthreads();
    } else {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// Sums rho, j_x, j_y, E of R cells (the four moment sums of Eq. (10)).
template <int R>
struct Sums {
    double r[R], jx[R], jy[R], E[R];
};

// Phase 2 of one tile: this wave's moving velocities. Instantiated once for
// interior tiles and once for boundary tiles, so that each loop is straight
// line code and the compiler tracks its outstanding loads and stores exactly.
// DEPTH planes are in flight ahead of the one being computed; every load is
// issued unconditionally (past the group's last plane the last plane is
// re-read) and consumed after the current plane's stores, so waiting for a
// staged plane never waits for stores. With CM the sums of the new values
// are accumulated into `acc`.
//
// late_load(tag) runs right after the first plane's loads are issued (tag: an
// integral_constant, true on boundary tiles): the state
// pass variants load the cell state there, so that staging the plane waits
// only for the plane (vector memory operations complete in issue order) and
// the x pass overlaps the state loads.
template <int R, int G, bool BND, int DEPTH, bool NT, int MODE, class SE, class LateLoad>
__device__ __forceinline__ void plane_loop(const StepGrid& a, const Consts& k, SE se,
                                           int grp, int x0, int y0, int lane, const TileMapG& t,
                                           int64_t plane, double* s_pl, double* s_dx,
                                           const double (&rho)[R], const double (&Tm)[R],
                                           const double (&uxt)[R], const double (&uyt)[R],
                                           const double (&t0)[MODE != PH_SUMS ? 1 : R],
                                           Sums<R>& acc, LateLoad&& late_load)
{
    constexpr bool CM = MODE == PH_CARRY;     // accumulate the new moment sums
    constexpr bool LEAN = MODE != PH_SUMS;    // rho[] = dt/tau rho, no t0[], no A cache
    constexpr int NPL = 18 / G;  // moving velocities per group
    static_assert(18 % G == 0, "G must divide the 18 moving velocities");
    static_assert(DEPTH == 1 || NPL % 2 == 0, "two-deep pipeline needs an even plane count");
    const int gx = x0 + lane;
    const int i0 = 1 + grp * NPL, iend = i0 + NPL;
    // (dt/tau) rho F_k(T) of the current speed shell: cached per shell, or
    // (lean register budget, where rho[] holds dt/tau rho and t0[] is
    // unused) recomputed per plane
    double A[LEAN ? 1 : R];
    int kcur = -1;
    const double omct = 1.0 - a.ct;
    const GridBC g = grid_bc(a);

    // f' = f - cx dh^x - cy dh^y - ct (f - f^eq)
    //    = (1 - ct) f + (ct rho F_k) poly(eta) - cx dh^x - cy dh^y,
    // dh the face flux differences of F = v f, here (cx v_x) and (cy v_y)
    // times those of f (weno_faces)
    auto compute = [&](int i) {
        const int ks = (i - 1) / 6;
        if (!LEAN && ks != kcur) {
            kcur = ks;
#pragma unroll
            for (int m = 0; m < (LEAN ? 1 : R); ++m) A[m] = (a.ct * rho[m]) * weight_c(k, ks, Tm[m]);
        }
        const double vx = k.vx[i], vy = k.vy[i];
        // the faces are those of f; v goes into the Courant factors
        const double cxv = a.cx * vx, cyv = a.cy * vy;
        if (vx < 0.0)
            x_pass<R, true>(s_pl, s_dx, lane, k.epsx[i]);
        else
            x_pass<R, false>(s_pl, s_dx, lane, k.epsx[i]);
        plane_sync<Waves<G, MODE>::N>();
        // one velocity per wave (lean state): fold the four state values of
        // each cell into the three the update needs, (dt/tau) rho F_k(T),
        // 1 - |u|^2/2T and eta = v.u/T, before the y pass (fewer live
        // registers there)
        constexpr bool FOLD = LEAN && NPL == 1;
        double fA[FOLD ? R : 1], ft0[FOLD ? R : 1], feta[FOLD ? R : 1];
        if constexpr (FOLD) {
#pragma unroll
            for (int m = 0; m < R; ++m) {
                fA[m] = rho[m] * weight_c(k, ks, Tm[m]);
                ft0[m] = __builtin_fma(-0.5 * Tm[m],
                                       __builtin_fma(uxt[m], uxt[m], uyt[m] * uyt[m]), 1.0);
                feta[m] = __builtin_fma(vx, uxt[m], vy * uyt[m]);
            }
        }
        double* base = a.fout + i * plane + (int64_t)y0 * a.nx + x0;
        const double hv = k.hv2[i];
        auto upd = [&](int m, double fcm, double dhy) {
            const double dhx = s_dx[m * XPITCH + lane];
            double eta, Am, t0m;
            if constexpr (FOLD) {
                eta = feta[m];
                Am = fA[m];
                t0m = ft0[m];
            } else if (LEAN) {
                eta = __builtin_fma(vx, uxt[m], vy * uyt[m]);
                Am = rho[m] * weight_c(k, ks, Tm[m]);
                // 1 - |u|^2 / 2T with u = T (u/T)
                t0m = __builtin_fma(-0.5 * Tm[m],
                                    __builtin_fma(uxt[m], uxt[m], uyt[m] * uyt[m]), 1.0);
            } else {
                eta = __builtin_fma(vx, uxt[m], vy * uyt[m]);
                Am = A[m];
                t0m = t0[m];
            }
            double fn = __builtin_fma(omct, fcm, Am * feq_poly(eta, t0m));
            fn = __builtin_fma(-cxv, dhx, fn);
            fn = __builtin_fma(-cyv, dhy, fn);
            if (CM) {
                acc.r[m] += fn;
                acc.jx[m] = __builtin_fma(fn, vx, acc.jx[m]);
                acc.jy[m] = __builtin_fma(fn, vy, acc.jy[m]);
                acc.E[m] = __builtin_fma(fn, hv, acc.E[m]);
            }
            double* dst = base + (int64_t)m * a.nx;
            if (!BND || (gx < a.nx && y0 + m < a.ny)) {
                if (NT)
                    __builtin_nontemporal_store(fn, &dst[(unsigned)lane]);
                else
                    dst[(unsigned)lane] = fn;
            }
        };
        if (vy > 0.0) {
            y_pass<R, false>(s_pl, lane, k.epsy[i], upd);
        } else if (vy < 0.0) {
            y_pass<R, true>(s_pl, lane, k.epsy[i], upd);
        } else {
#pragma unroll
            for (int m = 0; m < R; ++m) upd(m, s_pl[(m + HALO) * PITCH + lane + HALO], 0.0);
        }
    };

    double pa[Stage<R>::NPRE], pb[Stage<R>::NPRE];
    stage_load_g<R, HALO, PITCH, BND, false>(a.fin, g, k, i0, x0, y0, lane, t, plane, pa);
    late_load(std::integral_constant<bool, BND>{});
    stage_store_g<R, HALO, PITCH, BND, false>(g, k, se, i0, y0, lane, t, s_pl, pa);
    plane_sync<Waves<G, MODE>::N>();
    if constexpr (NPL == 1) {
        compute(i0);
        return;
    }
    if (DEPTH == 2) stage_load_g<R, HALO, PITCH, BND, false>(a.fin, g, k, i0 + 1 < iend ? i0 + 1 : i0, x0, y0, lane, t, plane, pb);
#pragma unroll 1
    for (int i = i0; i < iend; i += DEPTH) {
        if (DEPTH == 1) {
            stage_load_g<R, HALO, PITCH, BND, false>(a.fin, g, k, i + 1 < iend ? i + 1 : i, x0, y0, lane, t, plane, pa);
            compute(i);
            stage_store_g<R, HALO, PITCH, BND, false>(g, k, se, i + 1 < iend ? i + 1 : i, y0, lane, t, s_pl, pa);
            plane_sync<Waves<G, MODE>::N>();
        } else {
            stage_load_g<R, HALO, PITCH, BND, false>(a.fin, g, k, i + 2 < iend ? i + 2 : i, x0, y0, lane, t, plane, pa);
            compute(i);
            stage_store_g<R, HALO, PITCH, BND, false>(g, k, se, i + 1, y0, lane, t, s_pl, pb);
            plane_sync<Waves<G, MODE>::N>();
            stage_load_g<R, HALO, PITCH, BND, false>(a.fin, g, k, i + 3 < iend ? i + 3 : i, x0, y0, lane, t, plane, pb);
            compute(i + 1);
            stage_store_g<R, HALO, PITCH, BND, false>(g, k, se, i + 2 < iend ? i + 2 : i, y0, lane, t, s_pl, pa);
            plane_sync<Waves<G, MODE>::N>();
        }
    }
}

// Adds up the G waves' partial sums through LDS, in wave order, so that
// every wave (or wave 0 alone, `all` false) obtains the same totals. Ends
// with a workgroup barrier after which the LDS regions may be reused.
template <int R, int G>
__device__ __forceinline__ void exchange_sums(double* lds, int wave, int lane, Sums<R>& s, bool all)
{
    double* mine = lds + wave * WaveLds<R, 1>::SIZE;
#pragma unroll
    for (int m = 0; m < R; ++m) {
        mine[(0 * R + m) * 64 + lane] = s.r[m];
        mine[(1 * R + m) * 64 + lane] = s.jx[m];
        mine[(2 * R + m) * 64 + lane] = s.jy[m];
        mine[(3 * R + m) * 64 + lane] = s.E[m];
    }
    __syncthreads();
    if (all || wave == 0) {
#pragma unroll
        for (int m = 0; m < R; ++m) {
            const double* p0 = lds;
            double r = p0[(0 * R + m) * 64 + lane], jx = p0[(1 * R + m) * 64 + lane];
            double jy = p0[(2 * R + m) * 64 + lane], E = p0[(3 * R + m) * 64 + lane];
#pragma unroll
            for (int w = 1; w < G; ++w) {
                const double* p = lds + w * WaveLds<R, 1>::SIZE;
                r += p[(0 * R + m) * 64 + lane];
                jx += p[(1 * R + m) * 64 + lane];
                jy += p[(2 * R + m) * 64 + lane];
                E += p[(3 * R + m) * 64 + lane];
            }
            s.r[m] = r;
            s.jx[m] = jx;
            s.jy[m] = jy;
            s.E[m] = E;
        }
    }
    __syncthreads();
}

// One work item of a step: tile `tile` and, unless the moments are carried,
// velocity group `grp` (with carried moments the group is the wave's index).
// ke_dst, if not null, receives the tile's (sum, max) of rho u_n^2 / 2.
// m_in / m_out: PH_CARRY reads and writes the moment sums (rho, j_x, j_y, E,
// each [ny][nx]); PH_STATE reads the cell state (dt/tau rho, T, u/T, v/T)
// and leaves the rest particle and the diagnostics to the state pass. lds
// holds Waves<G, MODE>::N regions of WaveLds<R, MODE>::SIZE doubles.
template <int R, int G, int DEPTH, bool NT, int MODE, class SE>
__device__ __forceinline__ void step_work(const StepGrid& a, const Consts& k, SE se, int tile,
                                          int grp, double* ke_dst, double* lds,
                                          const double* __restrict__ m_in,
                                          double* __restrict__ m_out)
{
    constexpr bool CM = MODE == PH_CARRY, PS = MODE == PH_STATE, LEAN = MODE != PH_SUMS;
    constexpr int NW = Waves<G, MODE>::N;
    const int lane = threadIdx.x & 63;
    const int wave = NW > 1 ? __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) : 0;
    if (NW > 1) grp = wave;
    double* s_pl = lds + wave * WaveLds<R, MODE>::SIZE;
    double* s_dx = s_pl + WaveLds<R, MODE>::DX;
    const int ty = tile / a.tiles_x, tx = tile - ty * a.tiles_x;
    const int x0 = tx * TX, y0 = ty * R;
    const int64_t plane = (int64_t)a.nx * a.ny;
    const bool interior = fast_tile(grid_bc(a), x0, y0, TX, R, HALO);
    const int gx = x0 + lane;

    // ---- phase 1: moments, equilibrium data, rest particle, diagnostics ----
    // rho[] holds dt/tau rho in the lean modes (see plane_loop)
    double rho[R], Tm[R], uxt[R], uyt[R], t0[LEAN ? 1 : R];
    Sums<R> acc;
#pragma unroll
    for (int m = 0; m < R; ++m) acc.r[m] = acc.jx[m] = acc.jy[m] = acc.E[m] = 0.0;
    // PS: the cell state, loaded by plane_loop once the first plane's loads
    // are in flight
    auto load_state = [&](auto bnd) {
        if constexpr (PS) {
            // keep the scheduler from hoisting these above the plane's loads
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int m = 0; m < R; ++m) {
                const int64_t c = (int64_t)(y0 + m) * a.nx + gx;
                if constexpr (!decltype(bnd)::value) {
                    // fast tile: every lane holds a cell; unconditional loads
                    // keep the waits exact (no branch joins)
                    rho[m] = m_in[c];
                    Tm[m] = m_in[plane + c];
                    uxt[m] = m_in[2 * plane + c];
                    uyt[m] = m_in[3 * plane + c];
                } else {
                    const bool act = gx < a.nx && y0 + m < a.ny;
                    rho[m] = act ? m_in[c] : a.ct;  // idle lanes: unit state
                    Tm[m] = act ? m_in[plane + c] : 1.0;
                    uxt[m] = act ? m_in[2 * plane + c] : 0.0;
                    uyt[m] = act ? m_in[3 * plane + c] : 0.0;
                }
            }
        }
    };
    if constexpr (!PS) {
        Sums<R> sum;
        double fz[R];
#pragma unroll
        for (int m = 0; m < R; ++m) {
            const int gy = y0 + m;
            const bool act = gx < a.nx && gy < a.ny;
            double r = 0.0, jx = 0.0, jy = 0.0, E = 0.0, f0 = 0.0;
            if (act) {
                const int64_t c = (int64_t)gy * a.nx + gx;
                if (CM) {
                    r = m_in[c];
                    jx = m_in[plane + c];
                    jy = m_in[2 * plane + c];
                    E = m_in[3 * plane + c];
                    if (grp == 0) f0 = a.fin[c];
                } else {
                    const double* p = a.fin + (int64_t)gy * a.nx + x0;
#pragma unroll
                    for (int i = 0; i < NV; ++i) {
                        const double fi = (p + i * plane)[(unsigned)lane];
                        if (i == 0) f0 = fi;
                        r += fi;
                        jx = __builtin_fma(fi, k.vx[i], jx);
                        jy = __builtin_fma(fi, k.vy[i], jy);
                        E = __builtin_fma(fi, k.hv2[i], E);
                    }
                }
            }
            sum.r[m] = r;
            sum.jx[m] = jx;
            sum.jy[m] = jy;
            sum.E[m] = E;
            fz[m] = f0;
        }

        double ke_s = 0.0, ke_m = 0.0;
#pragma unroll
        for (int m = 0; m < R; ++m) {
            const bool act = gx < a.nx && y0 + m < a.ny;
            // idle lanes get a harmless unit state
            const double r = act ? sum.r[m] : 1.0, E = act ? sum.E[m] : 1.0;
            const double jx = act ? sum.jx[m] : 0.0, jy = act ? sum.jy[m] : 0.0;
            const CellEq c = cell_eq_from_sums(r, jx, jy, E);
            rho[m] = LEAN ? a.ct * c.rho : c.rho;
            Tm[m] = c.T;
            uxt[m] = c.uxt;
            uyt[m] = c.uyt;
            if (!LEAN) t0[m] = c.t0;
            if (act && grp == 0) {
                const double un = (a.ke_axis ? jx : jy) / r;
                const double e = 0.5 * r * un * un;
                ke_s += e;
                ke_m = fmax(ke_m, e);
                // rest particle: no convection, f^eq_0 = rho F_0 (1 - u^2/2T)
                const double F0 = 1.0 - 6.0 * (weight_c(k, 0, c.T) + weight_c(k, 1, c.T) +
                                               weight_c(k, 2, c.T));
                const double fe = c.rho * F0 * c.t0;
                const double fn = __builtin_fma(-a.ct, fz[m] - fe, fz[m]);
                (a.fout + (int64_t)(y0 + m) * a.nx + x0)[(unsigned)lane] = fn;
                acc.r[m] = fn;  // v_0 = 0: the rest particle adds to rho only
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
    }

    // ---- phase 2 ----
    const TileMapG t = tile_map_g<R, HALO, false>(grid_bc(a), x0, y0, lane, !interior);
    if (interior)
        plane_loop<R, G, false, DEPTH, NT, MODE>(a, k, se, grp, x0, y0, lane, t, plane, s_pl,
                                                 s_dx, rho, Tm, uxt, uyt, t0, acc, load_state);
    else
        plane_loop<R, G, true, DEPTH, NT, MODE>(a, k, se, grp, x0, y0, lane, t, plane, s_pl,
                                                s_dx, rho, Tm, uxt, uyt, t0, acc, load_state);

    // ---- phase 3: moment sums of f^{n+1} for the next step ----
    if (CM) {
        if (NW > 1) exchange_sums<R, NW>(lds, wave, lane, acc, false);
        if (wave == 0) {
#pragma unroll
            for (int m = 0; m < R; ++m) {
                if (gx < a.nx && y0 + m < a.ny) {
                    const int64_t c = (int64_t)(y0 + m) * a.nx + gx;
                    m_out[c] = acc.r[m];
                    m_out[plane + c] = acc.jx[m];
                    m_out[2 * plane + c] = acc.jy[m];
                    m_out[3 * plane + c] = acc.E[m];
                }
            }
        }
    }
}

// Step kernel variants: rows per lane R, velocity groups G (18/G moving
// velocities each), the wavefronts-per-SIMD target W that bounds the register
// budget, planes in flight D, non-temporal stores NT, the phase-1 mode M
// (PH_SUMS, PH_CARRY: the G groups are the waves of one workgroup, PH_STATE:
// a state pass runs first, PH_FAST: PH_CARRY with the fast tiles advanced by
// the kernel of lbm_fast.h and the others by the PH_CARRY kernel) and the
// wave target WB of the batched kernel,
// which keeps an instance descriptor live as well and so may need a larger
// register budget (a lower target) for the same variant. Both the
// single-grid and the batched kernel are instantiated for every entry, in
// this order. No kernel may spill registers to scratch memory (the build
// refuses one that does): the targets are chosen so that none does.
#define LBM_STEP_VARIANTS(X)                                                                     \
    X(4, 1, 3, 1, 0, 0, 2) X(4, 3, 3, 1, 0, 0, 2) X(8, 2, 2, 1, 0, 0, 1)                         \
    X(8, 1, 2, 1, 0, 0, 1) X(2, 3, 4, 1, 0, 0, 3) X(8, 2, 2, 1, 1, 0, 1)                         \
    X(4, 2, 3, 1, 0, 0, 2) X(4, 1, 2, 1, 0, 1, 2) X(4, 1, 2, 2, 1, 1, 2)                         \
    X(4, 3, 2, 1, 1, 1, 2) X(4, 1, 2, 2, 0, 1, 2) X(4, 18, 4, 1, 0, 2, 3)                        \
    X(2, 18, 5, 1, 0, 2, 4) X(4, 3, 3, 1, 0, 2, 3)                                               \
    X(2, 9, 4, 1, 0, 2, 3) X(2, 6, 4, 1, 0, 2, 3) X(4, 9, 3, 1, 0, 2, 3)                         \
    X(4, 6, 3, 1, 0, 2, 3) X(2, 1, 3, 1, 1, 1, 3) X(2, 1, 3, 1, 0, 1, 3)                         \
    X(4, 1, 2, 1, 1, 3, 2) X(4, 1, 2, 2, 1, 3, 2) X(4, 1, 2, 1, 0, 3, 2)

}  // namespace lbmd
