// lbm_forward.hip -- forward kernels of liblbm_hip for gfx950 (MI355X).
//
// One launch of k_step advances every cell by one forward-Euler step of the
// D2V19 FDLB model (Eq. (47) of arXiv:1010.4124). Work is split into
// one-wavefront workgroups, each owning a tile of 64 columns x R rows and one
// of G groups of the 18 moving velocities; each lane owns a column strip of R
// cells.
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
// A tile's G workgroups repeat phase 1 (the 19 centre values come from L2);
// G > 1 multiplies the number of workgroups on small grids. Workgroups are
// assigned XCD-major: hardware dispatches consecutive workgroups round-robin
// over the 8 XCDs, so workgroup b takes work item (b % 8) * per_xcd + b / 8
// and every XCD sweeps one contiguous band of tiles whose halos then meet in
// that XCD's L2. The per-context constants travel by value in the kernel
// arguments and are read with scalar loads.
#include "lbm_device.h"
#include "lbm_internal.h"
#include "lbm_stage.h"

namespace lbmd {

constexpr int TX = 64;
constexpr int PITCH = 71;   // LDS row pitch of a staged plane (odd: no bank conflicts)
constexpr int XPITCH = 65;  // LDS row pitch of the x flux differences

struct StepArgs {
    const double* __restrict__ fin;
    double* __restrict__ fout;
    double* __restrict__ ke_part;  // [ntiles][2] or null
    int nx, ny;
    int bc[4];
    int tiles_x, ntiles, nwork, per_xcd;
    double cx, cy, ct;  // dt/dx, dt/dy, dt/tau
    Consts k;
};

template <int R>
using Stage = StageG<R, HALO, PITCH>;

__device__ __forceinline__ GridBC grid_of(const StepArgs& a)
{
    return GridBC{a.nx, a.ny, {a.bc[0], a.bc[1], a.bc[2], a.bc[3]}};
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
template <int R, int G, bool BND, int DEPTH, bool NT>
__device__ __forceinline__ void plane_loop(const StepArgs& a, int grp, int x0, int y0, int lane,
                                           const TileMapG& t, int64_t plane, double* s_pl,
                                           double* s_dx, const double (&rho)[R],
                                           const double (&Tm)[R], const double (&uxt)[R],
                                           const double (&uyt)[R], const double (&t0)[R])
{
    constexpr int NPL = 18 / G;  // moving velocities per group
    static_assert(DEPTH == 1 || NPL % 2 == 0, "two-deep pipeline needs an even plane count");
    const int gx = x0 + lane;
    const int i0 = 1 + grp * NPL, iend = i0 + NPL;
    double A[R];  // (dt/tau) rho F_k(T) of the current speed shell
    int kcur = -1;
    const double omct = 1.0 - a.ct;
    const GridBC g = grid_of(a);

    // f' = f - cx dh^x - cy dh^y - ct (f - f^eq)
    //    = (1 - ct) f + (ct rho F_k) poly(eta) - cx dh^x - cy dh^y
    auto compute = [&](int i) {
        const int k = (i - 1) / 6;
        if (k != kcur) {
            kcur = k;
#pragma unroll
            for (int m = 0; m < R; ++m) A[m] = (a.ct * rho[m]) * weight_c(a.k, k, Tm[m]);
        }
        const double vx = a.k.vx[i], vy = a.k.vy[i], eps = a.k.eps;
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
    stage_load_g<R, HALO, PITCH, BND, false>(a.fin, g, a.k, i0, x0, y0, lane, t, plane, pa);
    stage_store_g<R, HALO, PITCH, BND, false>(g, a.k, i0, y0, lane, t, s_pl, pa);
    __syncthreads();
    if (DEPTH == 2) stage_load_g<R, HALO, PITCH, BND, false>(a.fin, g, a.k, i0 + 1 < iend ? i0 + 1 : i0, x0, y0, lane, t, plane, pb);
#pragma unroll 1
    for (int i = i0; i < iend; i += DEPTH) {
        if (DEPTH == 1) {
            stage_load_g<R, HALO, PITCH, BND, false>(a.fin, g, a.k, i + 1 < iend ? i + 1 : i, x0, y0, lane, t, plane, pa);
            compute(i);
            stage_store_g<R, HALO, PITCH, BND, false>(g, a.k, i + 1 < iend ? i + 1 : i, y0, lane, t, s_pl, pa);
            __syncthreads();
        } else {
            stage_load_g<R, HALO, PITCH, BND, false>(a.fin, g, a.k, i + 2 < iend ? i + 2 : i, x0, y0, lane, t, plane, pa);
            compute(i);
            stage_store_g<R, HALO, PITCH, BND, false>(g, a.k, i + 1, y0, lane, t, s_pl, pb);
            __syncthreads();
            stage_load_g<R, HALO, PITCH, BND, false>(a.fin, g, a.k, i + 3 < iend ? i + 3 : i, x0, y0, lane, t, plane, pb);
            compute(i + 1);
            stage_store_g<R, HALO, PITCH, BND, false>(g, a.k, i + 2 < iend ? i + 2 : i, y0, lane, t, s_pl, pa);
            __syncthreads();
        }
    }
}

template <int R, int G, int W, int DEPTH, bool NT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(W))) void k_step(StepArgs a)
{
    __shared__ double s_pl[Stage<R>::SLOTS];
    __shared__ double s_dx[R * XPITCH];

    const int b = blockIdx.x;
    const int work = (b & 7) * a.per_xcd + (b >> 3);
    if (work >= a.nwork) return;
    const int tile = work / G, grp = work - tile * G;
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
                jx = __builtin_fma(fi, a.k.vx[i], jx);
                jy = __builtin_fma(fi, a.k.vy[i], jy);
                E = __builtin_fma(fi, a.k.hv2[i], E);
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
            const double F0 = 1.0 - 6.0 * (weight_c(a.k, 0, c.T) + weight_c(a.k, 1, c.T) +
                                            weight_c(a.k, 2, c.T));
            const double fe = c.rho * F0 * c.t0;
            (a.fout + (int64_t)gy * a.nx + x0)[(unsigned)lane] = __builtin_fma(-a.ct, fz - fe, fz);
        }
    }
    if (a.ke_part && grp == 0) {
        ke_s = wave_sum(ke_s);
        ke_m = wave_max(ke_m);
        if (lane == 0) {
            a.ke_part[2 * tile] = ke_s;
            a.ke_part[2 * tile + 1] = ke_m;
        }
    }

    // ---- phase 2 ----
    const TileMapG t = tile_map_g<R, HALO, false>(grid_of(a), x0, y0, lane, !interior);
    if (interior)
        plane_loop<R, G, false, DEPTH, NT>(a, grp, x0, y0, lane, t, plane, s_pl, s_dx, rho, Tm, uxt,
                                           uyt, t0);
    else
        plane_loop<R, G, true, DEPTH, NT>(a, grp, x0, y0, lane, t, plane, s_pl, s_dx, rho, Tm, uxt,
                                          uyt, t0);
}

// ---------------------------------------------------------------------------
// f = f^eq(rho, u, T), one thread per cell (Eq. (28)).
__global__ void k_init(const double* __restrict__ rho, const double* __restrict__ ux,
                       const double* __restrict__ uy, const double* __restrict__ T,
                       double* __restrict__ f, int64_t n, Consts k)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const double r = rho[c], u = ux[c], v = uy[c], t = T[c];
    const double iT = 1.0 / t;
    const double t0 = 1.0 - (u * u + v * v) / (2.0 * t);
    const double uxt = u * iT, uyt = v * iT;
    double A[4];
    A[1] = r * weight_c(k, 0, t);
    A[2] = r * weight_c(k, 1, t);
    A[3] = r * weight_c(k, 2, t);
    A[0] = r * (1.0 - 6.0 * (weight_c(k, 0, t) + weight_c(k, 1, t) + weight_c(k, 2, t)));
    f[c] = A[0] * t0;
#pragma unroll
    for (int i = 1; i < NV; ++i) {
        const double eta = __builtin_fma(k.vx[i], uxt, k.vy[i] * uyt);
        f[i * n + c] = A[1 + (i - 1) / 6] * feq_poly(eta, t0);
    }
}

// Fixed-side equilibria: four (rho, ux, uy, T) states -> out[4][19].
__global__ void k_side_eq(double* out, double4 s0, double4 s1, double4 s2, double4 s3, Consts k)
{
    const int i = threadIdx.x;
    const int s = blockIdx.x;
    if (i >= NV || s >= 4) return;
    const double4 st = s == 0 ? s0 : s == 1 ? s1 : s == 2 ? s2 : s3;
    const double r = st.x, u = st.y, v = st.z, t = st.w;
    if (!(r > 0.0) || !(t > 0.0)) {
        out[s * NV + i] = 0.0;
        return;
    }
    const double iT = 1.0 / t;
    const double t0 = 1.0 - (u * u + v * v) / (2.0 * t);
    double A;
    if (i == 0)
        A = r * (1.0 - 6.0 * (weight_c(k, 0, t) + weight_c(k, 1, t) + weight_c(k, 2, t)));
    else
        A = r * weight_c(k, (i - 1) / 6, t);
    const double eta = __builtin_fma(k.vx[i], u * iT, k.vy[i] * (v * iT));
    out[s * NV + i] = A * feq_poly(eta, t0);
}

// Moments of Eq. (10) per cell.
__global__ void k_moments(const double* __restrict__ f, double* __restrict__ rho,
                          double* __restrict__ ux, double* __restrict__ uy,
                          double* __restrict__ T, int64_t n, Consts k)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    double r = 0.0, jx = 0.0, jy = 0.0, E = 0.0;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        const double fi = f[i * n + c];
        r += fi;
        jx = __builtin_fma(fi, k.vx[i], jx);
        jy = __builtin_fma(fi, k.vy[i], jy);
        E = __builtin_fma(fi, k.hv2[i], E);
    }
    const double u = jx / r, v = jy / r;
    rho[c] = r;
    ux[c] = u;
    uy[c] = v;
    T[c] = E / r - 0.5 * (u * u + v * v);
}

// Transverse kinetic energy partials: one (sum, max) pair per block of 256 cells.
__global__ __launch_bounds__(256) void k_kinetic_part(const double* __restrict__ f, int64_t n,
                                                      double* __restrict__ part, Consts k)
{
    __shared__ double sr[8];
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double e = 0.0;
    if (c < n) {
        double r = 0.0, jy = 0.0;
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const double fi = f[i * n + c];
            r += fi;
            jy = __builtin_fma(fi, k.vy[i], jy);
        }
        const double uy = jy / r;
        e = 0.5 * r * uy * uy;
    }
    const double s = wave_sum(e), mx = wave_max(e);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sr[2 * w] = s;
        sr[2 * w + 1] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = sr[0] + sr[2] + sr[4] + sr[6];
        part[2 * blockIdx.x + 1] = fmax(fmax(sr[1], sr[3]), fmax(sr[5], sr[7]));
    }
}

// Deterministic final reduction of n (sum, max) partials; out2[0] is scaled
// by dxdy.
__global__ __launch_bounds__(256) void k_reduce_pairs(const double* __restrict__ part, int n,
                                                      double dxdy, double* __restrict__ out2)
{
    __shared__ double sr[8];
    double s = 0.0, mx = 0.0;
    for (int j = threadIdx.x; j < n; j += 256) {
        s += part[2 * j];
        mx = fmax(mx, part[2 * j + 1]);
    }
    s = wave_sum(s);
    mx = wave_max(mx);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sr[2 * w] = s;
        sr[2 * w + 1] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        out2[0] = (sr[0] + sr[2] + sr[4] + sr[6]) * dxdy;
        out2[1] = fmax(fmax(sr[1], sr[3]), fmax(sr[5], sr[7]));
    }
}

// ---------------------------------------------------------------------------
// Step kernel variants: rows per lane R, velocity groups G, and the
// wavefronts-per-SIMD target W that bounds the register budget.
struct StepVariant {
    int R, G, W, D, NT;
    void (*kernel)(StepArgs);
};

// (rows per lane, velocity groups, waves-per-SIMD target, planes in flight,
// non-temporal stores)
#define LBM_STEP_VARIANT(R, G, W, D, NT) {R, G, W, D, NT, k_step<R, G, W, D, NT>}
static const StepVariant kStepVariants[] = {
    LBM_STEP_VARIANT(4, 1, 3, 1, 0), LBM_STEP_VARIANT(4, 3, 3, 1, 0), LBM_STEP_VARIANT(8, 2, 2, 1, 0),
    LBM_STEP_VARIANT(8, 1, 2, 1, 0), LBM_STEP_VARIANT(2, 3, 4, 1, 0), LBM_STEP_VARIANT(4, 1, 3, 2, 0),
    LBM_STEP_VARIANT(4, 3, 3, 2, 0), LBM_STEP_VARIANT(2, 3, 4, 2, 0), LBM_STEP_VARIANT(2, 1, 4, 2, 0),
    LBM_STEP_VARIANT(8, 1, 2, 2, 0), LBM_STEP_VARIANT(8, 2, 2, 1, 1), LBM_STEP_VARIANT(4, 1, 3, 2, 1),
    LBM_STEP_VARIANT(8, 1, 3, 1, 0), LBM_STEP_VARIANT(4, 1, 4, 2, 1), LBM_STEP_VARIANT(4, 3, 4, 1, 0),
};
#undef LBM_STEP_VARIANT
constexpr int kNumStepVariants = sizeof(kStepVariants) / sizeof(kStepVariants[0]);

int step_variant_count() { return kNumStepVariants; }
int step_variant_desc(int v, int* R, int* G, int* W, int* D, int* NT)
{
    if (v < 0 || v >= kNumStepVariants) return -1;
    *R = kStepVariants[v].R;
    *G = kStepVariants[v].G;
    *W = kStepVariants[v].W;
    *D = kStepVariants[v].D;
    *NT = kStepVariants[v].NT;
    return 0;
}

int step_ntiles(int variant, int nx, int ny)
{
    const StepVariant& V = kStepVariants[variant];
    return ((nx + TX - 1) / TX) * ((ny + V.R - 1) / V.R);
}

hipError_t launch_step(int variant, const double* fin, double* fout, const Consts& k,
                       double* ke_part, int nx, int ny, const int bc[4], double cx, double cy,
                       double ct, hipStream_t st)
{
    const StepVariant& V = kStepVariants[variant];
    StepArgs a;
    a.fin = fin;
    a.fout = fout;
    a.ke_part = ke_part;
    a.nx = nx;
    a.ny = ny;
    for (int s = 0; s < 4; ++s) a.bc[s] = bc[s];
    a.tiles_x = (nx + TX - 1) / TX;
    a.ntiles = a.tiles_x * ((ny + V.R - 1) / V.R);
    a.nwork = a.ntiles * V.G;
    a.per_xcd = (a.nwork + 7) / 8;
    a.cx = cx;
    a.cy = cy;
    a.ct = ct;
    a.k = k;
    hipLaunchKernelGGL(V.kernel, dim3(8 * a.per_xcd), dim3(64), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_reduce_pairs(const double* part, int n, double dxdy, double* out2,
                               hipStream_t st)
{
    hipLaunchKernelGGL(k_reduce_pairs, dim3(1), dim3(256), 0, st, part, n, dxdy, out2);
    return hipGetLastError();
}

hipError_t launch_init(const double* rho, const double* ux, const double* uy, const double* T,
                       double* f, const Consts& k, int64_t n, hipStream_t st)
{
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_init, dim3((unsigned)blocks), dim3(256), 0, st, rho, ux, uy, T, f, n, k);
    return hipGetLastError();
}

hipError_t launch_side_eq(double* out, const double s[4][4], const Consts& k, hipStream_t st)
{
    double4 q[4];
    for (int j = 0; j < 4; ++j) q[j] = make_double4(s[j][0], s[j][1], s[j][2], s[j][3]);
    hipLaunchKernelGGL(k_side_eq, dim3(4), dim3(32), 0, st, out, q[0], q[1], q[2], q[3], k);
    return hipGetLastError();
}

hipError_t launch_moments(const double* f, double* rho, double* ux, double* uy, double* T,
                          const Consts& k, int64_t n, hipStream_t st)
{
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_moments, dim3((unsigned)blocks), dim3(256), 0, st, f, rho, ux, uy, T, n,
                       k);
    return hipGetLastError();
}

hipError_t launch_kinetic_part(const double* f, const Consts& k, int64_t n, double* part,
                               int* nparts, hipStream_t st)
{
    const int64_t blocks = (n + 255) / 256;
    *nparts = (int)blocks;
    hipLaunchKernelGGL(k_kinetic_part, dim3((unsigned)blocks), dim3(256), 0, st, f, n, part, k);
    return hipGetLastError();
}

}  // namespace lbmd
