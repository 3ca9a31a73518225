// lbm_forward.hip -- forward kernels of liblbm_hip for gfx950 (MI355X).
//
// One launch of k_step advances every cell of one grid by one forward-Euler
// step of the D2V19 FDLB model (Eq. (47) of arXiv:1010.4124); the tile body
// is in lbm_step.h. Tiles map to workgroups (G wavefronts each) XCD-major:
// hardware dispatches consecutive workgroups round-robin over the 8 XCDs, so
// workgroup b takes work item (b % 8) * per_xcd + b / 8 and every XCD sweeps
// one contiguous stretch of the strip walk (strip_walk), whose tiles' halos
// then meet in that XCD's L2. The
// per-context constants travel by value in the kernel arguments and are read
// with scalar loads.
//
// The remaining kernels here are the cell-parallel helpers: f^eq
// initialisation, side equilibria, moments and the kinetic-energy reduction.
#include "lbm_device.h"
#include "lbm_fast.h"
#include "lbm_internal.h"
#include "lbm_stage.h"
#include "lbm_step.h"

namespace lbmd {

struct StepArgs {
    StepGrid s;
    double* __restrict__ ke_part;  // [ntiles][2] or null
    const double* __restrict__ m_in;  // carried moment sums [4][ny][nx] (M variants)
    double* __restrict__ m_out;
    int tiles_y;
    int nwork, per_xcd;  // work items: tiles (M = 1) or tiles x groups (M = 0, 2)
    int nband;           // M = 3: work items [0, nband) are the tiles around `rect`
    FastRect rect;       // M = 3: the rectangle of fast tiles
    int own_sums;        // M = 3: fast tiles form the sums of f themselves
    Consts k;
};

template <int R, int G, int W, int DEPTH, bool NT, int MODE>
__global__ __launch_bounds__((64 * Waves<G, MODE>::N)) __attribute__((amdgpu_waves_per_eu(W)))
void k_step(StepArgs a)
{
    __shared__ double lds[Waves<G, MODE>::N * WaveLds<R, MODE>::SIZE];

    const int b = blockIdx.x;
    const int work = (b & 7) * a.per_xcd + (b >> 3);
    if (work >= a.nwork) return;
    constexpr int GW = MODE == PH_CARRY ? 1 : G;  // groups per work item's tile index
    const int pos = work / GW, grp = work - pos * GW;
    const int tile = strip_walk(pos, a.s.tiles_x, a.tiles_y);
    step_work<R, G, DEPTH, NT, MODE>(a.s, a.k, SideEqConsts{}, tile, grp,
                                   a.ke_part ? a.ke_part + 2 * tile : nullptr, lds, a.m_in,
                                   a.m_out);
}

// The M = 3 variants (lbm_fast.h): the first nband work items are the tiles
// around the rectangle of fast tiles, advanced by the PH_CARRY tile body
// (dispatched first, so that their longer path overlaps the rest); the
// others walk the rectangle in strips with the fast-tile body. XCD-major as
// in k_step. One launch covers the grid.
template <int R, int W, int DEPTH, bool NT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(W))) void k_step_fast(StepArgs a)
{
    constexpr int NL = FastStage<R>::LDS > WaveLds<R, PH_CARRY>::SIZE ? FastStage<R>::LDS
                                                                     : WaveLds<R, PH_CARRY>::SIZE;
    __shared__ double lds[NL];

    const int b = blockIdx.x;
    const int work = (b & 7) * a.per_xcd + (b >> 3);
    if (work >= a.nwork) return;
    const FastRect& f = a.rect;
    if (work < a.nband) {
        const int tile = band_tile(work, f, a.s.tiles_x, a.tiles_y);
        step_work<R, 1, DEPTH, NT, PH_CARRY>(a.s, a.k, SideEqConsts{}, tile, 0,
                                             a.ke_part ? a.ke_part + 2 * tile : nullptr, lds,
                                             a.m_in, a.m_out);
        return;
    }
    const int cols = f.c1 - f.c0, rows = f.r1 - f.r0;
    const int t = strip_walk<FAST_STRIP>(work - a.nband, cols, rows);
    const int ty = t / cols, tx = t - ty * cols;
    const int tile = (f.r0 + ty) * a.s.tiles_x + f.c0 + tx;
    // the host's rectangle holds fast tiles only; never stage another here
    if (!fast_tile(grid_bc(a.s), (f.c0 + tx) * TX, (f.r0 + ty) * R, TX, R, HALO)) return;
    fast_tile_work<R, DEPTH, NT>(a.s, a.k, tile, a.ke_part ? a.ke_part + 2 * tile : nullptr, lds,
                                 a.m_in, a.m_out, a.own_sums != 0);
}

// Moment sums of the cells of the band tiles around a FastRect (work item w
// = blockIdx.x, tiles of 64 x R cells), as k_sums forms them: the input sums
// of a fast-tile step whose fast tiles form their own.
__global__ __launch_bounds__(64) void k_sums_band(const double* __restrict__ f,
                                                  double* __restrict__ m, int nx, int ny, int R,
                                                  FastRect rect, int tiles_x, int tiles_y,
                                                  Consts k)
{
    const int tile = band_tile(blockIdx.x, rect, tiles_x, tiles_y);
    const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
    const int x = tx * TX + (int)threadIdx.x;
    if (x >= nx) return;
    const int64_t n = (int64_t)nx * ny;
    for (int r = 0; r < R; ++r) {
        const int y = ty * R + r;
        if (y >= ny) break;
        const int64_t c = (int64_t)y * nx + x;
        double rho = 0.0, jx = 0.0, jy = 0.0, E = 0.0;
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const double fi = f[i * n + c];
            rho += fi;
            jx = __builtin_fma(fi, k.vx[i], jx);
            jy = __builtin_fma(fi, k.vy[i], jy);
            E = __builtin_fma(fi, k.hv2[i], E);
        }
        m[c] = rho;
        m[n + c] = jx;
        m[2 * n + c] = jy;
        m[3 * n + c] = E;
    }
}

// State pass of the PH_STATE variants, one thread per cell (state_block).
__global__ __launch_bounds__(256) void k_state(const double* __restrict__ f,
                                               double* __restrict__ fout,
                                               double* __restrict__ st, int64_t n, double ct,
                                               int ke_axis, double* __restrict__ part, Consts k,
                                               Ghosts gh)
{
    __shared__ double sr[8];
    state_block(f, fout, st, n, ct, ke_axis, part, k, blockIdx.x, sr, gh);
}

// Moment sums rho, j_x, j_y, E (Eq. (10)) per cell, in the order the step
// kernels accumulate them: the state a carried-moment step starts from.
__global__ void k_sums(const double* __restrict__ f, double* __restrict__ m, int64_t n, Consts k)
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
    m[c] = r;
    m[n + c] = jx;
    m[2 * n + c] = jy;
    m[3 * n + c] = E;
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

// Outflow ghosts of one grid (outflow_point), blockIdx.y = side.
__global__ __launch_bounds__(256) void k_outflow(const double* __restrict__ f, int nx, int ny,
                                                 double* g0, double* g1, double* g2, double* g3,
                                                 Consts k)
{
    const int side = blockIdx.y;
    double* g = side == 0 ? g0 : side == 1 ? g1 : side == 2 ? g2 : g3;
    if (g) outflow_point(f, nx, ny, g, side, blockIdx.x * 256 + threadIdx.x, k);
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

// Counters of the state check: cells found non-finite and non-physical, and
// the smallest index of each kind (all ones: none).
__global__ void k_check_clear(unsigned long long* cnt)
{
    if (threadIdx.x < 4) cnt[threadIdx.x] = threadIdx.x < 2 ? 0ull : ~0ull;
}

// State check, one thread per cell: the moments of Eq. (10) must be finite
// and have rho > 0, T > 0. Per wave, one atomic per counter: the number of
// offending lanes and the first offending cell (lanes hold consecutive cells).
__global__ __launch_bounds__(256) void k_check(const double* __restrict__ f, int64_t n, Consts k,
                                               unsigned long long* cnt)
{
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    bool bad = false, unphys = false;
    if (c < n) {
        double r = 0.0, jx = 0.0, jy = 0.0, E = 0.0;
        bool fin = true;
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const double fi = f[i * n + c];
            fin = fin && isfinite(fi);
            r += fi;
            jx = __builtin_fma(fi, k.vx[i], jx);
            jy = __builtin_fma(fi, k.vy[i], jy);
            E = __builtin_fma(fi, k.hv2[i], E);
        }
        const double ux = jx / r, uy = jy / r;
        const double T = E / r - 0.5 * (ux * ux + uy * uy);
        fin = fin && isfinite(r) && isfinite(ux) && isfinite(uy) && isfinite(T);
        bad = !fin;
        unphys = fin && !(r > 0.0 && T > 0.0);
    }
    const unsigned long long mb = __ballot(bad), mp = __ballot(unphys);
    if ((threadIdx.x & 63) == 0) {
        const unsigned long long w0 = (unsigned long long)(c);  // lane 0's cell
        if (mb) {
            atomicAdd(&cnt[0], (unsigned long long)__popcll(mb));
            atomicMin(&cnt[2], w0 + (unsigned long long)(__ffsll((long long)mb) - 1));
        }
        if (mp) {
            atomicAdd(&cnt[1], (unsigned long long)__popcll(mp));
            atomicMin(&cnt[3], w0 + (unsigned long long)(__ffsll((long long)mp) - 1));
        }
    }
}

// Kinetic energy partials of rho u_n^2 / 2 (u_n = u_y, or u_x with ke_axis):
// one (sum, max) pair per block of 256 cells.
__global__ __launch_bounds__(256) void k_kinetic_part(const double* __restrict__ f, int64_t n,
                                                      int ke_axis, double* __restrict__ part,
                                                      Consts k)
{
    __shared__ double sr[8];
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double e = 0.0;
    if (c < n) {
        double r = 0.0, jn = 0.0;
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const double fi = f[i * n + c];
            r += fi;
            jn = __builtin_fma(fi, ke_axis ? k.vx[i] : k.vy[i], jn);
        }
        const double un = jn / r;
        e = 0.5 * r * un * un;
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

// Deterministic final reduction of n (sum, max) partials per row, one
// workgroup per row: row b starts at part + b * stride and its result goes to
// out2[2b], out2[2b+1]; out2[2b] is scaled by dxdy.
__global__ __launch_bounds__(256) void k_reduce_pairs(const double* __restrict__ part, int n,
                                                      int64_t stride, double dxdy,
                                                      double* __restrict__ out2)
{
    __shared__ double sr[8];
    part += blockIdx.x * stride;
    out2 += 2 * blockIdx.x;
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
struct StepVariant {
    int R, G, W, D, NT, M;
    void (*kernel)(StepArgs);
};

template <int R, int G, int W, int D, bool NT, int M>
struct StepKernel {
    static constexpr void (*fn)(StepArgs) = k_step<R, G, W, D, NT, M>;
};
template <int R, int G, int W, int D, bool NT>
struct StepKernel<R, G, W, D, NT, PH_FAST> {
    static_assert(G == 1, "the fast-tile kernel advances all 18 velocities in one wave");
    static constexpr void (*fn)(StepArgs) = k_step_fast<R, W, D, NT>;
};

#define LBM_SINGLE_VARIANT(R, G, W, D, NT, M, WB) \
    {R, G, W, D, NT, M, StepKernel<R, G, W, D, NT, M>::fn},
static const StepVariant kStepVariants[] = {LBM_STEP_VARIANTS(LBM_SINGLE_VARIANT)};
#undef LBM_SINGLE_VARIANT
constexpr int kNumStepVariants = sizeof(kStepVariants) / sizeof(kStepVariants[0]);

int step_variant_count() { return kNumStepVariants; }
int step_variant_desc(int v, int info[6])
{
    if (v < 0 || v >= kNumStepVariants) return -1;
    const StepVariant& V = kStepVariants[v];
    info[0] = V.R;
    info[1] = V.G;
    info[2] = V.W;
    info[3] = V.D;
    info[4] = V.NT;
    info[5] = V.M;
    return 0;
}

int step_ntiles(int variant, int nx, int ny)
{
    const StepVariant& V = kStepVariants[variant];
    return ((nx + TX - 1) / TX) * ((ny + V.R - 1) / V.R);
}

hipError_t launch_step(int variant, const double* fin, double* fout, const Consts& k,
                       double* ke_part, int nx, int ny, const int bc[4], double cx, double cy,
                       double ct, int ke_axis, const double* const gb[4], const double* m_in,
                       double* m_out, hipStream_t st, bool own_sums)
{
    const StepVariant& V = kStepVariants[variant];
    if (own_sums && V.M != PH_FAST) {
        // only the fast-tile kernel forms sums in its tiles: the sums pass
        hipError_t e = launch_sums(fin, const_cast<double*>(m_in), k, (int64_t)nx * ny, st);
        if (e != hipSuccess) return e;
        own_sums = false;
    }
    StepArgs a;
    a.s.fin = fin;
    a.s.fout = fout;
    a.s.nx = nx;
    a.s.ny = ny;
    a.s.ke_axis = ke_axis;
    for (int j = 0; j < 4; ++j) {
        a.s.bc[j] = bc[j];
        a.s.gb[j] = gb ? gb[j] : nullptr;
    }
    a.s.tiles_x = (nx + TX - 1) / TX;
    a.s.cx = cx;
    a.s.cy = cy;
    a.s.ct = ct;
    a.ke_part = ke_part;
    a.m_in = m_in;
    a.m_out = m_out;
    a.tiles_y = (ny + V.R - 1) / V.R;
    a.k = k;
    a.nband = 0;
    a.own_sums = 0;
    a.rect = FastRect{0, 0, a.tiles_y, a.tiles_y};
    if (V.M == PH_FAST) {
        // the tiles around the rectangle of fast tiles first, then the
        // rectangle: every tile once
        a.rect = fast_rect(nx, ny, bc[XLO], V.R);
        a.nband = band_count(a.rect, a.s.tiles_x, a.tiles_y);
        a.nwork = a.nband + (a.rect.c1 - a.rect.c0) * (a.rect.r1 - a.rect.r0);
        a.per_xcd = (a.nwork + 7) / 8;
        if (own_sums) {
            // the band tiles read their sums from m_in: form those first
            if (a.nband > 0) {
                hipLaunchKernelGGL(k_sums_band, dim3(a.nband), dim3(64), 0, st, fin,
                                   const_cast<double*>(m_in), nx, ny, V.R, a.rect, a.s.tiles_x,
                                   a.tiles_y, k);
                hipError_t e = hipGetLastError();
                if (e != hipSuccess) return e;
            }
            a.own_sums = 1;
        }
        hipLaunchKernelGGL(V.kernel, dim3(8 * a.per_xcd), dim3(64), 0, st, a);
        return hipGetLastError();
    }
    a.nwork = a.s.tiles_x * a.tiles_y * (V.M == PH_CARRY ? 1 : V.G);
    a.per_xcd = (a.nwork + 7) / 8;
    hipLaunchKernelGGL(V.kernel, dim3(8 * a.per_xcd), dim3(64 * (V.M == PH_CARRY ? V.G : 1)), 0,
                       st, a);
    return hipGetLastError();
}

hipError_t launch_outflow(const double* f, int nx, int ny, double* const g[4], const Consts& k,
                          hipStream_t st)
{
    const int len = nx > ny ? nx : ny;
    hipLaunchKernelGGL(k_outflow, dim3((len + 255) / 256, 4), dim3(256), 0, st, f, nx, ny, g[0],
                       g[1], g[2], g[3], k);
    return hipGetLastError();
}

hipError_t launch_state(const double* f, double* fout, double* state, int nx, int ny, double ct,
                        int ke_axis, double* part, int* nparts, const Consts& k,
                        double* const gb[4], hipStream_t st)
{
    const int64_t n = (int64_t)nx * ny;
    const int64_t blocks = (n + 255) / 256;
    *nparts = (int)blocks;
    Ghosts gh;
    for (int q = 0; q < 4; ++q) gh.g[q] = gb ? gb[q] : nullptr;
    gh.nx = nx;
    gh.ny = ny;
    hipLaunchKernelGGL(k_state, dim3((unsigned)blocks), dim3(256), 0, st, f, fout, state, n, ct,
                       ke_axis, part, k, gh);
    return hipGetLastError();
}

hipError_t launch_sums(const double* f, double* m, const Consts& k, int64_t n, hipStream_t st)
{
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_sums, dim3((unsigned)blocks), dim3(256), 0, st, f, m, n, k);
    return hipGetLastError();
}

hipError_t launch_reduce_pairs(const double* part, int n, int rows, int64_t stride, double dxdy,
                               double* out2, hipStream_t st)
{
    hipLaunchKernelGGL(k_reduce_pairs, dim3((unsigned)rows), dim3(256), 0, st, part, n, stride,
                       dxdy, out2);
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

hipError_t launch_check(const double* f, const Consts& k, int64_t n, unsigned long long* cnt,
                        hipStream_t st)
{
    hipLaunchKernelGGL(k_check_clear, dim3(1), dim3(64), 0, st, cnt);
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_check, dim3((unsigned)blocks), dim3(256), 0, st, f, n, k, cnt);
    return hipGetLastError();
}

hipError_t launch_kinetic_part(const double* f, const Consts& k, int64_t n, int ke_axis,
                               double* part, int* nparts, hipStream_t st)
{
    const int64_t blocks = (n + 255) / 256;
    *nparts = (int)blocks;
    hipLaunchKernelGGL(k_kinetic_part, dim3((unsigned)blocks), dim3(256), 0, st, f, n, ke_axis,
                       part, k);
    return hipGetLastError();
}

}  // namespace lbmd
