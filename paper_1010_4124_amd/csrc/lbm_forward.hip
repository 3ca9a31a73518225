// lbm_forward.hip -- forward kernels of liblbm_hip for gfx950 (MI355X).
//
// One launch of k_step advances every cell of the grid by one forward-Euler
// step of the D2V19 FDLB model (Eq. (47) of arXiv:1010.4124). A workgroup of
// NW wavefronts owns a tile of 64 x (R*NW) cells; each wavefront owns 64
// columns x R rows and each lane a column strip of R cells.
//
//   phase 1  every lane loads the 19 values of its R cells, forms the
//            moments of Eq. (10) and keeps rho, T, u/T and 1-u^2/2T in
//            registers; the rest particle is relaxed and stored at once.
//   phase 2  for each moving velocity i = 1..18:
//            - the tile's plane f_i plus a 3-cell cross-shaped halo (ghosts
//              from the boundary rule) is staged in LDS; the plane after it
//              is already in flight into registers (software pipeline);
//            - x pass: lanes re-map to row strips of R cells and compute the
//              R+1 WENO faces of their strip once, sharing first and second
//              differences between faces; flux differences go to LDS;
//            - y pass (v_iy != 0): lanes compute the R+1 faces of their
//              column strip in registers;
//            - each lane combines convection, BGK relaxation toward f^eq and
//              the Euler update, and stores f_i^{n+1} (coalesced along x).
//
// Tiles are assigned XCD-major: consecutive workgroups are dispatched
// round-robin over the 8 XCDs, so workgroup b takes tile
// (b % 8) * per_xcd + b / 8 and every XCD sweeps one contiguous band of
// tiles whose halos then meet in that XCD's L2.
#include "lbm_device.h"

namespace lbmd {

constexpr int TX = 64;
constexpr int PITCH = 71;   // LDS row pitch of a staged plane (odd: no bank conflicts)
constexpr int XPITCH = 65;  // LDS row pitch of the x flux differences

struct StepArgs {
    const double* __restrict__ fin;
    double* __restrict__ fout;
    const Model* __restrict__ M;
    double* __restrict__ ke_part;  // [ntiles][2] or null
    int nx, ny;
    int bc0, bc1, bc2, bc3;
    int tiles_x, ntiles, per_xcd;
    double cx, cy, ct;  // dt/dx, dt/dy, dt/tau
};

__device__ __forceinline__ int side_bc(const StepArgs& a, int s)
{
    return s == 0 ? a.bc0 : s == 1 ? a.bc1 : s == 2 ? a.bc2 : a.bc3;
}

// Value of plane i at (gx, gy) for a position inside the domain or in the
// three-cell ghost layer of one side (never a corner for an active cell).
__device__ __forceinline__ double ghost_or_value(const StepArgs& a, int i, int gx, int gy,
                                                 int64_t plane)
{
    const bool inx = (unsigned)gx < (unsigned)a.nx;
    const bool iny = (unsigned)gy < (unsigned)a.ny;
    const Model* M = a.M;
    if (inx && iny) return a.fin[i * plane + (int64_t)gy * a.nx + gx];
    if (inx == iny) return 0.0;  // corner or beyond: never read by an active cell
    if (!inx) {
        const int side = gx < 0 ? XLO : XHI;
        const int m = gx < 0 ? -1 - gx : gx - a.nx;
        if (m >= HALO) return 0.0;
        const int bc = side_bc(a, side);
        if (bc == PERIODIC)
            return a.fin[i * plane + (int64_t)gy * a.nx + wrap_index(gx, a.nx)];
        if (bc == FIXED_EQ) return M->side_eq[side][i];
        // reflect: interior cell m of the x-mirrored velocity
        return a.fin[M->mirx[i] * plane + (int64_t)gy * a.nx + (gx < 0 ? m : a.nx - 1 - m)];
    }
    const int side = gy < 0 ? YLO : YHI;
    const int m = gy < 0 ? -1 - gy : gy - a.ny;
    if (m >= HALO) return 0.0;
    const int bc = side_bc(a, side);
    if (bc == PERIODIC)
        return a.fin[i * plane + (int64_t)wrap_index(gy, a.ny) * a.nx + gx];
    if (bc == FIXED_EQ) return M->side_eq[side][i];
    return a.fin[M->miry[i] * plane + (int64_t)(gy < 0 ? m : a.ny - 1 - m) * a.nx + gx];
}

// Staged region of a tile: TY rows of 70 (64 + 2*3 halo columns), then six
// halo rows of 64 (three above, three below).
template <int TY>
struct Stage {
    static constexpr int NEX = TY * (TX + 2 * HALO);
    static constexpr int NE = NEX + 2 * HALO * TX;
    __device__ static __forceinline__ void pos(int e, int& ly, int& lx)
    {
        if (e < NEX) {
            ly = e / (TX + 2 * HALO);
            lx = e - ly * (TX + 2 * HALO) - HALO;
        } else {
            const int e2 = e - NEX;
            const int hr = e2 / TX;
            lx = e2 - hr * TX;
            ly = hr < HALO ? hr - HALO : TY + hr - HALO;
        }
    }
};

template <int TY, int NT, int NPRE>
__device__ __forceinline__ void stage_load(const StepArgs& a, int i, int x0, int y0, bool interior,
                                           int64_t plane, double (&pre)[NPRE])
{
    const int tid = threadIdx.x;
#pragma unroll
    for (int j = 0; j < NPRE; ++j) {
        const int e = tid + j * NT;
        double v = 0.0;
        if (e < Stage<TY>::NE) {
            int ly, lx;
            Stage<TY>::pos(e, ly, lx);
            const int gx = x0 + lx, gy = y0 + ly;
            if (interior)
                v = a.fin[i * plane + (int64_t)gy * a.nx + gx];
            else
                v = ghost_or_value(a, i, gx, gy, plane);
        }
        pre[j] = v;
    }
}

template <int TY, int NT, int NPRE>
__device__ __forceinline__ void stage_store(double* s_pl, const double (&pre)[NPRE])
{
    const int tid = threadIdx.x;
#pragma unroll
    for (int j = 0; j < NPRE; ++j) {
        const int e = tid + j * NT;
        if (e < Stage<TY>::NE) {
            int ly, lx;
            Stage<TY>::pos(e, ly, lx);
            s_pl[(ly + HALO) * PITCH + lx + HALO] = pre[j];
        }
    }
}

// x pass: lane -> (row r = lane % R, strip s = lane / R) of this wave's R rows.
template <int R, bool NEG>
__device__ __forceinline__ void x_pass(const double* s_pl, double* s_dx, int w, int lane, double v,
                                       double eps)
{
    const int r = lane % R, s = lane / R;
    const int row = w * R + r;
    const double* b = s_pl + (row + HALO) * PITCH + s * R;
    double P[R + 5];
#pragma unroll
    for (int k = 0; k < R + 5; ++k) P[k] = v * (NEG ? b[R + 5 - k] : b[k]);
    double hq[R + 1];
    weno_faces<R>(P, eps, hq);
    double* out = s_dx + row * XPITCH + s * R;
#pragma unroll
    for (int m = 0; m < R; ++m) out[m] = NEG ? (hq[R - m - 1] - hq[R - m]) : (hq[m + 1] - hq[m]);
}

// y pass: lane = column, R rows of this wave. Also returns the centre values.
template <int R, bool NEG>
__device__ __forceinline__ void y_pass(const double* s_pl, int w, int lane, double v, double eps,
                                       double (&dhy)[R], double (&fc)[R])
{
    const double* col = s_pl + lane + HALO;
    double fw[R + 5];
#pragma unroll
    for (int k = 0; k < R + 5; ++k) fw[k] = NEG ? col[(w * R + R + 5 - k) * PITCH] : col[(w * R + k) * PITCH];
#pragma unroll
    for (int m = 0; m < R; ++m) fc[m] = NEG ? fw[R + 2 - m] : fw[m + 3];
    double P[R + 5];
#pragma unroll
    for (int k = 0; k < R + 5; ++k) P[k] = v * fw[k];
    double hq[R + 1];
    weno_faces<R>(P, eps, hq);
#pragma unroll
    for (int m = 0; m < R; ++m) dhy[m] = NEG ? (hq[R - m - 1] - hq[R - m]) : (hq[m + 1] - hq[m]);
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

template <int R, int NW>
__global__ __launch_bounds__(64 * NW) void k_step(StepArgs a)
{
    constexpr int TY = R * NW;
    constexpr int NT = 64 * NW;
    constexpr int NPRE = (Stage<TY>::NE + NT - 1) / NT;
    __shared__ double s_pl[(TY + 2 * HALO) * PITCH];
    __shared__ double s_dx[TY * XPITCH];
    __shared__ double s_red[2 * NW];

    const int b = blockIdx.x;
    const int tile = (b & 7) * a.per_xcd + (b >> 3);
    if (tile >= a.ntiles) return;  // uniform over the workgroup
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int ty = tile / a.tiles_x, tx = tile - ty * a.tiles_x;
    const int x0 = tx * TX, y0 = ty * TY;
    const int64_t plane = (int64_t)a.nx * a.ny;
    const Model* M = a.M;
    const bool interior =
        x0 >= HALO && x0 + TX + HALO <= a.nx && y0 >= HALO && y0 + TY + HALO <= a.ny;
    const int gx = x0 + lane;

    // ---- phase 1: moments, equilibrium data, rest particle, diagnostics ----
    double rho[R], Tm[R], uxt[R], uyt[R], t0[R];
    double ke_s = 0.0, ke_m = 0.0;
#pragma unroll
    for (int m = 0; m < R; ++m) {
        const int gy = y0 + w * R + m;
        const bool act = gx < a.nx && gy < a.ny;
        double r = 1.0, jx = 0.0, jy = 0.0, E = 1.0, fz = 0.0;
        if (act) {
            const double* p = a.fin + (int64_t)gy * a.nx + gx;
            r = 0.0;
            E = 0.0;
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                const double fi = p[i * plane];
                if (i == 0) fz = fi;
                r += fi;
                jx = __builtin_fma(fi, M->vx[i], jx);
                jy = __builtin_fma(fi, M->vy[i], jy);
                E = __builtin_fma(fi, M->hv2[i], E);
            }
        }
        const CellEq c = cell_eq_from_sums(r, jx, jy, E);
        rho[m] = c.rho;
        Tm[m] = c.T;
        uxt[m] = c.uxt;
        uyt[m] = c.uyt;
        t0[m] = c.t0;
        if (act) {
            const double uy = jy / r;
            const double e = 0.5 * r * uy * uy;
            ke_s += e;
            ke_m = fmax(ke_m, e);
            // rest particle: no convection, f^eq_0 = rho F_0 (1 - u^2/2T)
            const double F0 = 1.0 - 6.0 * (weight_k(M, 0, c.T) + weight_k(M, 1, c.T) +
                                            weight_k(M, 2, c.T));
            const double fe = c.rho * F0 * c.t0;
            a.fout[(int64_t)gy * a.nx + gx] = __builtin_fma(-a.ct, fz - fe, fz);
        }
    }
    if (a.ke_part) {
        ke_s = wave_sum(ke_s);
        ke_m = wave_max(ke_m);
        if (lane == 0) {
            s_red[2 * w] = ke_s;
            s_red[2 * w + 1] = ke_m;
        }
    }

    // ---- phase 2: the 18 moving velocities ----
    double pre[NPRE];
    stage_load<TY, NT, NPRE>(a, 1, x0, y0, interior, plane, pre);
    double A[R];
#pragma unroll 1
    for (int i = 1; i < NV; ++i) {
        const int k = (i - 1) / 6;
        if (i == 1 || i == 7 || i == 13) {
#pragma unroll
            for (int m = 0; m < R; ++m) A[m] = rho[m] * weight_k(M, k, Tm[m]);
        }
        stage_store<TY, NT, NPRE>(s_pl, pre);
        __syncthreads();
        if (i == 1 && a.ke_part && threadIdx.x == 0) {
            double s = 0.0, mx = 0.0;
            for (int q = 0; q < NW; ++q) {
                s += s_red[2 * q];
                mx = fmax(mx, s_red[2 * q + 1]);
            }
            a.ke_part[2 * tile] = s;
            a.ke_part[2 * tile + 1] = mx;
        }
        if (i + 1 < NV) stage_load<TY, NT, NPRE>(a, i + 1, x0, y0, interior, plane, pre);

        const double vx = M->vx[i], vy = M->vy[i], eps = M->eps;
        if (vx < 0.0)
            x_pass<R, true>(s_pl, s_dx, w, lane, vx, eps);
        else
            x_pass<R, false>(s_pl, s_dx, w, lane, vx, eps);
        double dhy[R], fc[R];
        if (vy > 0.0) {
            y_pass<R, false>(s_pl, w, lane, vy, eps, dhy, fc);
        } else if (vy < 0.0) {
            y_pass<R, true>(s_pl, w, lane, vy, eps, dhy, fc);
        } else {
#pragma unroll
            for (int m = 0; m < R; ++m) {
                fc[m] = s_pl[(w * R + m + HALO) * PITCH + lane + HALO];
                dhy[m] = 0.0;
            }
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < R; ++m) {
            const int gy = y0 + w * R + m;
            const double dhx = s_dx[(w * R + m) * XPITCH + lane];
            const double eta = __builtin_fma(vx, uxt[m], vy * uyt[m]);
            const double fe = A[m] * feq_poly(eta, t0[m]);
            double fn = __builtin_fma(-a.cx, dhx, fc[m]);
            fn = __builtin_fma(-a.cy, dhy[m], fn);
            fn = __builtin_fma(-a.ct, fc[m] - fe, fn);
            if (gx < a.nx && gy < a.ny) a.fout[i * plane + (int64_t)gy * a.nx + gx] = fn;
        }
    }
}

// ---------------------------------------------------------------------------
// f = f^eq(rho, u, T), one thread per cell (Eq. (28)).
__global__ void k_init(const double* __restrict__ rho, const double* __restrict__ ux,
                       const double* __restrict__ uy, const double* __restrict__ T,
                       double* __restrict__ f, const Model* __restrict__ M, int64_t n)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const double r = rho[c], u = ux[c], v = uy[c], t = T[c];
    const double iT = 1.0 / t;
    const double t0 = 1.0 - (u * u + v * v) / (2.0 * t);
    const double uxt = u * iT, uyt = v * iT;
    double A[4];
    A[1] = r * weight_k(M, 0, t);
    A[2] = r * weight_k(M, 1, t);
    A[3] = r * weight_k(M, 2, t);
    A[0] = r * (1.0 - 6.0 * (weight_k(M, 0, t) + weight_k(M, 1, t) + weight_k(M, 2, t)));
    f[c] = A[0] * t0;
#pragma unroll
    for (int i = 1; i < NV; ++i) {
        const double eta = __builtin_fma(M->vx[i], uxt, M->vy[i] * uyt);
        f[i * n + c] = A[1 + (i - 1) / 6] * feq_poly(eta, t0);
    }
}

// Fixed-side equilibria: four (rho, ux, uy, T) states -> M->side_eq.
__global__ void k_side_eq(Model* M, double4 s0, double4 s1, double4 s2, double4 s3)
{
    const int i = threadIdx.x;
    const int s = blockIdx.x;
    if (i >= NV || s >= 4) return;
    const double4 st = s == 0 ? s0 : s == 1 ? s1 : s == 2 ? s2 : s3;
    const double r = st.x, u = st.y, v = st.z, t = st.w;
    if (!(r > 0.0) || !(t > 0.0)) {
        M->side_eq[s][i] = 0.0;
        return;
    }
    const double iT = 1.0 / t;
    const double t0 = 1.0 - (u * u + v * v) / (2.0 * t);
    double A;
    if (i == 0)
        A = r * (1.0 - 6.0 * (weight_k(M, 0, t) + weight_k(M, 1, t) + weight_k(M, 2, t)));
    else
        A = r * weight_k(M, (i - 1) / 6, t);
    const double eta = __builtin_fma(M->vx[i], u * iT, M->vy[i] * (v * iT));
    M->side_eq[s][i] = A * feq_poly(eta, t0);
}

// Moments of Eq. (10) per cell.
__global__ void k_moments(const double* __restrict__ f, double* __restrict__ rho,
                          double* __restrict__ ux, double* __restrict__ uy,
                          double* __restrict__ T, const Model* __restrict__ M, int64_t n)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    double r = 0.0, jx = 0.0, jy = 0.0, E = 0.0;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        const double fi = f[i * n + c];
        r += fi;
        jx = __builtin_fma(fi, M->vx[i], jx);
        jy = __builtin_fma(fi, M->vy[i], jy);
        E = __builtin_fma(fi, M->hv2[i], E);
    }
    const double u = jx / r, v = jy / r;
    rho[c] = r;
    ux[c] = u;
    uy[c] = v;
    T[c] = E / r - 0.5 * (u * u + v * v);
}

// Transverse kinetic energy partials: one (sum, max) pair per block of 256 cells.
__global__ __launch_bounds__(256) void k_kinetic_part(const double* __restrict__ f,
                                                      const Model* __restrict__ M, int64_t n,
                                                      double* __restrict__ part)
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
            jy = __builtin_fma(fi, M->vy[i], jy);
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
// Launch table of the step kernel variants (rows per lane R, waves per
// workgroup NW).
struct StepVariant {
    int R, NW;
    void (*kernel)(StepArgs);
};

static const StepVariant kStepVariants[] = {
    {4, 4, k_step<4, 4>},
    {8, 4, k_step<8, 4>},
    {8, 2, k_step<8, 2>},
    {4, 8, k_step<4, 8>},
    {2, 8, k_step<2, 8>},
};
constexpr int kNumStepVariants = sizeof(kStepVariants) / sizeof(kStepVariants[0]);

int step_variant_count() { return kNumStepVariants; }
int step_variant_rows(int v) { return kStepVariants[v].R * kStepVariants[v].NW; }
int step_variant_desc(int v, int* R, int* NW)
{
    if (v < 0 || v >= kNumStepVariants) return -1;
    *R = kStepVariants[v].R;
    *NW = kStepVariants[v].NW;
    return 0;
}

hipError_t launch_step(int variant, const double* fin, double* fout, const Model* M,
                       double* ke_part, int nx, int ny, const int bc[4], double cx, double cy,
                       double ct, hipStream_t st)
{
    const StepVariant& V = kStepVariants[variant];
    const int TY = V.R * V.NW;
    StepArgs a;
    a.fin = fin;
    a.fout = fout;
    a.M = M;
    a.ke_part = ke_part;
    a.nx = nx;
    a.ny = ny;
    a.bc0 = bc[0];
    a.bc1 = bc[1];
    a.bc2 = bc[2];
    a.bc3 = bc[3];
    a.tiles_x = (nx + TX - 1) / TX;
    const int tiles_y = (ny + TY - 1) / TY;
    a.ntiles = a.tiles_x * tiles_y;
    a.per_xcd = (a.ntiles + 7) / 8;
    a.cx = cx;
    a.cy = cy;
    a.ct = ct;
    hipLaunchKernelGGL(V.kernel, dim3(8 * a.per_xcd), dim3(64 * V.NW), 0, st, a);
    return hipGetLastError();
}

int step_ntiles(int variant, int nx, int ny)
{
    const StepVariant& V = kStepVariants[variant];
    const int TY = V.R * V.NW;
    return ((nx + TX - 1) / TX) * ((ny + TY - 1) / TY);
}

hipError_t launch_reduce_pairs(const double* part, int n, double dxdy, double* out2,
                               hipStream_t st)
{
    hipLaunchKernelGGL(k_reduce_pairs, dim3(1), dim3(256), 0, st, part, n, dxdy, out2);
    return hipGetLastError();
}

hipError_t launch_init(const double* rho, const double* ux, const double* uy, const double* T,
                       double* f, const Model* M, int64_t n, hipStream_t st)
{
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_init, dim3((unsigned)blocks), dim3(256), 0, st, rho, ux, uy, T, f, M, n);
    return hipGetLastError();
}

hipError_t launch_side_eq(Model* M, const double s[4][4], hipStream_t st)
{
    double4 q[4];
    for (int k = 0; k < 4; ++k) q[k] = make_double4(s[k][0], s[k][1], s[k][2], s[k][3]);
    hipLaunchKernelGGL(k_side_eq, dim3(4), dim3(32), 0, st, M, q[0], q[1], q[2], q[3]);
    return hipGetLastError();
}

hipError_t launch_moments(const double* f, double* rho, double* ux, double* uy, double* T,
                          const Model* M, int64_t n, hipStream_t st)
{
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_moments, dim3((unsigned)blocks), dim3(256), 0, st, f, rho, ux, uy, T, M,
                       n);
    return hipGetLastError();
}

hipError_t launch_kinetic_part(const double* f, const Model* M, int64_t n, double* part,
                               int* nparts, hipStream_t st)
{
    const int64_t blocks = (n + 255) / 256;
    *nparts = (int)blocks;
    hipLaunchKernelGGL(k_kinetic_part, dim3((unsigned)blocks), dim3(256), 0, st, f, M, n, part);
    return hipGetLastError();
}

}  // namespace lbmd
