// lbm_schemes.hip -- the comparison convection schemes of Sec. III.B of
// arXiv:1010.4124 (Fig. 2): first- and second-order upwind fluxes in the same
// forward-Euler step (Eq. (47)) as the WENO5 path.
//
// These schemes exist for the shock-width comparison, not for speed: one
// thread per cell computes the moments (Eq. (10)), relaxes the rest particle
// and, for every moving velocity, the two face fluxes per axis from the
// upwind neighbours, resolving ghost cells per neighbour with the boundary
// rules of the main path (periodic wrap, specular walls, fixed equilibria,
// outflow ghost arrays). The face flux at I+1/2 from the upwind-ordered
// samples (b, c) = (F_{I-1}, F_I) (or their mirror images for v < 0) is c
// (first order) or c + (c - b)/2 (second order).
#include "lbm_device.h"
#include "lbm_internal.h"
#include "lbm_stage.h"
#include "lbm_step.h"

namespace lbmd {

struct LoArgs {
    StepGrid s;
    double* __restrict__ ke_part;  // per 256-cell block (sum, max) or null
    Consts k;
};

// f_i at (x, y) with x or y (not both) possibly in the three ghost layers.
__device__ __forceinline__ double lo_value(const StepGrid& a, const Consts& k, int i, int x, int y)
{
    const int64_t n = (int64_t)a.nx * a.ny;
    if (x < 0 || x >= a.nx) {
        const bool lo = x < 0;
        const int m = lo ? -1 - x : x - a.nx;
        const int bc = a.bc[lo ? XLO : XHI];
        if (bc == PERIODIC) return a.fin[i * n + (int64_t)y * a.nx + wrap_index(x, a.nx)];
        if (bc == REFLECT)
            return a.fin[k.mirx[i] * n + (int64_t)y * a.nx + (lo ? m : a.nx - 1 - m)];
        if (bc == OUTFLOW) return (lo ? a.gb[XLO] : a.gb[XHI])[(int64_t)i * a.ny + y];
        return k.side_eq[lo ? XLO : XHI][i];
    }
    if (y < 0 || y >= a.ny) {
        const bool lo = y < 0;
        const int m = lo ? -1 - y : y - a.ny;
        const int bc = a.bc[lo ? YLO : YHI];
        if (bc == PERIODIC) return a.fin[i * n + (int64_t)wrap_index(y, a.ny) * a.nx + x];
        if (bc == REFLECT)
            return a.fin[k.miry[i] * n + (int64_t)(lo ? m : a.ny - 1 - m) * a.nx + x];
        if (bc == OUTFLOW) return (lo ? a.gb[YLO] : a.gb[YHI])[(int64_t)i * a.nx + x];
        return k.side_eq[lo ? YLO : YHI][i];
    }
    return a.fin[i * n + (int64_t)y * a.nx + x];
}

template <int SCHEME>
__device__ __forceinline__ double lo_face(double b, double c)
{
    return SCHEME == 1 ? c : __builtin_fma(0.5, c - b, c);
}

// h_{I+1/2} - h_{I-1/2} along one axis for velocity component v, from the
// samples F(-2..2) = v f at offsets -2..2 of the cell.
template <int SCHEME>
__device__ __forceinline__ double lo_diff(double v, const double (&F)[5])
{
    if (v >= 0.0) return lo_face<SCHEME>(F[1], F[2]) - lo_face<SCHEME>(F[0], F[1]);
    // mirror image: face I+1/2 from (F_{I+2}, F_{I+1}), face I-1/2 from (F_{I+1}, F_I)
    return lo_face<SCHEME>(F[4], F[3]) - lo_face<SCHEME>(F[3], F[2]);
}

template <int SCHEME>
__global__ __launch_bounds__(256) void k_step_lo(LoArgs a)
{
    __shared__ double sr[8];
    const StepGrid& g = a.s;
    const Consts& k = a.k;
    const int64_t n = (int64_t)g.nx * g.ny;
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double e = 0.0;
    if (c < n) {
        const int y = (int)(c / g.nx), x = (int)(c - (int64_t)y * g.nx);
        double r = 0.0, jx = 0.0, jy = 0.0, E = 0.0;
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const double fi = g.fin[i * n + c];
            r += fi;
            jx = __builtin_fma(fi, k.vx[i], jx);
            jy = __builtin_fma(fi, k.vy[i], jy);
            E = __builtin_fma(fi, k.hv2[i], E);
        }
        const CellEq q = cell_eq_from_sums(r, jx, jy, E);
        const double un = (g.ke_axis ? jx : jy) / r;
        e = 0.5 * r * un * un;
        const double F1 = weight_c(k, 0, q.T), F2 = weight_c(k, 1, q.T), F3 = weight_c(k, 2, q.T);
        const double omct = 1.0 - g.ct;
        // rest particle: no convection
        const double f0 = g.fin[c];
        const double fe0 = q.rho * (1.0 - 6.0 * (F1 + F2 + F3)) * q.t0;
        g.fout[c] = __builtin_fma(-g.ct, f0 - fe0, f0);
        for (int i = 1; i < NV; ++i) {
            const double vx = k.vx[i], vy = k.vy[i];
            double Fx[5], Fy[5];
#pragma unroll
            for (int o = 0; o < 5; ++o) {
                Fx[o] = vx == 0.0 ? 0.0 : vx * lo_value(g, k, i, x - 2 + o, y);
                Fy[o] = vy == 0.0 ? 0.0 : vy * lo_value(g, k, i, x, y - 2 + o);
            }
            const double dhx = lo_diff<SCHEME>(vx, Fx);
            const double dhy = lo_diff<SCHEME>(vy, Fy);
            const double A = (g.ct * q.rho) * (i < 7 ? F1 : i < 13 ? F2 : F3);
            const double eta = __builtin_fma(vx, q.uxt, vy * q.uyt);
            double fn = __builtin_fma(omct, g.fin[i * n + c], A * feq_poly(eta, q.t0));
            fn = __builtin_fma(-g.cx, dhx, fn);
            fn = __builtin_fma(-g.cy, dhy, fn);
            g.fout[i * n + c] = fn;
        }
    }
    if (!a.ke_part) return;
    const double s = wave_sum(e), mx = wave_max(e);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sr[2 * w] = s;
        sr[2 * w + 1] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        a.ke_part[2 * blockIdx.x] = sr[0] + sr[2] + sr[4] + sr[6];
        a.ke_part[2 * blockIdx.x + 1] = fmax(fmax(sr[1], sr[3]), fmax(sr[5], sr[7]));
    }
}

hipError_t launch_step_lo(int scheme, const double* fin, double* fout, const Consts& k,
                          double* ke_part, int* nparts, int nx, int ny, const int bc[4],
                          double cx, double cy, double ct, int ke_axis,
                          const double* const gb[4], hipStream_t st)
{
    LoArgs a;
    a.s.fin = fin;
    a.s.fout = fout;
    a.s.nx = nx;
    a.s.ny = ny;
    a.s.ke_axis = ke_axis;
    for (int j = 0; j < 4; ++j) {
        a.s.bc[j] = bc[j];
        a.s.gb[j] = gb ? gb[j] : nullptr;
    }
    a.s.tiles_x = 0;
    a.s.cx = cx;
    a.s.cy = cy;
    a.s.ct = ct;
    a.ke_part = ke_part;
    a.k = k;
    const int64_t n = (int64_t)nx * ny;
    const int64_t blocks = (n + 255) / 256;
    *nparts = (int)blocks;
    if (scheme == 1)
        hipLaunchKernelGGL(k_step_lo<1>, dim3((unsigned)blocks), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL(k_step_lo<2>, dim3((unsigned)blocks), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace lbmd
