// lbm_device.h -- device-side constants and cell-local physics of the D2V19
// FDLB model (Gan, Xu, Zhang and Li, arXiv:1010.4124), shared by the forward,
// adjoint and batched kernels of liblbm_hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbmd {

constexpr int NV = 19;   // 1 rest + 3 speeds x 6 directions, Sec. II.A, Eq. (5)
constexpr int HALO = 3;  // WENO5 stencils reach three cells, Eqs. (49)-(51)

enum { PERIODIC = 0, FIXED_EQ = 1, REFLECT = 2, OUTFLOW = 3 };
enum { XLO = 0, XHI = 1, YLO = 2, YHI = 3 };

// Direction d = 0..5 is the angle (d+1) pi / 3. The components are exact
// tables so that sin(pi) and sin(2 pi) are exactly zero and the velocities
// on the x axis carry no y flux at all.
__host__ __device__ constexpr double dir_cos(int d)
{
    return d == 0 ? 0.5 : d == 1 ? -0.5 : d == 2 ? -1.0 : d == 3 ? -0.5 : d == 4 ? 0.5 : 1.0;
}
__host__ __device__ constexpr int dir_sin_sign(int d)
{
    return (d == 0 || d == 1) ? 1 : (d == 3 || d == 4) ? -1 : 0;
}
constexpr double SIN60 = 0.86602540378443864676;  // sqrt(3)/2
// Mirror partners: (vx, -vy) and (-vx, vy).
__host__ __device__ constexpr int mirror_y_dir(int d) { return d <= 4 ? 4 - d : 5; }
__host__ __device__ constexpr int mirror_x_dir(int d) { return (7 - d) % 6; }

// Per-context constants. They travel by value in kernel arguments, so every
// (wavefront-uniform) index into them becomes a scalar load.
struct Consts {
    double vx[NV], vy[NV];  // v_i components
    double hv2[NV];         // |v_i|^2 / 2
    // F_k(T) = T (Fc + T (Fb + T Fa)) for k = 1..3: the closed form of
    // Eqs. (44)-(46) with the constant denominator folded in.
    double Fa[3], Fb[3], Fc[3];
    double eps;             // WENO regulariser of Eq. (52)
    double side_eq[4][NV];  // f^eq of each fixed-equilibrium side
    int mirx[NV], miry[NV]; // indices of (-vx, vy) and (vx, -vy)
};

// F_k(T) of speed shell s = k-1 (Eqs. (44)-(46)).
__device__ __forceinline__ double weight_c(const Consts& k, int s, double T)
{
    return T * __builtin_fma(T, __builtin_fma(T, k.Fa[s], k.Fb[s]), k.Fc[s]);
}

// Per-cell quantities the equilibrium needs, from the raw sums of Eq. (10):
// rho = sum f, j = sum f v, E = sum f |v|^2/2; u = j / rho and
// T = E / rho - |u|^2 / 2.
struct CellEq {
    double rho, T;
    double uxt, uyt;  // u / T
    double t0;        // 1 - |u|^2 / (2T)
};

__device__ __forceinline__ CellEq cell_eq_from_sums(double r, double jx, double jy, double E)
{
    CellEq c;
    double ux = jx / r, uy = jy / r;
    double u2 = ux * ux + uy * uy;
    double T = E / r - 0.5 * u2;
    double iT = 1.0 / T;
    c.rho = r;
    c.T = T;
    c.uxt = ux * iT;
    c.uyt = uy * iT;
    c.t0 = 1.0 - u2 / (2.0 * T);
    return c;
}

// Equilibrium of Eq. (28) written in eta = (v_i . u) / T:
// f_i^eq = rho F_k [t0 + eta t0 + eta^2 / 2 + eta^3 / 6], t0 = 1 - u^2/(2T).
__device__ __forceinline__ double feq_poly(double eta, double t0)
{
    double in = __builtin_fma(eta, 1.0 / 6.0, 0.5);
    in = __builtin_fma(eta, in, t0);
    return __builtin_fma(eta, in, t0);
}

// n / d for the WENO normalisation: hardware reciprocal, two Newton steps and
// one residual correction (d is positive and far from the denormal and
// overflow ranges there).
__device__ __forceinline__ double div_nr(double n, double d)
{
    double r = __builtin_amdgcn_rcp(d);
    double e = __builtin_fma(-d, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-d, r, 1.0);
    r = __builtin_fma(r, e, r);
    double q = n * r;
    double res = __builtin_fma(-d, q, n);
    return __builtin_fma(res, r, q);
}

// WENO5-JS face fluxes along one strip of R cells (Sec. III.A, Eqs. (48)-(55)).
// P[0..R+4] are the flux samples F = v f in upwind order (for v < 0 the
// caller passes the line reversed: the paper's mirror image). hq[j],
// j = 0..R, is the numerical flux at the face between upwind-ordered strip
// cells j-1 and j, computed from P[j..j+4] = (F_{I-2}, ..., F_{I+2}).
//
// The arithmetic is that of Eqs. (48)-(55) regrouped so that the first and
// second differences of the samples are shared by the faces of the strip:
// with g_k = P_{k+1} - P_k and D_k = g_{k+1} - g_k,
//   sigma_1 = 13/12 D_j^2   + (D_j / 2 + g_{j+1})^2,
//   sigma_2 = 13/12 D_j+1^2 + ((g_{j+1} + g_{j+2}) / 2)^2,
//   sigma_3 = 13/12 D_j+2^2 + (D_{j+2} / 2 - g_{j+2})^2,
// h^q = c + r_q with r_1 = 5/6 g_{j+1} - 1/3 g_j, r_2 = 1/6 g_{j+1} + 1/3 g_{j+2},
// r_3 = 2/3 g_{j+2} - 1/6 g_{j+3}, and the weights delta_q / (eps+sigma_q)^2
// scaled by prod_p (eps+sigma_p)^2 / delta_1, so that one division per face
// remains.
template <int R>
__device__ __forceinline__ void weno_faces(const double (&P)[R + 5], double eps, double (&hq)[R + 1])
{
    double g[R + 4], D[R + 3], E[R + 3];
#pragma unroll
    for (int k = 0; k < R + 4; ++k) g[k] = P[k + 1] - P[k];
#pragma unroll
    for (int k = 0; k < R + 3; ++k) {
        D[k] = g[k + 1] - g[k];
        E[k] = (13.0 / 12.0) * D[k] * D[k];
    }
#pragma unroll
    for (int j = 0; j <= R; ++j) {
        const double b1 = __builtin_fma(0.5, D[j], g[j + 1]);
        const double b2 = 0.5 * (g[j + 1] + g[j + 2]);
        const double b3 = __builtin_fma(0.5, D[j + 2], -g[j + 2]);
        double q1 = eps + __builtin_fma(b1, b1, E[j]);
        double q2 = eps + __builtin_fma(b2, b2, E[j + 1]);
        double q3 = eps + __builtin_fma(b3, b3, E[j + 2]);
        q1 *= q1;
        q2 *= q2;
        q3 *= q3;
        const double W1 = q2 * q3;
        const double W2 = 6.0 * (q1 * q3);
        const double W3 = 3.0 * (q1 * q2);
        const double r1 = __builtin_fma(5.0 / 6.0, g[j + 1], -(1.0 / 3.0) * g[j]);
        const double r2 = __builtin_fma(1.0 / 3.0, g[j + 2], (1.0 / 6.0) * g[j + 1]);
        const double r3 = __builtin_fma(2.0 / 3.0, g[j + 2], -(1.0 / 6.0) * g[j + 3]);
        const double num = __builtin_fma(W1, r1, __builtin_fma(W2, r2, W3 * r3));
        const double den = W1 + W2 + W3;
        hq[j] = P[j + 2] + div_nr(num, den);
    }
}

__host__ __device__ __forceinline__ int wrap_index(int g, int n)
{
    int r = g % n;
    return r < 0 ? r + n : r;
}

}  // namespace lbmd
