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
    // F_k(T) = T (T (24 T - Fc4) + Fbc) / Fden for k = 1..3, the closed form
    // of Eqs. (44)-(46): Fc4 = 4 (b + c), Fbc = b c, Fden = 3 a (a - b) (a - c)
    // with a, b, c the squared speeds of shells k, k+1, k+2 (cyclic), and
    // Frden = 1 / Fden rounded to nearest.
    double Fc4[3], Fbc[3], Fden[3], Frden[3];
    double eps;             // WENO regulariser of Eq. (52)
    double epsx[NV], epsy[NV];  // eps / v_ix^2 and eps / v_iy^2 (0 where v = 0):
                                // the regulariser of WENO on f (weno_faces)
    double side_eq[4][NV];  // f^eq of each fixed-equilibrium side
    int mirx[NV], miry[NV]; // indices of (-vx, vy) and (vx, -vy)
};

// F_k(T) of speed shell s = k-1 (Eqs. (44)-(46)): the numerator in Horner
// form with its own coefficients (24, 4(b+c), bc), then the quotient by the
// denominator as P r corrected once by its residual, (P - den q) r, with r
// the rounded reciprocal. The coefficients are not divided by the
// denominator first: each would then carry a fixed rounding error, the same
// in every cell and step, which F_0 = 1 - 6 (F_1 + F_2 + F_3) amplifies and
// which a long run accumulates linearly (here ~2e-16 of f per step); the
// errors of this form vary in sign from cell to cell and step to step.
__device__ __forceinline__ double weight_c(const Consts& k, int s, double T)
{
    const double P = T * __builtin_fma(T, __builtin_fma(T, 24.0, -k.Fc4[s]), k.Fbc[s]);
    const double q = P * k.Frden[s];
    return __builtin_fma(__builtin_fma(-k.Fden[s], q, P), k.Frden[s], q);
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
    double u2 = __builtin_fma(ux, ux, uy * uy);
    double T = __builtin_fma(-0.5, u2, E / r);
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

// n / d for the WENO normalisation: the hardware reciprocal (relative error
// below 2^-24) and one residual correction, which leaves a relative error of
// order 1e-15 on the quotient; d is positive and far from the denormal and
// overflow ranges there.
__device__ __forceinline__ double div_nr(double n, double d)
{
    const double r = __builtin_amdgcn_rcp(d);
    const double q = n * r;
    const double res = __builtin_fma(-d, q, n);
    return __builtin_fma(res, r, q);
}

// WENO5-JS face fluxes along one strip of R cells (Sec. III.A, Eqs. (48)-(55)).
// P[0..R+4] are samples in upwind order (for v < 0 the caller passes the
// line reversed: the paper's mirror image). hq[j], j = 0..R, is the
// numerical flux at the face between upwind-ordered strip cells j-1 and j,
// computed from P[j..j+4] = (P_{I-2}, ..., P_{I+2}).
//
// The paper's samples are F = v f. The kernels pass f itself with eps / v^2
// in place of eps and scale the result by v: each smoothness indicator of
// v f is v^2 times that of f, so eps + sigma_q(v f) = v^2 (eps / v^2 +
// sigma_q(f)), the normalised weights are the same, and every candidate
// flux is v times that of f. The two agree exactly in real arithmetic.
//
// The arithmetic is that of Eqs. (48)-(55) regrouped so that the first and
// second differences of the samples are shared by the faces of the strip:
// with g_k = P_{k+1} - P_k and D_k = g_{k+1} - g_k,
//   eps + sigma_1 = E_j     + (D_j / 2 + g_{j+1})^2,
//   eps + sigma_2 = E_{j+1} + ((g_{j+1} + g_{j+2}) / 2)^2,
//   eps + sigma_3 = E_{j+2} + (D_{j+2} / 2 - g_{j+2})^2,   E_k = 13/12 D_k^2 + eps,
// h^q = c + r_q with r_1 = 5/6 g_{j+1} - 1/3 g_j, r_2 = 1/6 g_{j+1} + 1/3 g_{j+2},
// r_3 = 2/3 g_{j+2} - 1/6 g_{j+3}. With q_p = (eps + sigma_p)^2, the weights
// delta_p / q_p, delta = (1, 6, 3) / 10, multiplied through by 10 q_1 q_2 q_3
// leave one division per face:
//   h = c + [q_2 q_3 r_1 + q_1 (q_3 s_2 + q_2 s_3)] / [q_2 q_3 + q_1 (6 q_3 + 3 q_2)],
// s_2 = 6 r_2 = g_{j+1} + 2 g_{j+2}, s_3 = 3 r_3 = 2 g_{j+2} - g_{j+3} / 2.
// The differences are formed in a window that slides along the strip, which
// keeps few values live at a time.
template <int R, class OnFace>
__device__ __forceinline__ void weno_faces(const double (&P)[R + 5], double eps, OnFace&& on_face)
{
    constexpr double C13 = 13.0 / 12.0;
    double g0 = P[1] - P[0], g1 = P[2] - P[1], g2 = P[3] - P[2], g3 = P[4] - P[3];
    double D0 = g1 - g0, D1 = g2 - g1, D2 = g3 - g2;
    double E0 = __builtin_fma(C13 * D0, D0, eps);
    double E1 = __builtin_fma(C13 * D1, D1, eps);
    double E2 = __builtin_fma(C13 * D2, D2, eps);
#pragma unroll
    for (int j = 0; j <= R; ++j) {
        const double b1 = __builtin_fma(0.5, D0, g1);
        const double b2 = 0.5 * (g1 + g2);
        const double b3 = __builtin_fma(0.5, D2, -g2);
        double q1 = __builtin_fma(b1, b1, E0);
        double q2 = __builtin_fma(b2, b2, E1);
        double q3 = __builtin_fma(b3, b3, E2);
        q1 *= q1;
        q2 *= q2;
        q3 *= q3;
        const double W1 = q2 * q3;
        const double r1 = __builtin_fma(5.0 / 6.0, g1, -(1.0 / 3.0) * g0);
        const double s2 = __builtin_fma(2.0, g2, g1);
        const double s3 = __builtin_fma(2.0, g2, -0.5 * g3);
        const double num = __builtin_fma(q1, __builtin_fma(q3, s2, q2 * s3), W1 * r1);
        const double den = __builtin_fma(q1, __builtin_fma(6.0, q3, 3.0 * q2), W1);
        on_face(j, P[j + 2] + div_nr(num, den));
        if (j < R) {
            g0 = g1;
            g1 = g2;
            g2 = g3;
            g3 = P[j + 5] - P[j + 4];
            D0 = D1;
            D1 = D2;
            D2 = g3 - g2;
            E0 = E1;
            E1 = E2;
            E2 = __builtin_fma(C13 * D2, D2, eps);
        }
    }
}

// Flux differences of an R-cell strip as the faces of weno_faces complete:
// on_cell(m, h_{m+1/2} - h_{m-1/2}) for strip cell m in natural order, where
// NEG says the samples were passed reversed (v < 0).
template <int R, bool NEG, class OnCell>
__device__ __forceinline__ void weno_strip(const double (&P)[R + 5], double eps, OnCell&& on_cell)
{
    double hp = 0.0;
    weno_faces<R>(P, eps, [&](int j, double h) {
        if (j > 0) {
            if (NEG)
                on_cell(R - j, hp - h);
            else
                on_cell(j - 1, h - hp);
        }
        hp = h;
    });
}

__host__ __device__ __forceinline__ int wrap_index(int g, int n)
{
    int r = g % n;
    return r < 0 ? r + n : r;
}

}  // namespace lbmd

namespace lbmd {

// Reverse mode of one WENO5 face of weno_faces: for the upwind-ordered
// samples (a, b, c, d, e) = P[0..4] and the adjoint mu of the face flux,
// adds mu * dh/dP[k] to G[k]. It differentiates the same function (Eqs.
// (48)-(55)) in the same regrouped variables as the forward code.
__host__ __device__ __forceinline__ void weno_face_bar(const double* P, double eps, double mu,
                                                       double* G)
{
    constexpr double C13 = 13.0 / 12.0;
    const double g0 = P[1] - P[0], g1 = P[2] - P[1], g2 = P[3] - P[2], g3 = P[4] - P[3];
    const double D0 = g1 - g0, D1 = g2 - g1, D2 = g3 - g2;
    const double E0 = __builtin_fma(C13 * D0, D0, eps);
    const double E1 = __builtin_fma(C13 * D1, D1, eps);
    const double E2 = __builtin_fma(C13 * D2, D2, eps);
    const double b1 = __builtin_fma(0.5, D0, g1);
    const double b2 = 0.5 * (g1 + g2);
    const double b3 = __builtin_fma(0.5, D2, -g2);
    const double Q1 = __builtin_fma(b1, b1, E0);
    const double Q2 = __builtin_fma(b2, b2, E1);
    const double Q3 = __builtin_fma(b3, b3, E2);
    const double q1 = Q1 * Q1, q2 = Q2 * Q2, q3 = Q3 * Q3;
    const double W1 = q2 * q3, W2 = 6.0 * (q1 * q3), W3 = 3.0 * (q1 * q2);
    const double r1 = (5.0 / 6.0) * g1 - (1.0 / 3.0) * g0;
    const double r2 = (1.0 / 6.0) * g1 + (1.0 / 3.0) * g2;
    const double r3 = (2.0 / 3.0) * g2 - (1.0 / 6.0) * g3;
    const double iden = 1.0 / (W1 + W2 + W3);
    const double hq = (W1 * r1 + W2 * r2 + W3 * r3) * iden;  // h - c
    // h = c + (sum W_q r_q) / (sum W_q)
    const double r1b = mu * W1 * iden, r2b = mu * W2 * iden, r3b = mu * W3 * iden;
    const double W1b = mu * (r1 - hq) * iden, W2b = mu * (r2 - hq) * iden,
                 W3b = mu * (r3 - hq) * iden;
    // W1 = q2 q3, W2 = 6 q1 q3, W3 = 3 q1 q2
    const double q1b = 6.0 * W2b * q3 + 3.0 * W3b * q2;
    const double q2b = W1b * q3 + 3.0 * W3b * q1;
    const double q3b = W1b * q2 + 6.0 * W2b * q1;
    // q = Q^2, Q = b^2 + E
    const double Q1b = 2.0 * Q1 * q1b, Q2b = 2.0 * Q2 * q2b, Q3b = 2.0 * Q3 * q3b;
    const double b1b = 2.0 * b1 * Q1b, b2b = 2.0 * b2 * Q2b, b3b = 2.0 * b3 * Q3b;
    // E_k = 13/12 D_k^2 + eps
    double D0b = 2.0 * C13 * D0 * Q1b, D1b = 2.0 * C13 * D1 * Q2b, D2b = 2.0 * C13 * D2 * Q3b;
    // b1 = D0/2 + g1, b2 = (g1 + g2)/2, b3 = D2/2 - g2
    D0b += 0.5 * b1b;
    D2b += 0.5 * b3b;
    double g0b = 0.0, g1b = b1b + 0.5 * b2b, g2b = 0.5 * b2b - b3b, g3b = 0.0;
    // r's
    g1b += (5.0 / 6.0) * r1b + (1.0 / 6.0) * r2b;
    g0b -= (1.0 / 3.0) * r1b;
    g2b += (1.0 / 3.0) * r2b + (2.0 / 3.0) * r3b;
    g3b -= (1.0 / 6.0) * r3b;
    // D_k = g_{k+1} - g_k
    g1b += D0b;
    g0b -= D0b;
    g2b += D1b;
    g1b -= D1b;
    g3b += D2b;
    g2b -= D2b;
    // g_k = P_{k+1} - P_k, and c = P[2]
    G[0] += -g0b;
    G[1] += g0b - g1b;
    G[2] += g1b - g2b + mu;
    G[3] += g2b - g3b;
    G[4] += g3b;
}

}  // namespace lbmd
