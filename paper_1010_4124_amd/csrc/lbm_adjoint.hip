// lbm_adjoint.hip -- discrete adjoint of one forward-Euler step of the D2V19
// FDLB model (arXiv:1010.4124, Eq. (47)) and of the equilibrium
// initialisation, for gfx950.
//
// For the step S(f) with S_i(c) = f_i - cx dh^x_i - cy dh^y_i
// - ct (f_i - f_i^eq(m(c))), the kernel computes
//   lambda^n = (dS/df^n)^T lambda^{n+1} + w dE_y/df^n,
// E_y = sum_c rho u_y^2 / 2 dx dy, in gather form (every output is written
// once, so the result is deterministic):
//   lambda_i(c) = (1 - ct) lambda'_i(c)                          (identity, BGK)
//               + K0 + Kx v_ix + Ky v_iy + KE |v_i|^2/2           (through f^eq and
//                                                                   the objective)
//               + v_ix sum_faces mu_x dh/dF + v_iy sum_faces mu_y dh/dF  (WENO)
// where the per-cell K's hold ct sum_j lambda'_j d f_j^eq / d(rho, j, E) and
// the objective gradient, and mu of the face between cells I and I+1 is
// c (lambda'(I+1) - lambda'(I)).
//
// A one-wavefront workgroup owns a 64 x R tile and one of G groups of the 18
// moving velocities. Phase 1 forms the K's of its cells (19 values of f and
// of lambda' per cell) and group 0 writes the rest plane; in the state-pass
// variants a per-cell kernel has formed the K's and the rest plane already
// and phase 1 only reads them. Phase 2 stages, per moving velocity of the
// group, f_i with a 4-cell halo and lambda'_i
// with a 3-cell halo in LDS (lambda' is zero in ghost cells except on
// periodic axes: ghosts have no update). Each lane recomputes the R+4 faces
// whose stencils touch its R-cell strip and applies the reverse of the WENO
// face (weno_face_bar); x strips hand their sums to the column owners through
// LDS. On a reflecting wall, the ghost values of velocity i are interior
// values of its mirror j, so cells within three cells of the wall also gather
// the wall faces of plane j.
#include "lbm_device.h"
#include "lbm_fast.h"
#include "lbm_internal.h"
#include "lbm_stage.h"

namespace lbmd {

constexpr int ATX = 64;
constexpr int AP = 73;      // LDS pitch of the staged f (halo 4) and lambda (halo 3) images
constexpr int AXP = 65;     // LDS pitch of the x contributions
constexpr int FH = 4, LH = 3;

struct AdjArgs {
    const double* __restrict__ f;
    const double* __restrict__ lam1;
    double* __restrict__ lam0;
    const double* __restrict__ kst;  // K0, Kx, Ky, KE of each cell, side by side (state-pass
                                     // variants)
    int nx, ny;
    int bc[4];
    int tiles_x, tiles_y, nwork, per_xcd;
    double cx, cy, ct, wdxdy;  // w dx dy: weight of the objective term
    FastRect rect;             // marching variants: the marched tiles (64 x 4 units)
    int mh, nstrip, nchunk;    // marching variants: chunk rows, strips, chunks
    int nband, band_xcd;       // marching variants: band items (all, per XCD)
    Consts k;
};

__device__ __forceinline__ GridBC grid_of(const AdjArgs& a)
{
    return GridBC{a.nx, a.ny, {a.bc[0], a.bc[1], a.bc[2], a.bc[3]},
                  {nullptr, nullptr, nullptr, nullptr}};
}

__device__ __forceinline__ double dweight_c(const Consts& k, int s, double T)
{
    // dF_k/dT: (72 T^2 - 8 (b + c) T + b c) / den, the derivative of weight_c's
    // closed form
    return __builtin_fma(T, __builtin_fma(T, 72.0, -2.0 * k.Fc4[s]), k.Fbc[s]) * k.Frden[s];
}

// Reverse mode of one WENO5 face given its shared differences (the same
// function as weno_face_bar, Eqs. (48)-(55)): g[0..3] are the first
// differences of the face's five samples, D[0..2] the second differences,
// CD = 13/12 D and E[0..2] = 13/12 D^2 + eps. Returns in Gg[0..3]
// mu * dh/dg[k] (the centre sample's own term, mu, is added by the caller).
//
// With Q_k = b_k^2 + E (b_k the smoothness indicators' linear parts) and
// q_k = Q_k^2, the weights d_k / q_k are scaled by 10 q_1 q_2 q_3 into
// W_1 = q_2 q_3, W_2 = 6 q_1 q_3, W_3 = 3 q_1 q_2, and h = c + sum W_k r_k /
// sum W_k, r_k the candidate reconstructions less the centre sample c. The
// factors 6 and 3 are carried by the reconstructions instead (V_2 = q_1 q_3,
// rho_2 = 6 r_2, ...), and the backward sweep carries a factor 4 (m4 =
// 4 mu / sum W) that the derivative of q = (b^2 + E)^2 would otherwise
// multiply in three times; the constants of the last step take it out again.
// Fused multiply-adds throughout and 1/sum(W) from the hardware reciprocal
// and one Newton step (relative error near 2^-48).
__device__ __forceinline__ void weno_face_bar_g(const double (&g)[4], const double (&D)[3],
                                                const double (&CD)[3], const double (&E)[3],
                                                double mu, double (&Gg)[4])
{
    const double b1 = __builtin_fma(0.5, D[0], g[1]);
    const double b2 = 0.5 * (g[1] + g[2]);
    const double b3 = __builtin_fma(0.5, D[2], -g[2]);
    const double Q1 = __builtin_fma(b1, b1, E[0]);
    const double Q2 = __builtin_fma(b2, b2, E[1]);
    const double Q3 = __builtin_fma(b3, b3, E[2]);
    const double q1 = Q1 * Q1, q2 = Q2 * Q2, q3 = Q3 * Q3;
    // W_1, W_2 / 6, W_3 / 3 and r_1, 6 r_2, 3 r_3
    const double W1 = q2 * q3, V2 = q1 * q3, V3 = q1 * q2;
    const double p1 = __builtin_fma(5.0 / 6.0, g[1], -(1.0 / 3.0) * g[0]);
    const double p2 = __builtin_fma(2.0, g[2], g[1]);
    const double p3 = __builtin_fma(2.0, g[2], -0.5 * g[3]);
    const double S = __builtin_fma(6.0, V2, __builtin_fma(3.0, V3, W1));
    const double r0 = __builtin_amdgcn_rcp(S);
    const double iden = __builtin_fma(r0, __builtin_fma(-S, r0, 1.0), r0);
    const double hq = __builtin_fma(W1, p1, __builtin_fma(V2, p2, V3 * p3)) * iden;  // h - c
    const double m4 = 4.0 * (mu * iden);
    // 4 mu dh/d(p1, p2, p3) and 4 mu dh/d(W1, V2, V3)
    const double R1 = m4 * W1, R2 = m4 * V2, R3 = m4 * V3;
    const double A1 = m4 * (p1 - hq), A2 = m4 * __builtin_fma(-6.0, hq, p2),
                 A3 = m4 * __builtin_fma(-3.0, hq, p3);
    // u_k = 4 Q_k mu dh/dq_k: mu dh/db_k = b_k u_k, mu dh/dE_k = u_k / 2
    const double u1 = Q1 * __builtin_fma(A2, q3, A3 * q2);
    const double u2 = Q2 * __builtin_fma(A1, q3, A3 * q1);
    const double u3 = Q3 * __builtin_fma(A1, q2, A2 * q1);
    const double b1b = b1 * u1, b2b = b2 * u2, b3b = b3 * u3;
    // b1 = D0/2 + g1, b2 = (g1 + g2)/2, b3 = D2/2 - g2; E_k = 13/12 D_k^2 + eps
    const double D0b = __builtin_fma(CD[0], u1, 0.5 * b1b);
    const double D1b = CD[1] * u2;
    const double D2b = __builtin_fma(CD[2], u3, 0.5 * b3b);
    // p1 = 5/6 g1 - 1/3 g0, p2 = g1 + 2 g2, p3 = 2 g2 - g3 / 2 (R carries 4)
    double g1b = __builtin_fma(0.5, b2b, b1b);
    double g2b = __builtin_fma(0.5, b2b, -b3b);
    g1b = __builtin_fma(5.0 / 24.0, R1, __builtin_fma(0.25, R2, g1b));
    g2b = __builtin_fma(0.5, R2 + R3, g2b);
    // then D_k = g_{k+1} - g_k
    Gg[0] = __builtin_fma(-1.0 / 12.0, R1, -D0b);
    Gg[1] = g1b + (D0b - D1b);
    Gg[2] = g2b + (D1b - D2b);
    Gg[3] = __builtin_fma(-0.125, R3, D2b);
}

// Gather of one line strip: fw[0..R+7] are f at strip positions -4..R+3,
// lw[0..R+5] are lambda' at positions -3..R+2; returns in acc[m] the sum over
// the faces touching strip cell m of mu dh/df(m) (including the factor v).
// The faces' first and second differences and E terms slide along the strip
// as in the forward weno_faces.
template <int R, bool NEG>
__device__ __forceinline__ void gather_strip(const double (&fw)[R + 8], const double (&lw)[R + 6],
                                             double v, double cn, double eps, double (&acc)[R])
{
    constexpr double C13 = 13.0 / 12.0;
    double Pw[R + 8];
#pragma unroll
    for (int q = 0; q < R + 8; ++q) Pw[q] = v * (NEG ? fw[R + 7 - q] : fw[q]);
    // dL/dP at the R+8 upwind-ordered positions
    double Gp[R + 8];
#pragma unroll
    for (int q = 0; q < R + 8; ++q) Gp[q] = 0.0;
    double g[4] = {Pw[1] - Pw[0], Pw[2] - Pw[1], Pw[3] - Pw[2], Pw[4] - Pw[3]};
    double D[3] = {g[1] - g[0], g[2] - g[1], g[3] - g[2]};
    double E[3] = {__builtin_fma(C13 * D[0], D[0], eps), __builtin_fma(C13 * D[1], D[1], eps),
                   __builtin_fma(C13 * D[2], D[2], eps)};
#pragma unroll
    for (int t = 0; t < R + 4; ++t) {
        // face between strip positions I and I+1: I = t-2 (v >= 0) or R-t (v < 0)
        const double mu = NEG ? cn * (lw[R + 4 - t] - lw[R + 3 - t]) : cn * (lw[t + 2] - lw[t + 1]);
        double Gg[4];
        const double CD[3] = {C13 * D[0], C13 * D[1], C13 * D[2]};
        weno_face_bar_g(g, D, CD, E, mu, Gg);
        // g_k = P_{t+k+1} - P_{t+k}; the centre sample P_{t+2} adds mu
        Gp[t] -= Gg[0];
        Gp[t + 1] += Gg[0] - Gg[1];
        Gp[t + 2] += (Gg[1] - Gg[2]) + mu;
        Gp[t + 3] += Gg[2] - Gg[3];
        Gp[t + 4] += Gg[3];
        if (t + 1 < R + 4) {
            g[0] = g[1];
            g[1] = g[2];
            g[2] = g[3];
            g[3] = Pw[t + 5] - Pw[t + 4];
            D[0] = D[1];
            D[1] = D[2];
            D[2] = g[3] - g[2];
            E[0] = E[1];
            E[1] = E[2];
            E[2] = __builtin_fma(C13 * D[2], D[2], eps);
        }
    }
#pragma unroll
    for (int m = 0; m < R; ++m) acc[m] = v * Gp[NEG ? R + 3 - m : m + 4];
}

// x gather of a whole tile row, R >= 4, each face computed once. Seen from
// the upwind side (the mirrored row for v < 0: the "canonical" frame), a
// lane's strip of R cells owns the R faces between its positions t-2 and t-1,
// t = 0..R-1; their gradient reaches cells t-4..t, so every face feeds the
// owning strip and the 4 cells at the end of the strip before it. Those 4
// sums go through LDS (xl: 4 per lane) to that strip. The strip at the end
// of the row gets the same from the 4 faces of the strip beyond the tile,
// which lanes 0..4R-1 compute (one face each, xe: R x 4 x 4). A lane thus
// evaluates R + 1 faces instead of the R + 4 of gather_strip. Returns the
// sum over faces of mu dh/df for the lane's R cells (factor v included), in
// natural cell order, like gather_strip.
template <int R, bool NEG>
__device__ __forceinline__ void gather_x_row(const double* s_f, const double* s_l, double* xl,
                                             double* xe, int lane, double v, double cn,
                                             double eps, double (&acc)[R])
{
    static_assert(R >= 4 && 64 % R == 0, "a strip's neighbour covers the 4 cells a face reaches");
    constexpr double C13 = 13.0 / 12.0;
    constexpr int NS = 64 / R;
    const int r = lane % R, s = lane / R;
    const double cnc = NEG ? -cn : cn;  // mu = cnc (lambda_c(I+1) - lambda_c(I))
    // canonical position p of this strip <-> LDS column of row r
    const double* fr = s_f + (r + FH) * AP + FH;
    const double* lr = s_l + (r + LH) * AP + LH;
    auto col = [&](int p) { return NEG ? s * R + R - 1 - p : s * R + p; };
    double P[R + 4];  // v f at canonical positions -4..R-1
#pragma unroll
    for (int k = 0; k < R + 4; ++k) P[k] = v * fr[col(k - 4)];
    double Ac[R], LG[4];
#pragma unroll
    for (int m = 0; m < R; ++m) Ac[m] = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) LG[k] = 0.0;
    double g[4] = {P[1] - P[0], P[2] - P[1], P[3] - P[2], P[4] - P[3]};
    double D[3] = {g[1] - g[0], g[2] - g[1], g[3] - g[2]};
    double E[3] = {__builtin_fma(C13 * D[0], D[0], eps), __builtin_fma(C13 * D[1], D[1], eps),
                   __builtin_fma(C13 * D[2], D[2], eps)};
#pragma unroll
    for (int t = 0; t < R; ++t) {
        const double mu = cnc * (lr[col(t - 1)] - lr[col(t - 2)]);
        double Gg[4];
        const double CD[3] = {C13 * D[0], C13 * D[1], C13 * D[2]};
        weno_face_bar_g(g, D, CD, E, mu, Gg);
        const double G[5] = {-Gg[0], Gg[0] - Gg[1], (Gg[1] - Gg[2]) + mu, Gg[2] - Gg[3], Gg[3]};
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            const int d = t + q - 4;  // canonical cell of sample q
            if (d >= 0)
                Ac[d] += G[q];
            else
                LG[d + 4] += G[q];
        }
        if (t + 1 < R) {
            g[0] = g[1];
            g[1] = g[2];
            g[2] = g[3];
            g[3] = P[t + 5] - P[t + 4];
            D[0] = D[1];
            D[1] = D[2];
            D[2] = g[3] - g[2];
            E[0] = E[1];
            E[1] = E[2];
            E[2] = __builtin_fma(C13 * D[2], D[2], eps);
        }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) xl[4 * lane + k] = LG[k];
    // the 4 faces beyond each row's last canonical strip (positions R-2+u
    // and R-1+u of that strip, u = 0..3): lane 4 er + u for row er
    if (lane < 4 * R) {
        const int er = lane >> 2, u = lane & 3;
        const double* fe = s_f + (er + FH) * AP + FH;
        const double* le = s_l + (er + LH) * AP + LH;
        // canonical position p of the row's last canonical strip <-> column
        auto ecol = [&](int p) { return NEG ? R - 1 - p : (NS - 1) * R + p; };
        double Pe[5], Ge[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int q = 0; q < 5; ++q) Pe[q] = v * fe[ecol(R + u - 4 + q)];
        const double mu = cnc * (le[ecol(R + u - 1)] - le[ecol(R + u - 2)]);
        weno_face_bar(Pe, eps, mu, Ge);
#pragma unroll
        for (int q = 0; q < 4; ++q) xe[16 * er + 4 * u + q] = q < 4 - u ? Ge[q] : 0.0;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    const int S = NEG ? NS - 1 - s : s;  // canonical strip index
    if (S < NS - 1) {
        const int nb = NEG ? lane - R : lane + R;  // canonical next strip, same row
#pragma unroll
        for (int k = 0; k < 4; ++k) Ac[R - 4 + k] += xl[4 * nb + k];
    } else {
        // face u reaches cell R-4+u+q of this strip for q < 4-u
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            double sum = 0.0;
#pragma unroll
            for (int u = 0; u <= k; ++u) sum += xe[16 * r + 4 * u + (k - u)];
            Ac[R - 4 + k] += sum;
        }
    }
#pragma unroll
    for (int m = 0; m < R; ++m) acc[m] = v * Ac[NEG ? R - 1 - m : m];
}

// Value of plane i at (gx, gy) with the forward ghost rules (domain or the
// three-cell ghost layer of one side; anything else reads as 0).
__device__ __forceinline__ double f_at(const AdjArgs& a, int i, int gx, int gy)
{
    const int64_t plane = (int64_t)a.nx * a.ny;
    const bool inx = (unsigned)gx < (unsigned)a.nx, iny = (unsigned)gy < (unsigned)a.ny;
    if (inx && iny) return a.f[i * plane + (int64_t)gy * a.nx + gx];
    if (inx == iny) return 0.0;
    const bool xg = !inx;
    const int n = xg ? a.nx : a.ny, g = xg ? gx : gy;
    const bool lo = g < 0;
    const int m = lo ? -1 - g : g - n;
    if (m >= HALO) return 0.0;
    const int side = xg ? (lo ? XLO : XHI) : (lo ? YLO : YHI);
    const int bc = a.bc[side];
    if (bc == FIXED_EQ) return a.k.side_eq[side][i];
    int src_i = i, s = wrap_index(g, n);
    if (bc == REFLECT) {
        src_i = xg ? a.k.mirx[i] : a.k.miry[i];
        s = lo ? m : n - 1 - m;
    }
    const int sx = xg ? s : gx, sy = xg ? gy : s;
    return a.f[src_i * plane + (int64_t)sy * a.nx + sx];
}

__device__ __forceinline__ double lam_at(const AdjArgs& a, int i, int gx, int gy)
{
    const int64_t plane = (int64_t)a.nx * a.ny;
    if ((unsigned)gx < (unsigned)a.nx && (unsigned)gy < (unsigned)a.ny)
        return a.lam1[i * plane + (int64_t)gy * a.nx + gx];
    return 0.0;  // only used at positions inside the domain
}

// Contribution of the wall faces of plane j (mirror of plane i across a
// reflecting wall) to plane i at wall-local position p in 0..2. Wall-local
// coordinates run from the wall into the domain; (dx, dy) is that direction,
// (wx, wy) the global cell at p = 0, vn the velocity component of plane j
// along it and cn = dt / spacing.
__device__ __forceinline__ double wall_term(const AdjArgs& a, int j, int wx, int wy, int dx, int dy,
                                            int p, double vn, double cn)
{
    if (vn == 0.0) return 0.0;
    const double eps = a.k.eps;
    // F(q) of plane j at wall-local q = -3..4 (q < 0: ghosts = mirror values)
    double F[8];
#pragma unroll
    for (int q = -3; q <= 4; ++q) F[q + 3] = vn * f_at(a, j, wx + q * dx, wy + q * dy);
    double L[4];  // lambda'_j at q = -1..2 (ghost: zero)
    L[0] = 0.0;
#pragma unroll
    for (int q = 0; q <= 2; ++q) L[q + 1] = lam_at(a, j, wx + q * dx, wy + q * dy);
    double sum = 0.0;
    const int ghost = -1 - p;  // the ghost position that holds cell p
    if (vn > 0.0) {
#pragma unroll
        for (int J = -1; J <= 1; ++J) {
            const double mu = cn * (L[J + 2] - L[J + 1]);
            double G[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
            weno_face_bar(&F[J - 2 + 3], eps, mu, G);  // stencil J-2..J+2
#pragma unroll
            for (int q = 0; q < 5; ++q)
                if (J - 2 + q == ghost) sum += G[q];
        }
    } else {
#pragma unroll
        for (int J = -1; J <= 0; ++J) {
            const double mu = cn * (L[J + 2] - L[J + 1]);
            double P[5];
#pragma unroll
            for (int q = 0; q < 5; ++q) P[q] = F[J + 3 - q + 3];  // stencil J+3..J-1
            double G[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
            weno_face_bar(P, eps, mu, G);
#pragma unroll
            for (int q = 0; q < 5; ++q)
                if (J + 3 - q == ghost) sum += G[q];
        }
    }
    return vn * sum;
}

template <int R, int G, bool BND>
__device__ __forceinline__ void adj_planes(const AdjArgs& a, int grp, int x0, int y0, int lane,
                                           const TileMapG& tf, const TileMapG& tl, double* s_f,
                                           double* s_l, double* s_ax, double* s_xl,
                                           const double (&K0)[R],
                                           const double (&Kx)[R], const double (&Ky)[R],
                                           const double (&KE)[R])
{
    using SF = StageG<R, FH, AP>;
    using SL = StageG<R, LH, AP>;
    const GridBC g = grid_of(a);
    const SideEqConsts se{};
    const int64_t plane = (int64_t)a.nx * a.ny;
    const int gx = x0 + lane;
    const double omct = 1.0 - a.ct, eps = a.k.eps;
    const bool wall_ylo = a.bc[YLO] == REFLECT && y0 < HALO;
    const bool wall_yhi = a.bc[YHI] == REFLECT && y0 + R > a.ny - HALO;
    const bool wall_xlo = a.bc[XLO] == REFLECT && x0 < HALO;
    const bool wall_xhi = a.bc[XHI] == REFLECT && x0 + ATX > a.nx - HALO;
    const int i0 = 1 + grp * (18 / G), iend = i0 + 18 / G;
#pragma unroll 1
    for (int i = i0; i < iend; ++i) {
        double pf[SF::NPRE], pl[SL::NPRE];
        stage_load_g<R, FH, AP, BND, false>(a.f, g, a.k, i, x0, y0, lane, tf, plane, pf);
        stage_load_g<R, LH, AP, BND, true>(a.lam1, g, a.k, i, x0, y0, lane, tl, plane, pl);
        stage_store_g<R, FH, AP, BND, false>(g, a.k, se, i, y0, lane, tf, s_f, pf);
        stage_store_g<R, LH, AP, BND, true>(g, a.k, se, i, y0, lane, tl, s_l, pl);
        __syncthreads();
        const double vx = a.k.vx[i], vy = a.k.vy[i];
        {  // x strips: lane -> (row r = lane % R, strip s = lane / R)
            const int r = lane % R, s = lane / R;
            double acc[R];
            if constexpr (R >= 4) {
                if (vx < 0.0)
                    gather_x_row<R, true>(s_f, s_l, s_xl, s_xl + 256, lane, vx, a.cx, eps, acc);
                else
                    gather_x_row<R, false>(s_f, s_l, s_xl, s_xl + 256, lane, vx, a.cx, eps, acc);
            } else {
                double fw[R + 8], lw[R + 6];
#pragma unroll
                for (int q = 0; q < R + 8; ++q) fw[q] = s_f[(r + FH) * AP + s * R + q];
#pragma unroll
                for (int q = 0; q < R + 6; ++q) lw[q] = s_l[(r + LH) * AP + s * R + q];
                if (vx < 0.0)
                    gather_strip<R, true>(fw, lw, vx, a.cx, eps, acc);
                else
                    gather_strip<R, false>(fw, lw, vx, a.cx, eps, acc);
            }
#pragma unroll
            for (int m = 0; m < R; ++m) s_ax[r * AXP + s * R + m] = acc[m];
        }
        __syncthreads();
        double accy[R];
        if (vy != 0.0) {
            double fw[R + 8], lw[R + 6];
#pragma unroll
            for (int q = 0; q < R + 8; ++q) fw[q] = s_f[q * AP + lane + FH];
#pragma unroll
            for (int q = 0; q < R + 6; ++q) lw[q] = s_l[q * AP + lane + LH];
            if (vy < 0.0)
                gather_strip<R, true>(fw, lw, vy, a.cy, eps, accy);
            else
                gather_strip<R, false>(fw, lw, vy, a.cy, eps, accy);
        } else {
#pragma unroll
            for (int m = 0; m < R; ++m) accy[m] = 0.0;
        }
        double* dst = a.lam0 + i * plane + (int64_t)y0 * a.nx + x0;
        const double hv2 = a.k.hv2[i];
#pragma unroll
        for (int m = 0; m < R; ++m) {
            const int gy = y0 + m;
            const double lc = s_l[(m + LH) * AP + lane + LH];
            double out = __builtin_fma(omct, lc, K0[m]);
            out = __builtin_fma(Kx[m], vx, out);
            out = __builtin_fma(Ky[m], vy, out);
            out = __builtin_fma(KE[m], hv2, out);
            out += s_ax[m * AXP + lane] + accy[m];
            if (BND) {
                // reflecting walls: gather the wall faces of the mirrored plane
                if (wall_ylo && gy < HALO)
                    out += wall_term(a, a.k.miry[i], gx, 0, 0, 1, gy, a.k.vy[a.k.miry[i]], a.cy);
                if (wall_yhi && gy >= a.ny - HALO && gy < a.ny)
                    out += wall_term(a, a.k.miry[i], gx, a.ny - 1, 0, -1, a.ny - 1 - gy,
                                     -a.k.vy[a.k.miry[i]], a.cy);
                if (wall_xlo && gx < HALO)
                    out += wall_term(a, a.k.mirx[i], 0, gy, 1, 0, gx, a.k.vx[a.k.mirx[i]], a.cx);
                if (wall_xhi && gx >= a.nx - HALO && gx < a.nx)
                    out += wall_term(a, a.k.mirx[i], a.nx - 1, gy, -1, 0, a.nx - 1 - gx,
                                     -a.k.vx[a.k.mirx[i]], a.cx);
            }
            if (!BND || (gx < a.nx && gy < a.ny)) dst[(int64_t)m * a.nx + (unsigned)lane] = out;
        }
        __syncthreads();
    }
}

// Per-cell terms of phase 1 for one cell, given its f^n (fv(i)) and
// lambda^{n+1} (lv(i)) values, i = 0..18: the sums over i of lambda'_i times
// the partials of f_i^eq through (rho, j, E), scaled by dt/tau, plus the
// objective's gradient w dx dy (u_y v_iy - u_y^2/2).
struct AdjCell {
    double K0, Kx, Ky, KE, rest;  // rest: the rest particle's adjoint
};

// The cell's terms from its moment sums r = sum f, (jx, jy) = sum f v,
// E = sum f |v|^2 / 2 (Eq. (10)) and lambda'.
template <class LV>
__device__ __forceinline__ AdjCell adj_cell_sums(double r, double jx, double jy, double E, LV&& lv,
                                                 const Consts& k, double ct, double wdxdy)
{
    const double ux = jx / r, uy = jy / r;
    const double u2 = ux * ux + uy * uy;
    const double T = E / r - 0.5 * u2;
    const double iT = 1.0 / T;
    const double t0 = 1.0 - u2 / (2.0 * T);
    const double b = 1.0 - t0;
    const double F1 = weight_c(k, 0, T), F2 = weight_c(k, 1, T), F3 = weight_c(k, 2, T);
    const double F0 = 1.0 - 6.0 * (F1 + F2 + F3);
    const double d1 = dweight_c(k, 0, T), d2 = dweight_c(k, 1, T), d3 = dweight_c(k, 2, T);
    const double d0 = -6.0 * (d1 + d2 + d3);
    // sums over i of lambda'_i times the partials of f_i^eq (Eq. (28)),
    // with P = (1-b)(1+eta) + eta^2/2 + eta^3/6, eta = v.u / T
    double sP = 0.0, sX = 0.0, sY = 0.0, sT = 0.0, l0 = 0.0;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        const double L = lv(i);
        if (i == 0) l0 = L;
        // weight of the speed shell of velocity i and its T derivative
        const double Fs = i == 0 ? F0 : i < 7 ? F1 : i < 13 ? F2 : F3;
        const double dFs = i == 0 ? d0 : i < 7 ? d1 : i < 13 ? d2 : d3;
        const double eta = __builtin_fma(k.vx[i], ux * iT, k.vy[i] * (uy * iT));
        const double P = feq_poly(eta, t0);
        const double Pxi = t0 + eta * (1.0 + 0.5 * eta);        // T dP/dxi
        const double Pb = -(1.0 + eta);                          // dP/db
        const double PTT = -eta * (t0 + eta * (1.0 + 0.5 * eta));  // T dP/dT at fixed xi, b
        const double LF = L * Fs;
        sP = __builtin_fma(LF, P, sP);
        sX = __builtin_fma(LF, __builtin_fma(Pxi, k.vx[i], Pb * ux), sX);
        sY = __builtin_fma(LF, __builtin_fma(Pxi, k.vy[i], Pb * uy), sY);
        sT += L * __builtin_fma(dFs * T, P, Fs * (PTT - Pb * b));
    }
    // f^eq depends on (rho, ux, uy, T): d/drho = F P, d/du = rho F (Pxi v + Pb u)/T,
    // d/dT = rho (F' P + F (PTT - Pb b) / T)
    double rb = sP, uxb = r * iT * sX, uyb = r * iT * sY, Tb = r * iT * sT;
    // T = E/rho - u^2/2, u = j/rho
    const double Eb = Tb / r;
    rb -= Tb * (E / (r * r));
    const double uxb2 = uxb - Tb * ux, uyb2 = uyb - Tb * uy;
    const double jxb = uxb2 / r, jyb = uyb2 / r;
    rb -= (uxb2 * ux + uyb2 * uy) / r;
    AdjCell c;
    c.K0 = __builtin_fma(ct, rb, -0.5 * wdxdy * uy * uy);
    c.Kx = ct * jxb;
    c.Ky = __builtin_fma(ct, jyb, wdxdy * uy);
    c.KE = ct * Eb;
    // rest particle: no convection
    c.rest = __builtin_fma(1.0 - ct, l0, c.K0);
    return c;
}

// The same from f: its sums in the order of k_sums and of the carried-sum
// step kernels (velocity 0 first), so that sums carried from the forward
// step give the same terms bit for bit.
template <class FV, class LV>
__device__ __forceinline__ AdjCell adj_cell(FV&& fv, LV&& lv, const Consts& k, double ct,
                                            double wdxdy)
{
    double r = 0.0, jx = 0.0, jy = 0.0, E = 0.0;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        const double fi = fv(i);
        r += fi;
        jx = __builtin_fma(fi, k.vx[i], jx);
        jy = __builtin_fma(fi, k.vy[i], jy);
        E = __builtin_fma(fi, k.hv2[i], E);
    }
    return adj_cell_sums(r, jx, jy, E, lv, k, ct, wdxdy);
}

// One (tile, group) work item of the reverse step. PS: the K's come from
// a.kst (written with the rest plane by k_adj_state). BAND: the tiles are
// those around a.rect (band_tile), the rest being marched by k_adj_march.
template <int R>
struct TileLds {
    double f[StageG<R, FH, AP>::SLOTS];
    double l[StageG<R, LH, AP>::SLOTS];
    double ax[R * AXP];
    double xl[R >= 4 ? 256 + 16 * R : 1];  // x faces shared along a row
};

template <int R, int G, bool PS, bool BAND>
__device__ __forceinline__ void adjoint_item(const AdjArgs& a, int work, int lane, TileLds<R>& t)
{
    double* const s_f = t.f;
    double* const s_l = t.l;
    double* const s_ax = t.ax;
    double* const s_xl = t.xl;
    const int tile = work / G, grp = work - tile * G;
    const int rm = BAND ? band_tile(tile, a.rect, a.tiles_x, a.tiles_y)
                        : strip_walk(tile, a.tiles_x, a.tiles_y);
    const int ty = rm / a.tiles_x, tx = rm - ty * a.tiles_x;
    const int x0 = tx * ATX, y0 = ty * R;
    const int64_t plane = (int64_t)a.nx * a.ny;
    const int gx = x0 + lane;
    const bool interior = fast_tile(grid_of(a), x0, y0, ATX, R, FH);

    // ---- phase 1: per-cell adjoint of the equilibrium and the objective ----
    double K0[R], Kx[R], Ky[R], KE[R];
#pragma unroll
    for (int m = 0; m < R; ++m) {
        const int gy = y0 + m;
        const bool act = gx < a.nx && gy < a.ny;
        K0[m] = Kx[m] = Ky[m] = KE[m] = 0.0;
        if (!act) continue;
        const int64_t c = (int64_t)gy * a.nx + gx;
        if (PS) {
            K0[m] = a.kst[4 * c];
            Kx[m] = a.kst[4 * c + 1];
            Ky[m] = a.kst[4 * c + 2];
            KE[m] = a.kst[4 * c + 3];
        } else {
            // loads at their point of use: these variants have no registers
            // to spare for 38 values in flight
            const double* pf = a.f + c;
            const double* pl = a.lam1 + c;
            const AdjCell q = adj_cell([&](int i) { return pf[i * plane]; },
                                       [&](int i) { return pl[i * plane]; }, a.k, a.ct, a.wdxdy);
            K0[m] = q.K0;
            Kx[m] = q.Kx;
            Ky[m] = q.Ky;
            KE[m] = q.KE;
            if (grp == 0) a.lam0[c] = q.rest;
        }
    }

    // ---- phase 2: the group's moving velocities ----
    const GridBC g = grid_of(a);
    const TileMapG tf = tile_map_g<R, FH, false>(g, x0, y0, lane, !interior);
    const TileMapG tl = tile_map_g<R, LH, true>(g, x0, y0, lane, !interior);
    if (interior)
        adj_planes<R, G, false>(a, grp, x0, y0, lane, tf, tl, s_f, s_l, s_ax, s_xl, K0, Kx, Ky,
                                KE);
    else
        adj_planes<R, G, true>(a, grp, x0, y0, lane, tf, tl, s_f, s_l, s_ax, s_xl, K0, Kx, Ky,
                               KE);
}

template <int R, int G, int W, bool PS, bool BAND = false>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(W))) void k_adjoint(AdjArgs a)
{
    __shared__ TileLds<R> t;
    const int b = blockIdx.x;
    const int work = (b & 7) * a.per_xcd + (b >> 3);
    if (work >= a.nwork) return;
    adjoint_item<R, G, PS, BAND>(a, work, threadIdx.x, t);
}

// State pass of the reverse step, one thread per cell: the K's of phase 1
// (to kst) and the rest particle's adjoint (to plane 0 of lam0). SUMS: the
// cell's moment sums come from `sums` ([4][n], as k_sums writes them)
// instead of from f, which is then not read.
template <bool SUMS>
__global__ __launch_bounds__(256) void k_adj_state(const double* __restrict__ f,
                                                   const double* __restrict__ sums,
                                                   const double* __restrict__ lam1,
                                                   double* __restrict__ lam0,
                                                   double* __restrict__ kst, int64_t n, double ct,
                                                   double wdxdy, Consts k)
{
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= n) return;
    // all values are loaded before any is used, so that their latencies
    // overlap (left to itself the scheduler issues each load just before its
    // first use and waits for it: one round trip per value in sequence)
    constexpr int NF = SUMS ? 4 : NV;
    double fv[NF], lv[NV];
#pragma unroll
    for (int i = 0; i < NF; ++i) fv[i] = (SUMS ? sums : f)[i * n + c];
#pragma unroll
    for (int i = 0; i < NV; ++i) lv[i] = lam1[i * n + c];
    __builtin_amdgcn_sched_barrier(0);
    AdjCell q;
    if constexpr (SUMS)
        q = adj_cell_sums(fv[0], fv[1], fv[2], fv[3], [&](int i) { return lv[i]; }, k, ct, wdxdy);
    else
        q = adj_cell([&](int i) { return fv[i]; }, [&](int i) { return lv[i]; }, k, ct, wdxdy);
    // the four K's of a cell side by side (32 bytes): the marching kernel
    // takes them with two 16-byte loads
    kst[4 * c] = q.K0;
    kst[4 * c + 1] = q.Kx;
    kst[4 * c + 2] = q.Ky;
    kst[4 * c + 3] = q.KE;
    lam0[c] = q.rest;
}

// ---------------------------------------------------------------------------
// Marching reverse step (after the state pass). One wavefront takes one
// moving velocity i over a strip of 64 columns and a chunk of rows of the
// region whose stencils need no ghost cell (adj_rect); the tiles around it go
// to k_adjoint in band mode. Along x the lanes are canonical, i.e. seen from
// the upwind side: lane l holds canonical column l (natural column X0 + l,
// or X0 + 63 - l for v_x < 0), so that the face between canonical columns c
// and c+1 has the samples c-2..c+2 and feeds the cells c-2..c+2. Along y
// every wave walks the natural rows upwards, whatever the sign of v_y: step
// t completes row Y0 - 4 + t, for all velocities alike, so that the waves
// of a region read the same rows of the K planes and of the neighbouring
// strips at about the same time.
//  - y faces: each lane carries the sliding differences of the forward WENO
//    of the five rows Y0-4+t .. Y0+t of its column in upwind order; step t
//    evaluates the face between rows Y0-2+t and Y0-1+t (v_y > 0, samples
//    upwards from row Y0-4+t) or between rows Y0-3+t and Y0-2+t (v_y < 0,
//    samples downwards from row Y0+t), the last face that reaches row
//    Y0-4+t. Every y face is evaluated once, four of them ahead of the chunk.
//  - x faces: the completed row is exchanged through LDS; lane l evaluates
//    the face between canonical columns l and l+1 and the five
//    contributions of each face are gathered back through LDS. The four
//    faces beyond the strip's edges (canonical faces -2, -1, 64, 65), which
//    reach the cells 0, 1, 62 and 63, are saved per row and evaluated for a
//    batch of MB rows at once, one lane per face and row.
// The output rows wait in LDS until their batch's edge faces are done and
// are then written whole (full 128-byte lines). Loads run two steps ahead,
// each into the register it frees; f is loaded once per row, for the y
// window, and kept in registers until its row's x pass.
constexpr int MB = 16;

struct MarchLds {
    double P[72];           // v_x f of the row, canonical columns -4..67
    double L[72];           // lambda' of the row, canonical columns -4..67 (-2..66 used)
    double G[4][68];        // G_0, G_1, G_3, G_4 of canonical faces -2..65 (-2, -1, 64, 65: 0)
    double ring[MB][18];    // per row: P(-4..1), P(62..67), L(-2..0), L(64..66)
    double part[MB][4][2];  // cells 0, 1, 62, 63: output without the x term, partial x sum
    double eg[64][2];       // contributions of the edge faces
    double orow[MB][64];    // the output rows of the batch, canonical columns
    double dump[4][64];     // where the lanes without a value to save write theirs (one row
                            // per store, 8-byte lane stride: no bank conflicts)
};

// mu dh/dP_q (q = 0..4) of one face from its five upwind-ordered samples; the
// centre sample's own term mu is included.
__device__ __forceinline__ void face_g5(double P0, double P1, double P2, double P3, double P4,
                                        double eps, double mu, double (&G)[5])
{
    constexpr double C13 = 13.0 / 12.0;
    const double g[4] = {P1 - P0, P2 - P1, P3 - P2, P4 - P3};
    const double D[3] = {g[1] - g[0], g[2] - g[1], g[3] - g[2]};
    const double CD[3] = {C13 * D[0], C13 * D[1], C13 * D[2]};
    const double E[3] = {__builtin_fma(CD[0], D[0], eps), __builtin_fma(CD[1], D[1], eps),
                         __builtin_fma(CD[2], D[2], eps)};
    double Gg[4];
    weno_face_bar_g(g, D, CD, E, mu, Gg);
    G[0] = -Gg[0];
    G[1] = Gg[0] - Gg[1];
    G[2] = (Gg[1] - Gg[2]) + mu;
    G[3] = Gg[2] - Gg[3];
    G[4] = Gg[3];
}

// The marching workgroup is one wavefront, and the LDS carries out one
// wavefront's accesses in the order they are issued: a read issued after a
// write of another lane sees it. Only the compiler has to keep the accesses
// in program order across these points.
__device__ __forceinline__ void wave_lds_order() { asm volatile("" ::: "memory"); }

// Raw buffer access to planes below 2 GiB in all: the row (and plane)
// offset goes in the scalar offset, the lane's column in the vector offset.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const double* p, int64_t cells)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(p), 0, (int)(cells * 8),
                                             0x00020000);
}
__device__ __forceinline__ double bload(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
__device__ __forceinline__ void bstore(double v, __amdgpu_buffer_rsrc_t r, unsigned voff,
                                       unsigned soff)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, v), r, voff, soff, 0);
}

template <bool HASY, bool NEGY>
__device__ __forceinline__ void march_velocity(const AdjArgs& a, MarchLds& s, int i, int X0, int Y0,
                                               int H, int lane)
{
    constexpr double C13 = 13.0 / 12.0;
    const int nx = a.nx;
    const int64_t plane = (int64_t)nx * a.ny;
    const double vx = a.k.vx[i], vy = a.k.vy[i], hv2 = a.k.hv2[i];
    const bool negx = vx < 0.0;
    const double cnx = negx ? -a.cx : a.cx, cy = a.cy;
    const double eps = a.k.eps, omct = 1.0 - a.ct;
    // natural column of canonical column c (c in -4..67: one period at most
    // away, which happens on a periodic x axis only)
    auto colc = [&](int c) {
        int x = negx ? X0 + 63 - c : X0 + c;
        x = x < 0 ? x + nx : x;
        return x >= nx ? x - nx : x;
    };
    // byte offset of row Y0 - 4 + t (t in 0..H+7: the marched rows are at
    // least four rows from either end)
    const int rowbytes = nx * 8, base = (Y0 - 4) * rowbytes;
    auto rowt = [&](int t) { return (unsigned)(base + t * rowbytes); };
    const unsigned co = 8u * (unsigned)colc(lane);
    // extra samples of the edge faces: f at canonical -4..-1 and 64..67
    // (lanes 0..7), lambda' at -2, -1, 64, 65, 66 (lanes 0..4); the other
    // lanes repeat the addresses of the first ones, so that each of these
    // loads touches two cache lines
    const int l8 = lane & 7, l4 = lane & 3;
    const unsigned cxf = 8u * (unsigned)colc(l8 < 4 ? l8 - 4 : 60 + l8);
    const unsigned cxl = 8u * (unsigned)colc(lane < 5 ? (lane < 2 ? lane - 2 : 62 + lane)
                                                      : (l4 < 2 ? l4 - 2 : 62 + l4));
    const __amdgpu_buffer_rsrc_t rf = plane_rsrc(a.f + i * plane, plane);
    const __amdgpu_buffer_rsrc_t rl = plane_rsrc(a.lam1 + i * plane, plane);
    const __amdgpu_buffer_rsrc_t ro = plane_rsrc(a.lam0 + i * plane, plane);
    // the K's of the output, 32 bytes per cell: two 16-byte loads per lane
    const __amdgpu_buffer_rsrc_t rk = plane_rsrc(a.kst, 4 * plane);
    auto kload = [&](double (&K)[4], unsigned row) {
        typedef unsigned u4 __attribute__((ext_vector_type(4)));
        typedef unsigned u2 __attribute__((ext_vector_type(2)));
        const u4 v0 = __builtin_amdgcn_raw_buffer_load_b128(rk, 4u * co, 4u * row, 0);
        const u4 v1 = __builtin_amdgcn_raw_buffer_load_b128(rk, 4u * co + 16u, 4u * row, 0);
        K[0] = __builtin_bit_cast(double, (u2){v0[0], v0[1]});
        K[1] = __builtin_bit_cast(double, (u2){v0[2], v0[3]});
        K[2] = __builtin_bit_cast(double, (u2){v1[0], v1[1]});
        K[3] = __builtin_bit_cast(double, (u2){v1[2], v1[3]});
    };
    // per-lane LDS slots (lanes with nothing to save write to s.dump): the
    // edge samples' destinations, the ring's sources and destinations, the
    // saved outputs of cells 0, 1, 62 and 63
    double* const dxf = lane < 8 ? s.P + (lane < 4 ? lane : 64 + lane) : &s.dump[0][lane];
    double* const dxl = lane < 5 ? s.L + (lane < 2 ? lane + 2 : 66 + lane) : &s.dump[1][lane];
    const double* const rsrc = lane < 6    ? s.P + lane
                               : lane < 12 ? s.P + 60 + lane
                               : lane < 15 ? s.L + lane - 10
                               : lane < 18 ? s.L + 53 + lane
                                           : s.P;
    double* const rdst = lane < 18 ? &s.ring[0][lane] : &s.dump[2][lane];
    const int rstride = lane < 18 ? 18 : 0;
    const bool edge = lane < 2 || lane >= 62;
    double* const pdst0 = edge ? &s.part[0][lane < 2 ? lane : lane - 60][0] : &s.dump[3][lane];
    double* const pdst1 = edge ? pdst0 + 1 : &s.dump[0][lane];
    const int pstride = edge ? 8 : 0;

    if (lane < 4) {
        s.G[lane][0] = s.G[lane][1] = 0.0;
        s.G[lane][66] = s.G[lane][67] = 0.0;
    }
    // state at step t: L = lambda' of rows Y0-4+t .. Y0-1+t, Acc[j] = the y
    // sum of row Y0-4+t+j so far (j < 4); g: the first differences of the
    // face's samples v_y f (rows Y0-4+t .. Y0+t) in upwind order, slid from
    // step to step with the second differences D, 13/12 D and the smoothness
    // terms E; Pl: v_y f of row Y0+t; F = f of rows Y0-4+t .. Y0+t
    double L[4], Acc[4] = {0.0, 0.0, 0.0, 0.0};
    double Pl = 0.0, g[4] = {0.0, 0.0, 0.0, 0.0}, F[5];
    double yD[3] = {0.0, 0.0, 0.0}, yC[3] = {0.0, 0.0, 0.0}, yE[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < 4; ++q) L[q] = bload(rl, co, rowt(q));
#pragma unroll
    for (int q = 0; q < 5; ++q) F[q] = bload(rf, co, rowt(q));
    if constexpr (HASY) {
        double P[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) P[q] = vy * F[NEGY ? 4 - q : q];
#pragma unroll
        for (int q = 0; q < 4; ++q) g[q] = P[q + 1] - P[q];
        Pl = P[NEGY ? 0 : 4];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            yD[q] = g[q + 1] - g[q];
            yC[q] = C13 * yD[q];
            yE[q] = __builtin_fma(yC[q], yD[q], eps);
        }
    }
    // slot k = t mod 2 holds what step t consumes: f of row Y0+1+t,
    // lambda' of row Y0+t and, for the x pass of row Y0-4+t, the edge
    // samples and the K's; the loads run two steps ahead
    double fb[2], lb[2], xfb[2], xlb[2], kb[2][4];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        fb[k] = bload(rf, co, rowt(5 + k));
        lb[k] = bload(rl, co, rowt(4 + k));
        xfb[k] = xlb[k] = 0.0;
        kb[k][0] = kb[k][1] = kb[k][2] = kb[k][3] = 0.0;
    }

    auto face = [&](auto kc, auto outc, int t) {
        constexpr int k = decltype(kc)::value;
        constexpr bool OUT = decltype(outc)::value;
        const unsigned r = (unsigned)(t - 4), rr = r % MB;  // output row Y0 + r
        if constexpr (OUT) {
            // the completed row into LDS for its x faces
            s.P[lane + 4] = vx * F[0];
            s.L[lane + 4] = L[0];
            *dxf = vx * xfb[k];
            *dxl = xlb[k];
        }
        double Gl = 0.0;  // the contribution to the row entering the window
        if constexpr (HASY) {
            // v_y > 0: the face between rows Y0-2+t and Y0-1+t, samples rows
            // Y0-4+t.. upwards; v_y < 0: between rows Y0-3+t and Y0-2+t,
            // samples rows Y0+t.. downwards
            const double mu = NEGY ? cy * (L[2] - L[1]) : cy * (L[3] - L[2]);
            double Gg[4];
            weno_face_bar_g(g, yD, yC, yE, mu, Gg);
            const double G0 = -Gg[0], G1 = Gg[0] - Gg[1], G2 = (Gg[1] - Gg[2]) + mu,
                         G3 = Gg[2] - Gg[3], G4 = Gg[3];
            if constexpr (NEGY) {  // sample q is row Y0+t-q
                Acc[0] += G4;
                Acc[1] += G3;
                Acc[2] += G2;
                Acc[3] += G1;
                Gl = G0;
            } else {  // sample q is row Y0-4+t+q
                Acc[0] += G0;
                Acc[1] += G1;
                Acc[2] += G2;
                Acc[3] += G3;
                Gl = G4;
            }
        }
        double out = 0.0, Gx2 = 0.0;
        if constexpr (OUT) {
            wave_lds_order();
            const double* Pp = s.P + lane + 2;
            const double mux = cnx * (s.L[lane + 5] - L[0]);
            double Gx[5];
            face_g5(Pp[0], Pp[1], Pp[2], Pp[3], Pp[4], eps, mux, Gx);
            rdst[rr * rstride] = *rsrc;
            s.G[0][lane + 2] = Gx[0];
            s.G[1][lane + 2] = Gx[1];
            s.G[2][lane + 2] = Gx[3];
            s.G[3][lane + 2] = Gx[4];
            Gx2 = Gx[2];
            out = __builtin_fma(omct, L[0], kb[k][0]);
            out = __builtin_fma(kb[k][1], vx, out);
            out = __builtin_fma(kb[k][2], vy, out);
            out = __builtin_fma(kb[k][3], hv2, out);
            if constexpr (HASY) out = __builtin_fma(vy, Acc[0], out);
        }
        // slide to step t+1, consuming slot k
#pragma unroll
        for (int q = 0; q < 3; ++q) L[q] = L[q + 1];
        L[3] = lb[k];
#pragma unroll
        for (int q = 0; q < 4; ++q) F[q] = F[q + 1];
        F[4] = fb[k];
        if constexpr (HASY) {
#pragma unroll
            for (int q = 0; q < 3; ++q) Acc[q] = Acc[q + 1];
            Acc[3] = Gl;
            const double Pn = vy * fb[k];
            if constexpr (NEGY) {  // the new row is the first sample
                g[3] = g[2];
                g[2] = g[1];
                g[1] = g[0];
                g[0] = Pl - Pn;
#pragma unroll
                for (int q = 2; q > 0; --q) {
                    yD[q] = yD[q - 1];
                    yC[q] = yC[q - 1];
                    yE[q] = yE[q - 1];
                }
                yD[0] = g[1] - g[0];
                yC[0] = C13 * yD[0];
                yE[0] = __builtin_fma(yC[0], yD[0], eps);
            } else {  // the new row is the last sample
#pragma unroll
                for (int q = 0; q < 3; ++q) g[q] = g[q + 1];
                g[3] = Pn - Pl;
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    yD[q] = yD[q + 1];
                    yC[q] = yC[q + 1];
                    yE[q] = yE[q + 1];
                }
                yD[2] = g[3] - g[2];
                yC[2] = C13 * yD[2];
                yE[2] = __builtin_fma(yC[2], yD[2], eps);
            }
            Pl = Pn;
        }
        // refill slot k for step t+2
        fb[k] = bload(rf, co, rowt(min(t + 7, H + 7)));
        lb[k] = bload(rl, co, rowt(min(t + 6, H + 6)));
        {
            const unsigned rx = rowt(min(t + 2, H + 3));
            xfb[k] = bload(rf, cxf, rx);
            xlb[k] = bload(rl, cxl, rx);
            kload(kb[k], rx);
        }
        if constexpr (OUT) {
            wave_lds_order();
            const double xs = ((s.G[0][lane + 4] + s.G[1][lane + 3]) + Gx2) +
                              (s.G[2][lane + 1] + s.G[3][lane]);
            pdst0[rr * pstride] = out;
            pdst1[rr * pstride] = xs;
            s.orow[rr][lane] = __builtin_fma(vx, xs, out);  // (edge cells: completed later)
            wave_lds_order();
        }
    };

    // the four steps ahead of the chunk's first row
    face(std::integral_constant<int, 0>{}, std::false_type{}, 0);
    face(std::integral_constant<int, 1>{}, std::false_type{}, 1);
    face(std::integral_constant<int, 0>{}, std::false_type{}, 2);
    face(std::integral_constant<int, 1>{}, std::false_type{}, 3);
    // the strip-edge faces of the rows since the last batch, done = output
    // rows so far
    auto flush = [&](int done) {
        const int nrows = done - (done - 1) / MB * MB, r0 = done - nrows;
        const int rr = lane >> 2, e = lane & 3;
        double c0 = 0.0, c1 = 0.0;
        if (rr < nrows) {
            const double* Rw = s.ring[rr];
            const int b0 = e < 2 ? e : 4 + e;
            const int lo = e < 2 ? 12 + e : 13 + e;
            const double mu = cnx * (Rw[lo + 1] - Rw[lo]);
            double Ge[5];
            face_g5(Rw[b0], Rw[b0 + 1], Rw[b0 + 2], Rw[b0 + 3], Rw[b0 + 4], eps, mu, Ge);
            // face -2 -> cell 0: G_4; face -1 -> cells 0, 1: G_3, G_4;
            // face 64 -> cells 62, 63: G_0, G_1; face 65 -> cell 63: G_0
            c0 = e == 0 ? Ge[4] : e == 1 ? Ge[3] : Ge[0];
            c1 = e == 1 ? Ge[4] : e == 2 ? Ge[1] : 0.0;
        }
        s.eg[lane][0] = c0;
        s.eg[lane][1] = c1;
        wave_lds_order();
        if (rr < nrows) {
            const int b = 4 * rr;
            const double add = e == 0   ? s.eg[b][0] + s.eg[b + 1][0]
                               : e == 1 ? s.eg[b + 1][1]
                               : e == 2 ? s.eg[b + 2][0]
                                        : s.eg[b + 2][1] + s.eg[b + 3][0];
            const int cell = e < 2 ? e : 60 + e;
            // (the row differs between lanes: it goes in the vector offset)
            s.orow[rr][cell] = __builtin_fma(vx, s.part[rr][e][1] + add, s.part[rr][e][0]);
        }
        wave_lds_order();
        for (int q = 0; q < nrows; ++q) bstore(s.orow[q][lane], ro, co, rowt(r0 + q + 4));
        wave_lds_order();
    };

    // Eight steps per trip: a loaded value lives at most six steps (two in
    // its slot, four in the window), so every load of the body keeps one
    // register from trip to trip and none is copied at the loop head.
    const int nblk = H / 4;
    int bk = 0;
#pragma unroll 1
    for (; bk + 2 <= nblk; bk += 2) {
        const int p0 = __builtin_amdgcn_readfirstlane(4 + 4 * bk);
        face(std::integral_constant<int, 0>{}, std::true_type{}, p0);
        face(std::integral_constant<int, 1>{}, std::true_type{}, p0 + 1);
        face(std::integral_constant<int, 0>{}, std::true_type{}, p0 + 2);
        face(std::integral_constant<int, 1>{}, std::true_type{}, p0 + 3);
        face(std::integral_constant<int, 0>{}, std::true_type{}, p0 + 4);
        face(std::integral_constant<int, 1>{}, std::true_type{}, p0 + 5);
        face(std::integral_constant<int, 0>{}, std::true_type{}, p0 + 6);
        face(std::integral_constant<int, 1>{}, std::true_type{}, p0 + 7);
        const int done = 4 * bk + 8;  // a multiple of 8: the ring holds MB = 16 rows
        if (done % MB == 0 || bk + 2 == nblk) flush(done);
    }
    if (bk < nblk) {
        const int p0 = 4 + 4 * bk;
        face(std::integral_constant<int, 0>{}, std::true_type{}, p0);
        face(std::integral_constant<int, 1>{}, std::true_type{}, p0 + 1);
        face(std::integral_constant<int, 0>{}, std::true_type{}, p0 + 2);
        face(std::integral_constant<int, 1>{}, std::true_type{}, p0 + 3);
        flush(4 * bk + 4);
    }
}

// One launch for the marched region and the band tiles around it: each XCD
// takes a.per_xcd march items and then a.band_xcd band items (one velocity
// of a 64 x 4 tile each, k_adjoint's band mode), which fill the tail that
// the marching waves leave.
template <int W>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(W))) void k_adj_march(AdjArgs a)
{
    __shared__ union {
        MarchLds m;
        TileLds<4> t;
    } u;
    MarchLds& s = u.m;
    const int b = blockIdx.x, j = b >> 3;
    if (j >= a.per_xcd) {
        const int w = (b & 7) * a.band_xcd + (j - a.per_xcd);
        if (w < a.nband) adjoint_item<4, 18, true, true>(a, w, threadIdx.x, u.t);
        return;
    }
    const int work = (b & 7) * a.per_xcd + j;
    if (work >= a.nwork) return;
    const int reg = work / 18;
    const int i = 1 + (work - reg * 18);
    const int chunk = reg / a.nstrip, strip = reg - chunk * a.nstrip;
    const int X0 = (a.rect.c0 + strip) * ATX;
    const int Y0 = a.rect.r0 * 4 + chunk * a.mh;
    const int H = min(a.mh, a.rect.r1 * 4 - Y0);
    const double vy = a.k.vy[i];
    if (vy > 0.0)
        march_velocity<true, false>(a, s, i, X0, Y0, H, threadIdx.x);
    else if (vy < 0.0)
        march_velocity<true, true>(a, s, i, X0, Y0, H, threadIdx.x);
    else
        march_velocity<false, false>(a, s, i, X0, Y0, H, threadIdx.x);
}

// The region the marching kernel takes, in tiles of 64 x 4 cells: along x
// the whole tiles of a periodic axis (the stencils wrap), else the tiles whose
// cells are at least four cells (the reach of a face's stencil plus one)
// from either end, so that no stencil reaches a ghost cell and no wall term
// applies; along y always the latter, so that no row index wraps.
FastRect adj_rect(int nx, int ny, const int bc[4])
{
    FastRect r;
    const int ty = (ny + 3) / 4;
    if (bc[XLO] == PERIODIC) {
        r.c0 = 0;
        r.c1 = nx / ATX;
    } else {
        r.c0 = 1;
        r.c1 = nx >= 4 ? (nx - 4) / ATX : 0;
    }
    // (on a periodic y axis too, so that the marched rows never wrap)
    r.r0 = 1;
    r.r1 = bc[YLO] == PERIODIC ? ny / 4 - 1 : ny >= 4 ? (ny - 4) / 4 : 0;
    if (r.c1 <= r.c0 || r.r1 <= r.r0) {
        r.c0 = r.c1 = 0;
        r.r0 = r.r1 = ty;
    }
    return r;
}

// ---------------------------------------------------------------------------
// VJP of the equilibrium initialisation: g_q = sum_i lam_i d f_i^eq / d q for
// q in (rho, ux, uy, T), one thread per cell.
__global__ void k_init_vjp(const double* __restrict__ rho, const double* __restrict__ ux,
                           const double* __restrict__ uy, const double* __restrict__ T,
                           const double* __restrict__ lam, double* __restrict__ grho,
                           double* __restrict__ gux, double* __restrict__ guy,
                           double* __restrict__ gT, int64_t n, Consts k)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const double r = rho[c], u = ux[c], v = uy[c], t = T[c];
    const double iT = 1.0 / t;
    const double t0 = 1.0 - (u * u + v * v) / (2.0 * t);
    const double b = 1.0 - t0;
    double Fk[4], dF[4];
    Fk[1] = weight_c(k, 0, t);
    Fk[2] = weight_c(k, 1, t);
    Fk[3] = weight_c(k, 2, t);
    Fk[0] = 1.0 - 6.0 * (Fk[1] + Fk[2] + Fk[3]);
    dF[1] = dweight_c(k, 0, t);
    dF[2] = dweight_c(k, 1, t);
    dF[3] = dweight_c(k, 2, t);
    dF[0] = -6.0 * (dF[1] + dF[2] + dF[3]);
    double sP = 0.0, sX = 0.0, sY = 0.0, sT = 0.0;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        const double L = lam[i * n + c];
        const int s = i == 0 ? 0 : 1 + (i - 1) / 6;
        const double eta = __builtin_fma(k.vx[i], u * iT, k.vy[i] * (v * iT));
        const double P = feq_poly(eta, t0);
        const double Pxi = t0 + eta * (1.0 + 0.5 * eta);
        const double Pb = -(1.0 + eta);
        const double PTT = -eta * (t0 + eta * (1.0 + 0.5 * eta));
        const double LF = L * Fk[s];
        sP = __builtin_fma(LF, P, sP);
        sX = __builtin_fma(LF, __builtin_fma(Pxi, k.vx[i], Pb * u), sX);
        sY = __builtin_fma(LF, __builtin_fma(Pxi, k.vy[i], Pb * v), sY);
        sT += L * __builtin_fma(dF[s] * t, P, Fk[s] * (PTT - Pb * b));
    }
    grho[c] = sP;
    gux[c] = r * iT * sX;
    guy[c] = r * iT * sY;
    gT[c] = r * iT * sT;
}

// out[m] = sum_{y,x} A[m, x] B[y] g[y, x] in two deterministic passes: column
// sums weighted by B, then the row products with A.
__global__ __launch_bounds__(256) void k_colsum(const double* __restrict__ g,
                                                const double* __restrict__ B, int nx, int ny,
                                                double* __restrict__ col)
{
    const int x = blockIdx.x * 256 + threadIdx.x;
    if (x >= nx) return;
    double s = 0.0;
    for (int y = 0; y < ny; ++y) s = __builtin_fma(B[y], g[(int64_t)y * nx + x], s);
    col[x] = s;
}

__global__ __launch_bounds__(256) void k_rowdot(const double* __restrict__ A,
                                                const double* __restrict__ col, int nx, int M,
                                                double* __restrict__ out)
{
    __shared__ double sr[4];
    const int m = blockIdx.x;
    if (m >= M) return;
    double s = 0.0;
    for (int x = threadIdx.x; x < nx; x += 256) s = __builtin_fma(A[(int64_t)m * nx + x], col[x], s);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) sr[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[m] = sr[0] + sr[1] + sr[2] + sr[3];
}

// ---------------------------------------------------------------------------
// Reverse-step variants: rows per lane R, velocity groups G, waves-per-SIMD
// target W and whether a state pass forms the K's first (PS).
// PS = 2: the state pass, then k_adj_march over adj_rect in chunks of R
// rows and k_adjoint<4, 18, 2, true> in band mode around it.
struct AdjVariant {
    int R, G, W, PS;
    void (*kernel)(AdjArgs);
};

#define LBM_ADJ_VARIANT(R, G, W, PS) {R, G, W, PS, k_adjoint<R, G, W, PS>},
#define LBM_ADJ_MARCH(R, W) {R, 18, W, 2, k_adj_march<W>},
// (no variant may spill registers: multi-plane groups under the two-wave
// budget, and one velocity group per tile, are left out for that)
static const AdjVariant kAdjVariants[] = {
    LBM_ADJ_VARIANT(4, 3, 1, 0) LBM_ADJ_VARIANT(4, 6, 1, 0)
    LBM_ADJ_VARIANT(4, 18, 1, 1) LBM_ADJ_VARIANT(4, 18, 2, 1) LBM_ADJ_VARIANT(2, 18, 2, 1)
    LBM_ADJ_VARIANT(4, 6, 1, 1) LBM_ADJ_VARIANT(4, 3, 1, 1)
    LBM_ADJ_MARCH(64, 2) LBM_ADJ_MARCH(128, 2) LBM_ADJ_MARCH(256, 2) LBM_ADJ_MARCH(32, 2)
    LBM_ADJ_MARCH(16, 2)
};
#undef LBM_ADJ_VARIANT
#undef LBM_ADJ_MARCH
constexpr int kNumAdjVariants = sizeof(kAdjVariants) / sizeof(kAdjVariants[0]);

int adj_variant_count() { return kNumAdjVariants; }
int adj_variant_desc(int v, int info[4])
{
    if (v < 0 || v >= kNumAdjVariants) return -1;
    info[0] = kAdjVariants[v].R;
    info[1] = kAdjVariants[v].G;
    info[2] = kAdjVariants[v].W;
    info[3] = kAdjVariants[v].PS;
    return 0;
}

hipError_t launch_adjoint(int variant, const double* f, const double* sums, const double* lam1,
                          double* lam0, double* kst, const Consts& k, int nx, int ny,
                          const int bc[4], double cx, double cy, double ct, double wdxdy,
                          hipStream_t st)
{
    const AdjVariant& V = kAdjVariants[variant];
    AdjArgs a;
    a.f = f;
    a.lam1 = lam1;
    a.lam0 = lam0;
    a.kst = kst;
    a.nx = nx;
    a.ny = ny;
    for (int s = 0; s < 4; ++s) a.bc[s] = bc[s];
    a.tiles_x = (nx + ATX - 1) / ATX;
    a.tiles_y = (ny + V.R - 1) / V.R;
    a.nwork = a.tiles_x * a.tiles_y * V.G;
    a.per_xcd = (a.nwork + 7) / 8;
    a.cx = cx;
    a.cy = cy;
    a.ct = ct;
    a.wdxdy = wdxdy;
    a.k = k;
    if (V.PS) {
        const int64_t n = (int64_t)nx * ny;
        if (sums)
            hipLaunchKernelGGL(k_adj_state<true>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                               st, f, sums, lam1, lam0, kst, n, ct, wdxdy, k);
        else
            hipLaunchKernelGGL(k_adj_state<false>, dim3((unsigned)((n + 255) / 256)), dim3(256),
                               0, st, f, sums, lam1, lam0, kst, n, ct, wdxdy, k);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (V.PS == 2) {
        // band tiles (64 x 4, one velocity each), then the marched region;
        // grids whose 4 K planes reach 2 GiB (32-bit buffer offsets) are all
        // band
        a.tiles_y = (ny + 3) / 4;
        a.rect = adj_rect(nx, ny, bc);
        if ((int64_t)nx * ny * 32 > INT32_MAX) {
            a.rect.c0 = a.rect.c1 = 0;
            a.rect.r0 = a.rect.r1 = a.tiles_y;
        }
        const int nband = band_count(a.rect, a.tiles_x, a.tiles_y);
        if (a.rect.c1 <= a.rect.c0) {
            // nothing to march: the band tiles are the whole grid
            a.nwork = nband * 18;
            a.per_xcd = (a.nwork + 7) / 8;
            hipLaunchKernelGGL((k_adjoint<4, 18, 2, true, true>), dim3(8 * a.per_xcd), dim3(64), 0,
                               st, a);
            return hipGetLastError();
        }
        a.mh = V.R;
        a.nstrip = a.rect.c1 - a.rect.c0;
        a.nchunk = ((a.rect.r1 - a.rect.r0) * 4 + V.R - 1) / V.R;
        a.nwork = a.nstrip * a.nchunk * 18;
        a.per_xcd = (a.nwork + 7) / 8;
        a.nband = nband * 18;
        a.band_xcd = (a.nband + 7) / 8;
        hipLaunchKernelGGL(V.kernel, dim3(8 * (a.per_xcd + a.band_xcd)), dim3(64), 0, st, a);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(V.kernel, dim3(8 * a.per_xcd), dim3(64), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_init_vjp(const double* rho, const double* ux, const double* uy, const double* T,
                           const double* lam, double* grho, double* gux, double* guy, double* gT,
                           const Consts& k, int64_t n, hipStream_t st)
{
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_init_vjp, dim3((unsigned)blocks), dim3(256), 0, st, rho, ux, uy, T, lam,
                       grho, gux, guy, gT, n, k);
    return hipGetLastError();
}

hipError_t launch_sep_project(const double* g, const double* A, const double* B, int nx, int ny,
                              int M, double* col, double* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_colsum, dim3((nx + 255) / 256), dim3(256), 0, st, g, B, nx, ny, col);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rowdot, dim3(M), dim3(256), 0, st, A, col, nx, M, out);
    return hipGetLastError();
}

}  // namespace lbmd
