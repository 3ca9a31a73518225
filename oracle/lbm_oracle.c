/*
 * lbm_oracle.c -- plain FP64 CPU oracle for the D2V19 finite-difference
 * lattice-Boltzmann (FDLB) model of Gan, Xu, Zhang and Li, "Lattice Boltzmann
 * study on Kelvin-Helmholtz instability: the roles of velocity and density
 * gradients" (arXiv:1010.4124).
 *
 * TEST INFRASTRUCTURE ONLY. Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load or call this library. It shares
 * no code, header, table or helper with the GPU library; the two agree only
 * on the memory layout of their arguments:
 *   a field of 19 planes is double[19][ny][nx] (x fastest), a scalar plane is
 *   double[ny][nx].
 *
 * Every function follows the paper's definitions in the paper's order, with
 * no blocking, fusion or reordering. Compile with -O2 -ffp-contract=off and
 * without fast-math so that every expression is rounded as written.
 *
 * Where the paper is silent the following readings are taken (they are the
 * same readings the GPU library documents):
 *   - velocity directions use exact cos/sin tables (sin(pi) is exactly 0);
 *   - moments are taken from f itself (Sec. II.B defines them on f^eq; the
 *     collision conserves them, so the two coincide);
 *   - WENO5 is applied to F = v_a f with the unscaled epsilon 1e-6 of
 *     Eq. (52); for v_a < 0 the "mirror image" of Sec. III.A is the same
 *     formula on the reversed stencil;
 *   - ghost layers are three cells deep (Eq. (57) uses nodes -2, -1, 0);
 *   - reflecting walls (not in the paper) are specular with the wall on the
 *     cell face: ghost -1-m holds interior cell m of the mirrored velocity;
 *   - the outflow ghosts of Eqs. (63)-(64) are f^eq of the macroscopic state
 *     of the nearest interior node at the current time.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NV 19
#define G 3 /* ghost depth */

enum { BC_PERIODIC = 0, BC_FIXED_EQ = 1, BC_REFLECT = 2, BC_OUTFLOW = 3 };
enum { XLO = 0, XHI = 1, YLO = 2, YHI = 3 };

typedef struct {
    int32_t nx, ny;
    int32_t bc[4];            /* x-lo, x-hi, y-lo, y-hi */
    double dx, dy, dt, tau;
    double vk[3];             /* particle speeds v_1, v_2, v_3 */
    double eps;               /* WENO regulariser, 1e-6 in Eq. (52) */
    double side_state[4][4];  /* (rho, ux, uy, T) of each FIXED_EQ side */
    int32_t scheme;           /* convection: 0 WENO5, 1 first-, 2 second-order upwind */
    int32_t pad;
} orc_params;

/* ------------------------------------------------------------------------ */
/* Discrete velocity model, Eq. (5) with N = 6 and three speeds.             */
/* Index 0 is the rest particle; i = 1 + 6(k-1) + (j-1) is speed k in        */
/* direction j (angle j*pi/3), k = 1..3, j = 1..6.                           */
/* ------------------------------------------------------------------------ */
static const double COS6[6] = {0.5, -0.5, -1.0, -0.5, 0.5, 1.0};
static double sin6(int d)
{
    const double s = sqrt(3.0) / 2.0;
    const double t[6] = {s, s, 0.0, -s, -s, 0.0};
    return t[d];
}

typedef struct {
    double vx[NV], vy[NV];
    double vsq[NV];   /* |v_i|^2 = v_k^2 exactly */
    int shell[NV];    /* k (0 for the rest particle) */
    int dir[NV];      /* j-1 in 0..5, -1 for the rest particle */
    int mirx[NV];     /* index of (-vx, vy) */
    int miry[NV];     /* index of (vx, -vy) */
} vset;

static void make_vset(const double vk[3], vset* V)
{
    V->vx[0] = 0.0; V->vy[0] = 0.0; V->vsq[0] = 0.0;
    V->shell[0] = 0; V->dir[0] = -1;
    for (int k = 1; k <= 3; ++k)
        for (int d = 0; d < 6; ++d) {
            int i = 1 + 6 * (k - 1) + d;
            V->vx[i] = vk[k - 1] * COS6[d];
            V->vy[i] = vk[k - 1] * sin6(d);
            V->vsq[i] = vk[k - 1] * vk[k - 1];
            V->shell[i] = k;
            V->dir[i] = d;
        }
    /* mirror partners found by search on the exact direction tables */
    for (int i = 0; i < NV; ++i) {
        V->mirx[i] = i;
        V->miry[i] = i;
        if (i == 0) continue;
        for (int m = 1; m < NV; ++m) {
            if (V->shell[m] != V->shell[i]) continue;
            if (COS6[V->dir[m]] == -COS6[V->dir[i]] && sin6(V->dir[m]) == sin6(V->dir[i]))
                V->mirx[i] = m;
            if (COS6[V->dir[m]] == COS6[V->dir[i]] && sin6(V->dir[m]) == -sin6(V->dir[i]))
                V->miry[i] = m;
        }
    }
}

int orc_velocity_table(const double vk[3], double* vx, double* vy, double* vsq,
                       int32_t* shell, int32_t* mirx, int32_t* miry)
{
    vset V;
    make_vset(vk, &V);
    for (int i = 0; i < NV; ++i) {
        vx[i] = V.vx[i]; vy[i] = V.vy[i]; vsq[i] = V.vsq[i];
        shell[i] = V.shell[i]; mirx[i] = V.mirx[i]; miry[i] = V.miry[i];
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Weights F_k(T): Sec. II.C, Eqs. (44)-(46), the solution of the sum rules  */
/* Eqs. (40)-(43). Indices k+1, k+2 are taken cyclically in 1..3.            */
/* ------------------------------------------------------------------------ */
void orc_weights(double T, const double vk[3], double F[4])
{
    double sum = 0.0;
    for (int k = 0; k < 3; ++k) {
        double a = vk[k] * vk[k];
        double b = vk[(k + 1) % 3] * vk[(k + 1) % 3];
        double c = vk[(k + 2) % 3] * vk[(k + 2) % 3];
        double num = 24.0 * T * T * T - 4.0 * (b + c) * T * T + b * c * T;
        double den = 3.0 * a * (a - b) * (a - c);
        F[k + 1] = num / den;
    }
    sum = F[1] + F[2] + F[3];
    F[0] = 1.0 - 6.0 * sum;
}

/* dF_k/dT, the derivative of the same closed form */
static void weights_dT(double T, const double vk[3], double dF[4])
{
    for (int k = 0; k < 3; ++k) {
        double a = vk[k] * vk[k];
        double b = vk[(k + 1) % 3] * vk[(k + 1) % 3];
        double c = vk[(k + 2) % 3] * vk[(k + 2) % 3];
        double num = 72.0 * T * T - 8.0 * (b + c) * T + b * c;
        double den = 3.0 * a * (a - b) * (a - c);
        dF[k + 1] = num / den;
    }
    dF[0] = -6.0 * (dF[1] + dF[2] + dF[3]);
}

/* ------------------------------------------------------------------------ */
/* Equilibrium, Eq. (28): the third-order expansion in u,                    */
/*   f_i^eq = rho F_k [ (1-u^2/2T) + (xi/T)(1-u^2/2T) + xi^2/2T^2 + xi^3/6T^3 ] */
/* with xi = v_i . u.                                                        */
/* ------------------------------------------------------------------------ */
static void feq_cell(const vset* V, const double vk[3], double rho, double ux, double uy,
                     double T, double feq[NV])
{
    double F[4];
    orc_weights(T, vk, F);
    double b = (ux * ux + uy * uy) / (2.0 * T);
    for (int i = 0; i < NV; ++i) {
        double xi = V->vx[i] * ux + V->vy[i] * uy;
        double t0 = 1.0 - b;
        double t1 = (xi / T) * t0;
        double t2 = (xi * xi) / (2.0 * T * T);
        double t3 = (xi * xi * xi) / (6.0 * T * T * T);
        feq[i] = rho * F[V->shell[i]] * (t0 + t1 + t2 + t3);
    }
}

void orc_feq_cell(double rho, double ux, double uy, double T, const double vk[3], double* feq)
{
    vset V;
    make_vset(vk, &V);
    feq_cell(&V, vk, rho, ux, uy, T, feq);
}

/* Partial derivatives of f_i^eq with respect to (rho, ux, uy, T). */
static void feq_partials(const vset* V, const double vk[3], double rho, double ux,
                         double uy, double T, int i, double d[4])
{
    double F[4], dF[4];
    orc_weights(T, vk, F);
    weights_dT(T, vk, dF);
    int k = V->shell[i];
    double b = (ux * ux + uy * uy) / (2.0 * T);
    double xi = V->vx[i] * ux + V->vy[i] * uy;
    double P = (1.0 - b) * (1.0 + xi / T) + xi * xi / (2.0 * T * T) + xi * xi * xi / (6.0 * T * T * T);
    double P_xi = (1.0 - b) / T + xi / (T * T) + xi * xi / (2.0 * T * T * T);
    double P_b = -(1.0 + xi / T);
    double P_T = (1.0 - b) * (-xi / (T * T)) - xi * xi / (T * T * T) - xi * xi * xi / (2.0 * T * T * T * T);
    double b_ux = ux / T, b_uy = uy / T, b_T = -b / T;
    d[0] = F[k] * P;
    d[1] = rho * F[k] * (P_xi * V->vx[i] + P_b * b_ux);
    d[2] = rho * F[k] * (P_xi * V->vy[i] + P_b * b_uy);
    d[3] = rho * dF[k] * P + rho * F[k] * (P_T + P_b * b_T);
}

/* ------------------------------------------------------------------------ */
/* Macroscopic moments, Eq. (10): rho = sum f, rho u = sum f v,              */
/* rho T = sum f |v - u|^2 / 2, evaluated as E/rho - |u|^2/2 with            */
/* E = sum f |v|^2 / 2.                                                      */
/* ------------------------------------------------------------------------ */
static void moments_cell(const vset* V, const double* f, ptrdiff_t stride, double m[4],
                         double raw[4])
{
    double rho = 0.0, jx = 0.0, jy = 0.0, E = 0.0;
    for (int i = 0; i < NV; ++i) {
        double fi = f[i * stride];
        rho += fi;
        jx += fi * V->vx[i];
        jy += fi * V->vy[i];
        E += fi * (0.5 * V->vsq[i]);
    }
    double ux = jx / rho, uy = jy / rho;
    double T = E / rho - 0.5 * (ux * ux + uy * uy);
    m[0] = rho; m[1] = ux; m[2] = uy; m[3] = T;
    if (raw) { raw[0] = rho; raw[1] = jx; raw[2] = jy; raw[3] = E; }
}

void orc_moments_cell(const double* f, const double vk[3], double* m)
{
    vset V;
    make_vset(vk, &V);
    moments_cell(&V, f, 1, m, NULL);
}

/* ------------------------------------------------------------------------ */
/* WENO5 numerical flux at face I+1/2 for an upwind-from-the-left stencil    */
/* (a,b,c,d,e) = (F_{I-2}, F_{I-1}, F_I, F_{I+1}, F_{I+2}):                   */
/* candidates Eqs. (49)-(51), weights Eq. (52), smoothness Eqs. (53)-(55),   */
/* convex combination Eq. (48).                                              */
/* ------------------------------------------------------------------------ */
static const double DELTA[3] = {1.0 / 10.0, 3.0 / 5.0, 3.0 / 10.0};

double orc_weno5(double a, double b, double c, double d, double e, double eps)
{
    double h1 = (1.0 / 3.0) * a - (7.0 / 6.0) * b + (11.0 / 6.0) * c;
    double h2 = -(1.0 / 6.0) * b + (5.0 / 6.0) * c + (1.0 / 3.0) * d;
    double h3 = (1.0 / 3.0) * c + (5.0 / 6.0) * d - (1.0 / 6.0) * e;
    double A1 = a - 2.0 * b + c, B1 = a - 4.0 * b + 3.0 * c;
    double A2 = b - 2.0 * c + d, B2 = b - d;
    double A3 = c - 2.0 * d + e, B3 = 3.0 * c - 4.0 * d + e;
    double s1 = (13.0 / 12.0) * A1 * A1 + (1.0 / 4.0) * B1 * B1;
    double s2 = (13.0 / 12.0) * A2 * A2 + (1.0 / 4.0) * B2 * B2;
    double s3 = (13.0 / 12.0) * A3 * A3 + (1.0 / 4.0) * B3 * B3;
    double wt1 = DELTA[0] / ((eps + s1) * (eps + s1));
    double wt2 = DELTA[1] / ((eps + s2) * (eps + s2));
    double wt3 = DELTA[2] / ((eps + s3) * (eps + s3));
    double S = wt1 + wt2 + wt3;
    double w1 = wt1 / S, w2 = wt2 / S, w3 = wt3 / S;
    return w1 * h1 + w2 * h2 + w3 * h3;
}

/* Reverse mode of orc_weno5: adds hbar * dh/d(a..e) into g[0..4]. */
static void weno5_bar(double a, double b, double c, double d, double e, double eps,
                      double hbar, double g[5])
{
    double h1 = (1.0 / 3.0) * a - (7.0 / 6.0) * b + (11.0 / 6.0) * c;
    double h2 = -(1.0 / 6.0) * b + (5.0 / 6.0) * c + (1.0 / 3.0) * d;
    double h3 = (1.0 / 3.0) * c + (5.0 / 6.0) * d - (1.0 / 6.0) * e;
    double A1 = a - 2.0 * b + c, B1 = a - 4.0 * b + 3.0 * c;
    double A2 = b - 2.0 * c + d, B2 = b - d;
    double A3 = c - 2.0 * d + e, B3 = 3.0 * c - 4.0 * d + e;
    double s1 = (13.0 / 12.0) * A1 * A1 + (1.0 / 4.0) * B1 * B1;
    double s2 = (13.0 / 12.0) * A2 * A2 + (1.0 / 4.0) * B2 * B2;
    double s3 = (13.0 / 12.0) * A3 * A3 + (1.0 / 4.0) * B3 * B3;
    double q1 = eps + s1, q2 = eps + s2, q3 = eps + s3;
    double wt1 = DELTA[0] / (q1 * q1);
    double wt2 = DELTA[1] / (q2 * q2);
    double wt3 = DELTA[2] / (q3 * q3);
    double S = wt1 + wt2 + wt3;
    double w1 = wt1 / S, w2 = wt2 / S, w3 = wt3 / S;
    double h = w1 * h1 + w2 * h2 + w3 * h3;
    /* h = sum w_q h_q */
    double h1b = hbar * w1, h2b = hbar * w2, h3b = hbar * w3;
    double w1b = hbar * h1, w2b = hbar * h2, w3b = hbar * h3;
    /* w_q = wt_q / S  =>  wt_q_bar = (w_q_bar - sum_p w_p_bar w_p) / S */
    double dot = w1b * w1 + w2b * w2 + w3b * w3;
    double wt1b = (w1b - dot) / S, wt2b = (w2b - dot) / S, wt3b = (w3b - dot) / S;
    (void)h;
    /* wt_q = delta_q / q_q^2  =>  q_q_bar = -2 delta_q / q_q^3 * wt_q_bar */
    double s1b = wt1b * (-2.0 * DELTA[0] / (q1 * q1 * q1));
    double s2b = wt2b * (-2.0 * DELTA[1] / (q2 * q2 * q2));
    double s3b = wt3b * (-2.0 * DELTA[2] / (q3 * q3 * q3));
    /* s_q = 13/12 A_q^2 + 1/4 B_q^2 */
    double A1b = s1b * (13.0 / 6.0) * A1, B1b = s1b * 0.5 * B1;
    double A2b = s2b * (13.0 / 6.0) * A2, B2b = s2b * 0.5 * B2;
    double A3b = s3b * (13.0 / 6.0) * A3, B3b = s3b * 0.5 * B3;
    /* A1 = a-2b+c, B1 = a-4b+3c */
    g[0] += A1b + B1b;
    g[1] += -2.0 * A1b - 4.0 * B1b;
    g[2] += A1b + 3.0 * B1b;
    /* A2 = b-2c+d, B2 = b-d */
    g[1] += A2b + B2b;
    g[2] += -2.0 * A2b;
    g[3] += A2b - B2b;
    /* A3 = c-2d+e, B3 = 3c-4d+e */
    g[2] += A3b + 3.0 * B3b;
    g[3] += -2.0 * A3b - 4.0 * B3b;
    g[4] += A3b + B3b;
    /* candidate fluxes */
    g[0] += (1.0 / 3.0) * h1b;
    g[1] += -(7.0 / 6.0) * h1b - (1.0 / 6.0) * h2b;
    g[2] += (11.0 / 6.0) * h1b + (5.0 / 6.0) * h2b + (1.0 / 3.0) * h3b;
    g[3] += (1.0 / 3.0) * h2b + (5.0 / 6.0) * h3b;
    g[4] += -(1.0 / 6.0) * h3b;
}

void orc_weno5_grad(double a, double b, double c, double d, double e, double eps, double* g)
{
    for (int k = 0; k < 5; ++k) g[k] = 0.0;
    weno5_bar(a, b, c, d, e, eps, 1.0, g);
}

/* ------------------------------------------------------------------------ */
/* Comparison schemes of Sec. III.B (Fig. 2): the numerical flux at face      */
/* I+1/2 from the upwind-ordered samples (a, b, c, d, e) = F_{I-2..I+2} (the  */
/* same ordering as the WENO5 face; c is the upwind cell I).                  */
/*   first-order upwind:  h = c                                               */
/*   second-order upwind: h = c + (c - b) / 2   (linear extrapolation from    */
/*                        the two upwind cells)                               */
/* ------------------------------------------------------------------------ */
static double face_value(int scheme, double a, double b, double c, double d, double e, double eps)
{
    if (scheme == 1) return c;
    if (scheme == 2) return c + 0.5 * (c - b);
    return orc_weno5(a, b, c, d, e, eps);
}

/* Face fluxes of a periodic line of n values F[0..n-1] with any scheme:
 * h[I] is the flux at face I+1/2, upwinded to the left for sign >= 0 and to
 * the right (mirror image) for sign < 0. */
void orc_scheme_periodic_line(const double* F, int n, int sign, int scheme, double eps, double* h)
{
#define W(j) F[(((j) % n) + n) % n]
    for (int I = 0; I < n; ++I) {
        if (sign >= 0)
            h[I] = face_value(scheme, W(I - 2), W(I - 1), W(I), W(I + 1), W(I + 2), eps);
        else
            h[I] = face_value(scheme, W(I + 3), W(I + 2), W(I + 1), W(I), W(I - 1), eps);
    }
#undef W
}

/* Face fluxes of a periodic line of n values F[0..n-1]: h[I] is the flux at
 * face I+1/2, upwinded to the left for sign >= 0 and to the right (mirror
 * image) for sign < 0. */
void orc_weno_periodic_line(const double* F, int n, int sign, double eps, double* h)
{
#define W(j) F[(((j) % n) + n) % n]
    for (int I = 0; I < n; ++I) {
        if (sign >= 0)
            h[I] = orc_weno5(W(I - 2), W(I - 1), W(I), W(I + 1), W(I + 2), eps);
        else
            h[I] = orc_weno5(W(I + 3), W(I + 2), W(I + 1), W(I), W(I - 1), eps);
    }
#undef W
}

/* ------------------------------------------------------------------------ */
/* Ghost layers: padded planes of (ny+2G) x (nx+2G), corners unused (NaN).   */
/* ------------------------------------------------------------------------ */
typedef struct {
    int nx, ny, px, py;
} grid;

static inline ptrdiff_t P(const grid* g, int i, int y, int x)
{
    return ((ptrdiff_t)i * g->py + (y + G)) * g->px + (x + G);
}
static inline ptrdiff_t C(const grid* g, int i, int y, int x)
{
    return ((ptrdiff_t)i * g->ny + y) * g->nx + x;
}
static inline int wrap(int a, int n) { return ((a % n) + n) % n; }

static int check_params(const orc_params* p)
{
    if (!p || p->nx < 1 || p->ny < 1) return -1;
    if (!(p->dt > 0.0) || !(p->tau > 0.0) || !(p->dx > 0.0) || !(p->dy > 0.0)) return -1;
    for (int s = 0; s < 4; ++s) {
        if (p->bc[s] < 0 || p->bc[s] > 3) return -1;
        int n = (s < 2) ? p->nx : p->ny;
        if (p->bc[s] != BC_PERIODIC && n < G) return -1;
    }
    /* periodic must be periodic on both ends of an axis */
    if ((p->bc[XLO] == BC_PERIODIC) != (p->bc[XHI] == BC_PERIODIC)) return -1;
    if ((p->bc[YLO] == BC_PERIODIC) != (p->bc[YHI] == BC_PERIODIC)) return -1;
    if (p->vk[0] == p->vk[1] || p->vk[1] == p->vk[2] || p->vk[0] == p->vk[2]) return -1;
    if (p->scheme < 0 || p->scheme > 2) return -1;
    return 0;
}

/* Fill the ghost value of plane i at padded position (y, x) that lies on
 * side s, m cells beyond the boundary (m = 0, 1, 2). */
static void fill_ghosts(const orc_params* p, const vset* V, const grid* g, const double* f,
                        double* fp, double geq[4][NV])
{
    const int nx = g->nx, ny = g->ny;
    for (ptrdiff_t k = 0; k < (ptrdiff_t)NV * g->px * g->py; ++k) fp[k] = NAN;
    for (int i = 0; i < NV; ++i)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) fp[P(g, i, y, x)] = f[C(g, i, y, x)];
    /* x ghosts on every interior row */
    for (int y = 0; y < ny; ++y) {
        double feq_lo[NV], feq_hi[NV];
        if (p->bc[XLO] == BC_OUTFLOW) {
            double m[4];
            moments_cell(V, f + C(g, 0, y, 0), (ptrdiff_t)nx * ny, m, NULL);
            feq_cell(V, p->vk, m[0], m[1], m[2], m[3], feq_lo);
        }
        if (p->bc[XHI] == BC_OUTFLOW) {
            double m[4];
            moments_cell(V, f + C(g, 0, y, nx - 1), (ptrdiff_t)nx * ny, m, NULL);
            feq_cell(V, p->vk, m[0], m[1], m[2], m[3], feq_hi);
        }
        for (int i = 0; i < NV; ++i)
            for (int m = 0; m < G; ++m) {
                double lo = 0.0, hi = 0.0;
                switch (p->bc[XLO]) {
                case BC_PERIODIC: lo = f[C(g, i, y, wrap(-1 - m, nx))]; break;
                case BC_FIXED_EQ: lo = geq[XLO][i]; break;
                case BC_REFLECT: lo = f[C(g, V->mirx[i], y, m)]; break;
                case BC_OUTFLOW: lo = feq_lo[i]; break;
                }
                switch (p->bc[XHI]) {
                case BC_PERIODIC: hi = f[C(g, i, y, wrap(nx + m, nx))]; break;
                case BC_FIXED_EQ: hi = geq[XHI][i]; break;
                case BC_REFLECT: hi = f[C(g, V->mirx[i], y, nx - 1 - m)]; break;
                case BC_OUTFLOW: hi = feq_hi[i]; break;
                }
                fp[P(g, i, y, -1 - m)] = lo;
                fp[P(g, i, y, nx + m)] = hi;
            }
    }
    /* y ghosts on every interior column */
    for (int x = 0; x < nx; ++x) {
        double feq_lo[NV], feq_hi[NV];
        if (p->bc[YLO] == BC_OUTFLOW) {
            double m[4];
            moments_cell(V, f + C(g, 0, 0, x), (ptrdiff_t)nx * ny, m, NULL);
            feq_cell(V, p->vk, m[0], m[1], m[2], m[3], feq_lo);
        }
        if (p->bc[YHI] == BC_OUTFLOW) {
            double m[4];
            moments_cell(V, f + C(g, 0, ny - 1, x), (ptrdiff_t)nx * ny, m, NULL);
            feq_cell(V, p->vk, m[0], m[1], m[2], m[3], feq_hi);
        }
        for (int i = 0; i < NV; ++i)
            for (int m = 0; m < G; ++m) {
                double lo = 0.0, hi = 0.0;
                switch (p->bc[YLO]) {
                case BC_PERIODIC: lo = f[C(g, i, wrap(-1 - m, ny), x)]; break;
                case BC_FIXED_EQ: lo = geq[YLO][i]; break;
                case BC_REFLECT: lo = f[C(g, V->miry[i], m, x)]; break;
                case BC_OUTFLOW: lo = feq_lo[i]; break;
                }
                switch (p->bc[YHI]) {
                case BC_PERIODIC: hi = f[C(g, i, wrap(ny + m, ny), x)]; break;
                case BC_FIXED_EQ: hi = geq[YHI][i]; break;
                case BC_REFLECT: hi = f[C(g, V->miry[i], ny - 1 - m, x)]; break;
                case BC_OUTFLOW: hi = feq_hi[i]; break;
                }
                fp[P(g, i, -1 - m, x)] = lo;
                fp[P(g, i, ny + m, x)] = hi;
            }
    }
}

static void side_equilibria(const orc_params* p, const vset* V, double geq[4][NV])
{
    for (int s = 0; s < 4; ++s) {
        for (int i = 0; i < NV; ++i) geq[s][i] = 0.0;
        if (p->bc[s] == BC_FIXED_EQ) {
            const double* st = p->side_state[s];
            feq_cell(V, p->vk, st[0], st[1], st[2], st[3], geq[s]);
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Initialisation f = f^eq(rho, u, T) on every cell.                         */
/* ------------------------------------------------------------------------ */
int orc_init(const orc_params* p, const double* rho, const double* ux, const double* uy,
             const double* T, double* f)
{
    if (check_params(p)) return -1;
    vset V;
    make_vset(p->vk, &V);
    const ptrdiff_t n = (ptrdiff_t)p->nx * p->ny;
    for (ptrdiff_t c = 0; c < n; ++c) {
        double fe[NV];
        feq_cell(&V, p->vk, rho[c], ux[c], uy[c], T[c], fe);
        for (int i = 0; i < NV; ++i) f[i * n + c] = fe[i];
    }
    return 0;
}

int orc_moments(const orc_params* p, const double* f, double* rho, double* ux, double* uy,
                double* T)
{
    if (check_params(p)) return -1;
    vset V;
    make_vset(p->vk, &V);
    const ptrdiff_t n = (ptrdiff_t)p->nx * p->ny;
    for (ptrdiff_t c = 0; c < n; ++c) {
        double m[4];
        moments_cell(&V, f + c, n, m, NULL);
        rho[c] = m[0]; ux[c] = m[1]; uy[c] = m[2]; T[c] = m[3];
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* One forward-Euler step, Eq. (47):                                         */
/*   f^{n+1} = f - dt/dx (h^x_{I+1/2} - h^x_{I-1/2})                         */
/*               - dt/dy (h^y_{J+1/2} - h^y_{J-1/2}) - dt/tau (f - f^eq)      */
/* with the fluxes of Eq. (48) upwinded by the sign of v_a.                  */
/* ------------------------------------------------------------------------ */
static double face_flux_x(const grid* g, const double* fp, int i, double v, int y, int x,
                          double eps, int scheme)
{
    /* face x+1/2 of row y, F = v f */
#define FX(xx) (v * fp[P(g, i, y, (xx))])
    if (v >= 0.0)
        return face_value(scheme, FX(x - 2), FX(x - 1), FX(x), FX(x + 1), FX(x + 2), eps);
    return face_value(scheme, FX(x + 3), FX(x + 2), FX(x + 1), FX(x), FX(x - 1), eps);
#undef FX
}

static double face_flux_y(const grid* g, const double* fp, int i, double v, int y, int x,
                          double eps, int scheme)
{
    /* face y+1/2 of column x */
#define FY(yy) (v * fp[P(g, i, (yy), x)])
    if (v >= 0.0)
        return face_value(scheme, FY(y - 2), FY(y - 1), FY(y), FY(y + 1), FY(y + 2), eps);
    return face_value(scheme, FY(y + 3), FY(y + 2), FY(y + 1), FY(y), FY(y - 1), eps);
#undef FY
}

static int step_once(const orc_params* p, const vset* V, double geq[4][NV], const double* f,
                     double* fo, double* fp, double* mom, int nthreads)
{
    grid g = {p->nx, p->ny, p->nx + 2 * G, p->ny + 2 * G};
    const int nx = p->nx, ny = p->ny;
    const ptrdiff_t n = (ptrdiff_t)nx * ny;
    const double cx = p->dt / p->dx, cy = p->dt / p->dy, ct = p->dt / p->tau;
    (void)nthreads;
    fill_ghosts(p, V, &g, f, fp, geq);
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            double m[4];
            moments_cell(V, f + (ptrdiff_t)y * nx + x, n, m, NULL);
            for (int k = 0; k < 4; ++k) mom[4 * ((ptrdiff_t)y * nx + x) + k] = m[k];
        }
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const double* m = mom + 4 * ((ptrdiff_t)y * nx + x);
            double fe[NV];
            feq_cell(V, p->vk, m[0], m[1], m[2], m[3], fe);
            for (int i = 0; i < NV; ++i) {
                double dhx = 0.0, dhy = 0.0;
                if (V->vx[i] != 0.0)
                    dhx = face_flux_x(&g, fp, i, V->vx[i], y, x, p->eps, p->scheme) -
                          face_flux_x(&g, fp, i, V->vx[i], y, x - 1, p->eps, p->scheme);
                if (V->vy[i] != 0.0)
                    dhy = face_flux_y(&g, fp, i, V->vy[i], y, x, p->eps, p->scheme) -
                          face_flux_y(&g, fp, i, V->vy[i], y - 1, x, p->eps, p->scheme);
                double fi = f[C(&g, i, y, x)];
                fo[C(&g, i, y, x)] = fi - cx * dhx - cy * dhy - ct * (fi - fe[i]);
            }
        }
    return 0;
}

/* nsteps forward steps from f_in; the result lands in f_out. f_in is not
 * modified. nthreads only splits rows between threads: every cell is
 * computed identically, so results do not depend on it. */
int orc_step(const orc_params* p, const double* f_in, double* f_out, int nsteps, int nthreads)
{
    if (check_params(p) || nsteps < 0) return -1;
    if (nthreads < 1) nthreads = 1;
    vset V;
    make_vset(p->vk, &V);
    double geq[4][NV];
    side_equilibria(p, &V, geq);
    const ptrdiff_t n = (ptrdiff_t)p->nx * p->ny;
    const ptrdiff_t np = (ptrdiff_t)(p->nx + 2 * G) * (p->ny + 2 * G);
    double* fp = (double*)malloc(sizeof(double) * NV * np);
    double* mom = (double*)malloc(sizeof(double) * 4 * n);
    double* a = (double*)malloc(sizeof(double) * NV * n);
    double* b = (double*)malloc(sizeof(double) * NV * n);
    if (!fp || !mom || !a || !b) { free(fp); free(mom); free(a); free(b); return -3; }
    memcpy(a, f_in, sizeof(double) * NV * n);
    for (int s = 0; s < nsteps; ++s) {
        step_once(p, &V, geq, a, b, fp, mom, nthreads);
        double* t = a; a = b; b = t;
    }
    memcpy(f_out, a, sizeof(double) * NV * n);
    free(fp); free(mom); free(a); free(b);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Transverse kinetic energy E_y = sum over cells of rho u_y^2 / 2 dx dy and */
/* its cell maximum (the diagnostic of Sec. IV with the interface normal    */
/* along y).                                                                 */
/* ------------------------------------------------------------------------ */
int orc_kinetic_y(const orc_params* p, const double* f, double* out2)
{
    if (check_params(p)) return -1;
    vset V;
    make_vset(p->vk, &V);
    const ptrdiff_t n = (ptrdiff_t)p->nx * p->ny;
    double sum = 0.0, mx = 0.0;
    for (ptrdiff_t c = 0; c < n; ++c) {
        double m[4];
        moments_cell(&V, f + c, n, m, NULL);
        double e = 0.5 * m[0] * m[2] * m[2];
        sum += e * p->dx * p->dy;
        if (e > mx) mx = e;
    }
    out2[0] = sum;
    out2[1] = mx;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Reverse mode (discrete adjoint) of one step, written as the transpose of  */
/* step_once taken statement by statement in reverse order (scatter form):  */
/*   lam_n = (dS/df^n)^T lam_{n+1} + w dE_y/df^n.                           */
/* Fixed-eq ghosts are constants; periodic and reflecting ghosts send their  */
/* adjoint back to the interior cell they copy. Outflow is not supported.   */
/* ------------------------------------------------------------------------ */
int orc_adjoint_step(const orc_params* p, const double* f_n, const double* lam1, double w,
                     double* lam_n)
{
    if (check_params(p)) return -1;
    if (p->scheme != 0) return -2; /* the reverse mode covers WENO5 only */
    for (int s = 0; s < 4; ++s)
        if (p->bc[s] == BC_OUTFLOW) return -2;
    vset V;
    make_vset(p->vk, &V);
    double geq[4][NV];
    side_equilibria(p, &V, geq);
    const int nx = p->nx, ny = p->ny;
    grid g = {nx, ny, nx + 2 * G, ny + 2 * G};
    const ptrdiff_t n = (ptrdiff_t)nx * ny;
    const ptrdiff_t np = (ptrdiff_t)g.px * g.py;
    const double cx = p->dt / p->dx, cy = p->dt / p->dy, ct = p->dt / p->tau;
    double* fp = (double*)malloc(sizeof(double) * NV * np);
    double* lp = (double*)calloc((size_t)NV * np, sizeof(double));
    double* mom = (double*)malloc(sizeof(double) * 4 * n);
    double* mbar = (double*)calloc((size_t)4 * n, sizeof(double));
    double* hbx = (double*)malloc(sizeof(double) * (size_t)(nx + 1) * ny);
    double* hby = (double*)malloc(sizeof(double) * (size_t)nx * (ny + 1));
    if (!fp || !lp || !mom || !mbar || !hbx || !hby) {
        free(fp); free(lp); free(mom); free(mbar); free(hbx); free(hby);
        return -3;
    }
    fill_ghosts(p, &V, &g, f_n, fp, geq);
    for (ptrdiff_t c = 0; c < n; ++c) moments_cell(&V, f_n + c, n, mom + 4 * c, NULL);

    for (int i = 0; i < NV; ++i) {
        /* fo = fi - cx*dhx - cy*dhy - ct*(fi - fe) */
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                double L = lam1[C(&g, i, y, x)];
                double* m = mom + 4 * ((ptrdiff_t)y * nx + x);
                lp[P(&g, i, y, x)] += L;            /* the leading fi */
                lp[P(&g, i, y, x)] += -ct * L;      /* -ct * fi */
                double fe_bar = ct * L;             /* +ct * fe */
                double d[4];
                feq_partials(&V, p->vk, m[0], m[1], m[2], m[3], i, d);
                double* mb = mbar + 4 * ((ptrdiff_t)y * nx + x);
                for (int k = 0; k < 4; ++k) mb[k] += fe_bar * d[k];
            }
        /* x convection: dhx = h(x+1/2) - h(x-1/2), face index X = x+1 for x+1/2 */
        if (V.vx[i] != 0.0) {
            const double v = V.vx[i];
            for (ptrdiff_t k = 0; k < (ptrdiff_t)(nx + 1) * ny; ++k) hbx[k] = 0.0;
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    double L = lam1[C(&g, i, y, x)];
                    hbx[(ptrdiff_t)y * (nx + 1) + (x + 1)] += -cx * L;
                    hbx[(ptrdiff_t)y * (nx + 1) + x] += cx * L;
                }
            for (int y = 0; y < ny; ++y)
                for (int X = 0; X <= nx; ++X) {
                    int x = X - 1; /* face x+1/2 */
                    double hb = hbx[(ptrdiff_t)y * (nx + 1) + X];
                    int pos[5];
                    if (v >= 0.0) { for (int k = 0; k < 5; ++k) pos[k] = x - 2 + k; }
                    else { for (int k = 0; k < 5; ++k) pos[k] = x + 3 - k; }
                    double s[5], gr[5] = {0, 0, 0, 0, 0};
                    for (int k = 0; k < 5; ++k) s[k] = v * fp[P(&g, i, y, pos[k])];
                    weno5_bar(s[0], s[1], s[2], s[3], s[4], p->eps, hb, gr);
                    for (int k = 0; k < 5; ++k) lp[P(&g, i, y, pos[k])] += v * gr[k];
                }
        }
        if (V.vy[i] != 0.0) {
            const double v = V.vy[i];
            for (ptrdiff_t k = 0; k < (ptrdiff_t)nx * (ny + 1); ++k) hby[k] = 0.0;
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    double L = lam1[C(&g, i, y, x)];
                    hby[(ptrdiff_t)(y + 1) * nx + x] += -cy * L;
                    hby[(ptrdiff_t)y * nx + x] += cy * L;
                }
            for (int Y = 0; Y <= ny; ++Y)
                for (int x = 0; x < nx; ++x) {
                    int y = Y - 1;
                    double hb = hby[(ptrdiff_t)Y * nx + x];
                    int pos[5];
                    if (v >= 0.0) { for (int k = 0; k < 5; ++k) pos[k] = y - 2 + k; }
                    else { for (int k = 0; k < 5; ++k) pos[k] = y + 3 - k; }
                    double s[5], gr[5] = {0, 0, 0, 0, 0};
                    for (int k = 0; k < 5; ++k) s[k] = v * fp[P(&g, i, pos[k], x)];
                    weno5_bar(s[0], s[1], s[2], s[3], s[4], p->eps, hb, gr);
                    for (int k = 0; k < 5; ++k) lp[P(&g, i, pos[k], x)] += v * gr[k];
                }
        }
    }
    /* (rho, ux, uy, T) <- (rho, jx, jy, E) <- f, per cell */
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            ptrdiff_t c = (ptrdiff_t)y * nx + x;
            double raw[4], m[4];
            moments_cell(&V, f_n + c, n, m, raw);
            double rho = raw[0], jx = raw[1], jy = raw[2], E = raw[3];
            double ux = m[1], uy = m[2];
            double rb = mbar[4 * c + 0], uxb = mbar[4 * c + 1], uyb = mbar[4 * c + 2],
                   Tb = mbar[4 * c + 3];
            /* T = E/rho - 0.5 (ux^2 + uy^2) */
            double Eb = Tb / rho;
            rb += Tb * (-E / (rho * rho));
            uxb += Tb * (-ux);
            uyb += Tb * (-uy);
            /* ux = jx/rho, uy = jy/rho */
            double jxb = uxb / rho, jyb = uyb / rho;
            rb += uxb * (-jx / (rho * rho)) + uyb * (-jy / (rho * rho));
            for (int i = 0; i < NV; ++i)
                lp[P(&g, i, y, x)] += rb + jxb * V.vx[i] + jyb * V.vy[i] + Eb * (0.5 * V.vsq[i]);
        }
    /* transpose of the ghost fill */
    for (int y = 0; y < ny; ++y)
        for (int i = 0; i < NV; ++i)
            for (int m = 0; m < G; ++m) {
                double glo = lp[P(&g, i, y, -1 - m)], ghi = lp[P(&g, i, y, nx + m)];
                switch (p->bc[XLO]) {
                case BC_PERIODIC: lp[P(&g, i, y, wrap(-1 - m, nx))] += glo; break;
                case BC_REFLECT: lp[P(&g, V.mirx[i], y, m)] += glo; break;
                default: break;
                }
                switch (p->bc[XHI]) {
                case BC_PERIODIC: lp[P(&g, i, y, wrap(nx + m, nx))] += ghi; break;
                case BC_REFLECT: lp[P(&g, V.mirx[i], y, nx - 1 - m)] += ghi; break;
                default: break;
                }
            }
    for (int x = 0; x < nx; ++x)
        for (int i = 0; i < NV; ++i)
            for (int m = 0; m < G; ++m) {
                double glo = lp[P(&g, i, -1 - m, x)], ghi = lp[P(&g, i, ny + m, x)];
                switch (p->bc[YLO]) {
                case BC_PERIODIC: lp[P(&g, i, wrap(-1 - m, ny), x)] += glo; break;
                case BC_REFLECT: lp[P(&g, V.miry[i], m, x)] += glo; break;
                default: break;
                }
                switch (p->bc[YHI]) {
                case BC_PERIODIC: lp[P(&g, i, wrap(ny + m, ny), x)] += ghi; break;
                case BC_REFLECT: lp[P(&g, V.miry[i], ny - 1 - m, x)] += ghi; break;
                default: break;
                }
            }
    /* objective term w dE_y/df, E_y = sum rho uy^2/2 dx dy */
    for (int i = 0; i < NV; ++i)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                double uy = mom[4 * ((ptrdiff_t)y * nx + x) + 2];
                double dE = p->dx * p->dy * (uy * V.vy[i] - 0.5 * uy * uy);
                lam_n[C(&g, i, y, x)] = lp[P(&g, i, y, x)] + w * dE;
            }
    free(fp); free(lp); free(mom); free(mbar); free(hbx); free(hby);
    return 0;
}

/* Gradient of E_y with respect to f (the objective term alone). */
int orc_kinetic_y_grad(const orc_params* p, const double* f, double* g_out)
{
    if (check_params(p)) return -1;
    vset V;
    make_vset(p->vk, &V);
    const ptrdiff_t n = (ptrdiff_t)p->nx * p->ny;
    for (ptrdiff_t c = 0; c < n; ++c) {
        double m[4];
        moments_cell(&V, f + c, n, m, NULL);
        double uy = m[2];
        for (int i = 0; i < NV; ++i)
            g_out[i * n + c] = p->dx * p->dy * (uy * V.vy[i] - 0.5 * uy * uy);
    }
    return 0;
}

/* Vector-Jacobian product of orc_init: g_q = sum_i lam_i d f_i^eq / d q for
 * q in (rho, ux, uy, T), per cell. */
int orc_init_vjp(const orc_params* p, const double* rho, const double* ux, const double* uy,
                 const double* T, const double* lam0, double* g_rho, double* g_ux,
                 double* g_uy, double* g_T)
{
    if (check_params(p)) return -1;
    vset V;
    make_vset(p->vk, &V);
    const ptrdiff_t n = (ptrdiff_t)p->nx * p->ny;
    for (ptrdiff_t c = 0; c < n; ++c) {
        double acc[4] = {0, 0, 0, 0};
        for (int i = 0; i < NV; ++i) {
            double d[4];
            feq_partials(&V, p->vk, rho[c], ux[c], uy[c], T[c], i, d);
            for (int k = 0; k < 4; ++k) acc[k] += lam0[i * n + c] * d[k];
        }
        g_rho[c] = acc[0]; g_ux[c] = acc[1]; g_uy[c] = acc[2]; g_T[c] = acc[3];
    }
    return 0;
}

/* Partials of one equilibrium value, exposed for the tests. */
void orc_feq_partials(double rho, double ux, double uy, double T, const double vk[3], int i,
                      double* d)
{
    vset V;
    make_vset(vk, &V);
    feq_partials(&V, vk, rho, ux, uy, T, i, d);
}
