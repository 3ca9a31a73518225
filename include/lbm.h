/*
 * lbm.h -- C-ABI of the MI355X (gfx950) D2V19 + WENO5 finite-difference
 * lattice-Boltzmann library (liblbm_hip.so).
 *
 * The method is the FDLB model of Gan, Xu, Zhang and Li (arXiv:1010.4124):
 * 19 discrete velocities (Sec. II.A, Eq. (5)), closed-form weights F_k(T)
 * (Sec. II.C, Eqs. (44)-(46)), third-order equilibrium (Eq. (28)), BGK
 * collision (Eq. (4)), fifth-order WENO fluxes upwinded by the sign of each
 * velocity component (Sec. III.A, Eqs. (48)-(55)) and forward-Euler time
 * stepping (Eq. (47)).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All field pointers are DEVICE pointers to float64 memory owned by the
 *    caller. The library never frees or reallocates them.
 *  - A distribution field is 19 planes: element (i, y, x) sits at
 *    f[i*ny*nx + y*nx + x] (structure of arrays, x fastest). A scalar field
 *    is one plane, element (y, x) at p[y*nx + x].
 *  - Velocity i = 0 is the rest particle; i = 1 + 6(k-1) + (j-1) is speed
 *    v_k (k = 1..3) in direction j (angle j*pi/3, j = 1..6).
 *  - Every call is asynchronous on `stream` (a hipStream_t; NULL is the
 *    default stream). Device faults surface at the caller's next
 *    synchronisation.
 *  - Return value: LBM_OK (0) or a negative LBM_E* code; the message of the
 *    last failure on the calling thread is returned by lbm_last_error().
 *    No C++ exception crosses this interface.
 *  - Input and output buffers of one call must not overlap (LBM_EINVAL where
 *    the base pointers coincide).
 *  - Calls on one context must not run concurrently on different streams:
 *    a context's scratch buffers are shared by its calls.
 */
#ifndef LBM_H
#define LBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void* lbm_stream; /* hipStream_t */

enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,       /* bad argument: null pointer, sizes, aliasing, parameters */
    LBM_EUNSUPPORTED = -2, /* valid request the library does not implement */
    LBM_EHIP = -3,         /* HIP runtime error (message in lbm_last_error) */
    LBM_ENOMEM = -4,       /* device allocation failed */
    LBM_ENONFINITE = -5,   /* lbm_check_state: a NaN or infinity in the state */
    LBM_ENONPHYS = -6      /* lbm_check_state: a cell with rho <= 0 or T <= 0 */
};

/* Boundary treatment of one side. */
enum {
    LBM_BC_PERIODIC = 0, /* wrap; both sides of an axis must be periodic */
    LBM_BC_FIXED_EQ = 1, /* ghosts hold f^eq of side_state: Sec. III.B, Eqs. (57)-(58) */
    LBM_BC_REFLECT = 2,  /* specular wall on the cell face: ghost -1-m holds
                            interior cell m of the mirrored velocity (the
                            paper has no walls; this is the shear-layer setup) */
    LBM_BC_OUTFLOW = 3   /* zeroth-order extrapolation, Sec. IV.A, Eqs. (63)-(64):
                            the three ghost layers hold f^eq of the moments
                            of the nearest interior cell at the current time
                            (forward calls only: lbm_adjoint_step returns
                            LBM_EUNSUPPORTED) */
};

enum { LBM_XLO = 0, LBM_XHI = 1, LBM_YLO = 2, LBM_YHI = 3 };

typedef struct {
    int32_t nx, ny;            /* cells; each >= 1, >= 3 on an axis with a non-periodic side */
    int32_t bc[4];             /* LBM_BC_* of x-lo, x-hi, y-lo, y-hi */
    double dx, dy, dt, tau;    /* > 0 */
    double vk[3];              /* particle speeds, distinct and > 0; the paper uses 1, 2, 3 */
    double weno_eps;           /* WENO regulariser, 1e-6 in Eq. (52); > 0 */
    double side_state[4][4];   /* (rho, ux, uy, T) of each LBM_BC_FIXED_EQ side */
    int32_t ke_axis;           /* velocity component u_n of the kinetic-energy
                                  diagnostics rho u_n^2 / 2: 0 = u_y, 1 = u_x
                                  (the interface normal; Sec. IV uses u_x) */
    int32_t scheme;            /* convection flux of lbm_step (Sec. III.B, Fig. 2):
                                  LBM_SCHEME_WENO5 (the method), or one of the
                                  two upwind schemes the paper compares it with;
                                  anything else is LBM_EINVAL. Only WENO5 has a
                                  reverse step, step variants and a batch path
                                  (LBM_EUNSUPPORTED otherwise) */
} lbm_params;

enum {
    LBM_SCHEME_WENO5 = 0,    /* fifth-order WENO faces, Eqs. (48)-(55) */
    LBM_SCHEME_UPWIND1 = 1,  /* first-order upwind: the face takes the upwind
                                cell's flux v f */
    LBM_SCHEME_UPWIND2 = 2   /* second-order upwind: the upwind cell's flux
                                plus half its difference to the next cell
                                upstream, F_I + (F_I - F_{I-1}) / 2 for v > 0
                                and the mirror image for v < 0 */
};

typedef struct lbm_ctx lbm_ctx;

/* Validate `p` and create a context. Allocates on the current device: one
 * 19-plane ping-pong state (used by lbm_step when nsteps > 1), per-tile
 * diagnostic partials and the fixed-side equilibria. Synchronous.
 * Errors: LBM_EINVAL (null or invalid parameters), LBM_ENOMEM, LBM_EHIP. */
int lbm_create(const lbm_params* p, lbm_ctx** out);

/* Free a context and its device buffers (synchronises the device). NULL is
 * a no-op. */
void lbm_destroy(lbm_ctx* ctx);

/* f = f^eq(rho, ux, uy, T) on every cell: Eq. (28) with the weights of
 * Eqs. (44)-(46). Inputs: four scalar fields; output: one 19-plane field. */
int lbm_init(lbm_ctx* ctx, const double* rho, const double* ux, const double* uy,
             const double* T, double* f_out, lbm_stream stream);

/* Advance nsteps >= 1 forward-Euler steps (Eq. (47)) from f_in; the result
 * lands in f_out and f_in is left unchanged. Each step computes, per cell,
 * the moments of Eq. (10) from f, f^eq, the flux differences of every
 * velocity along x and y (WENO5, or the upwind scheme that p.scheme names:
 * one thread per cell, a plain comparison kernel) and the BGK relaxation.
 * ke_log: NULL, or device double[2*nsteps] receiving for each step n the
 * transverse kinetic energy of the state the step starts from,
 * ke_log[2n] = sum_cells rho u_n^2 / 2 * dx * dy and ke_log[2n+1] =
 * max_cells rho u_n^2 / 2, u_n the velocity component that ke_axis names
 * (the Sec. IV growth diagnostic, u_n normal to the interface). */
int lbm_step(lbm_ctx* ctx, const double* f_in, double* f_out, int32_t nsteps,
             double* ke_log, lbm_stream stream);

/* Moment sums of f per cell, the conserved quantities of Eq. (10): sums =
 * [4][ny][nx] device doubles holding rho = sum_i f_i, j_x = sum_i f_i v_ix,
 * j_y = sum_i f_i v_iy, E = sum_i f_i |v_i|^2 / 2 (= rho T + rho |u|^2 / 2),
 * each summed over i = 0..18 in that order. sums must not overlap f. */
int lbm_sums(lbm_ctx* ctx, const double* f, double* sums, lbm_stream stream);

/* One step as lbm_step(f_in -> f_out, nsteps = 1, no energy log), carrying
 * the moment sums: sums_in is NULL or the sums of f_in as lbm_sums or an
 * earlier lbm_step_sums gave them, and sums_out receives the sums of f_out
 * (layout of lbm_sums). With a carried-sum step variant (mode 1 or 3) the
 * step reads sums_in instead of forming them from f_in and writes sums_out
 * as it writes f_out (lbm_sums of f_out up to rounding; bit for bit for the
 * fast-tile variants, mode 3, which sum in lbm_sums's order); with the
 * others sums_out is lbm_sums of f_out. f_out is lbm_step's result bit for
 * bit when sums_in is lbm_sums(f_in).
 * For a sequence of single steps whose sums feed lbm_adjoint_step_sums.
 * Outputs must not overlap the inputs or each other. */
int lbm_step_sums(lbm_ctx* ctx, const double* f_in, const double* sums_in, double* f_out,
                  double* sums_out, lbm_stream stream);

/* (rho, ux, uy, T) of f per cell, Eq. (10): rho = sum f, rho u = sum f v,
 * rho T = sum f |v - u|^2 / 2. */
int lbm_moments(lbm_ctx* ctx, const double* f, double* rho, double* ux, double* uy,
                double* T, lbm_stream stream);

/* out2[0] = sum_cells rho u_n^2 / 2 * dx * dy, out2[1] = max_cells
 * rho u_n^2 / 2 of f (device double[2]); u_n is u_y, or u_x when
 * ke_axis = 1 (as in every energy log below). */
int lbm_kinetic_y(lbm_ctx* ctx, const double* f, double* out2, lbm_stream stream);

/* lbm_kinetic_y without a context and without allocating, for callers that
 * cannot allocate device memory (code under stream capture, serving loops,
 * harnesses that forbid hipMalloc). Validates p as lbm_create does and
 * computes out2 from f with the same kernels and summation order as
 * lbm_kinetic_y (identical results), keeping their per-block partials in a
 * fixed device array of the library instead of a context buffer: 1 MiB per
 * GPU, held until the process ends, for grids of at most 2^24 cells
 * (nx * ny larger: LBM_EINVAL, nothing launched). Calls no hipMalloc, hipFree
 * or other allocating routine. Every call on one GPU shares that GPU's array:
 * calls that overlap in time on one GPU race and must be ordered by the
 * caller (one stream, or events). f: one 19-plane field; out2: device
 * double[2]. */
int lbm_kinetic_y_noalloc(const lbm_params* p, const double* f, double* out2,
                          lbm_stream stream);

/* Sanity check of a state: per cell, the moments of Eq. (10) must be finite
 * and describe a gas, rho > 0 and T > 0 (the weights F_k(T) of Eqs. (44)-(46)
 * and the equilibrium of Eq. (28) divide by rho and T; an explicit step that
 * has gone unstable shows here first). A cell is non-finite if one of its 19
 * values or its (rho, u, T) is a NaN or an infinity, and non-physical if all
 * are finite but rho <= 0 or T <= 0. f: one 19-plane field. out4: NULL or host
 * int64[4] = (non-finite cells, non-physical cells, index y*nx + x of the
 * first non-finite cell or -1, of the first non-physical cell or -1).
 * Synchronous: waits for the check on `stream`. Returns LBM_ENONFINITE if any
 * cell is non-finite, else LBM_ENONPHYS if any is non-physical, else LBM_OK
 * (LBM_EINVAL, LBM_EHIP as usual); the message names the first such cell. */
int lbm_check_state(lbm_ctx* ctx, const double* f, int64_t* out4, lbm_stream stream);

/* Discrete adjoint of one step (reverse mode of lbm_step with nsteps = 1):
 *   lam_n = (dS/df)^T lam_np1 + w dE_y/df,   S = the step of Eq. (47),
 * evaluated at f = f_n, with E_y = sum_cells rho u_y^2 / 2 * dx * dy (the
 * objective is E_y: ke_axis must be 0; outflow sides and schemes other than
 * WENO5 are not supported: LBM_EUNSUPPORTED). The
 * transpose covers the WENO5 fluxes including their nonlinear weights
 * (Eqs. (48)-(55)), the equilibrium through the moments (Eqs. (10), (28),
 * (44)-(46)), the BGK term and the ghost layers (periodic images, mirrored
 * planes of reflecting walls; fixed-equilibrium ghosts are constants).
 * f_n, lam_np1: 19-plane inputs; lam_n: 19-plane output (must not overlap
 * them). Deterministic: every output value is written once. */
int lbm_adjoint_step(lbm_ctx* ctx, const double* f_n, const double* lam_np1, double w,
                     double* lam_n, lbm_stream stream);

/* lbm_adjoint_step with the moment sums of f_n supplied (sums_n, layout of
 * lbm_sums, not NULL): the variants with a per-cell pass (PS >= 1) take the
 * equilibrium and objective terms from sums_n and lam_np1 without reading
 * f_n a second time. With sums_n = lbm_sums(f_n) the result is
 * lbm_adjoint_step's bit for bit. lam_n must not overlap any input. */
int lbm_adjoint_step_sums(lbm_ctx* ctx, const double* f_n, const double* sums_n,
                          const double* lam_np1, double w, double* lam_n, lbm_stream stream);

/* Reverse-step variants (same role as the step variants). info4 = (R, G, W,
 * PS): tiles of 64 x R cells, the 18 moving velocities split into G groups
 * (one workgroup per tile and group), W the wavefronts-per-SIMD target, and
 * PS = 1 when a per-cell pass first forms the equilibrium/objective terms
 * and the rest plane (then the context's [4][ny][nx] buffer holds them);
 * PS = 2: the same pass, then one workgroup per moving velocity marches
 * along y over 64-column strips in chunks of R rows, each face evaluated
 * once, the tiles next to non-periodic sides as PS = 1 with R = 4.
 * Every variant computes the same result up to rounding. */
int lbm_adjoint_variant_count(void);
int lbm_adjoint_variant_info(int32_t variant, int32_t* info4);
int lbm_set_adjoint_variant(lbm_ctx* ctx, int32_t variant);
int lbm_get_adjoint_variant(lbm_ctx* ctx, int32_t* variant);

/* Autotuner of the reverse step: times lbm_adjoint_step(f_n, lam_np1 ->
 * lam_tmp) for variants[0..nv) (nv = 0: all), one warm-up call then nsteps
 * timed calls with HIP events on `stream`; ms_out: NULL or host
 * double[nv or count] (ms per call). Leaves the fastest selected.
 * Synchronous. */
int lbm_tune_adjoint(lbm_ctx* ctx, const double* f_n, const double* lam_np1, double* lam_tmp,
                     int32_t nsteps, const int32_t* variants, int32_t nv, double* ms_out,
                     lbm_stream stream);

/* Vector-Jacobian product of lbm_init: g_q = sum_i lam0_i d f_i^eq / d q for
 * q = rho, ux, uy, T per cell (Eq. (28) with Eqs. (44)-(46)). Inputs: the four
 * scalar fields lbm_init took and a 19-plane lam0; outputs: four scalar
 * fields that must not overlap the inputs or each other. */
int lbm_init_vjp(lbm_ctx* ctx, const double* rho, const double* ux, const double* uy,
                 const double* T, const double* lam0, double* g_rho, double* g_ux,
                 double* g_uy, double* g_T, lbm_stream stream);

/* Separable projection of a scalar field g (ny x nx): out[m] =
 * sum_{y,x} A[m*nx + x] * B[y] * g[y*nx + x] for m < M, in a fixed summation
 * order (column sums weighted by B, then one dot product per m). Chains the
 * initial-field gradient to parameters whose tangents factor as
 * (x profile) x (y profile). A: M x nx, B: ny, out: M (device). */
int lbm_sep_project(lbm_ctx* ctx, const double* g, const double* A, int32_t M, const double* B,
                    double* out, lbm_stream stream);

/* Step-kernel variants for the autotuner. lbm_step_variant_info fills
 * info6[0..5] = (R, G, W, D, NT, M). Tiles are 64 x R cells; the 18 moving
 * velocities are split into G groups; W is the wavefronts-per-SIMD target
 * that bounds the register budget; D planes are prefetched ahead of the one
 * being computed; NT = 1 stores f^{n+1} with non-temporal stores. M says how
 * a tile obtains its moments (Eq. (10)):
 *   0  every (tile, group) workgroup sums the 19 planes of f^n itself;
 *   1  the sums rho, j, E are carried from each step to the next (a call
 *      first forms them from f_in) and the G groups are the waves of one
 *      workgroup;
 *   2  a state pass per step forms the cell state (dt/tau rho, T, u/T, v/T),
 *      updates the rest particle and the energy partials; every (tile, group)
 *      workgroup then reads the state;
 *   3  as 1 (G = 1), with the tiles whose stencils need no boundary rule
 *      advanced by a fast-tile body that takes all 18 velocities in one
 *      wavefront; a call's first step forms the sums of f_in in those tiles
 *      (in lbm_sums's order) and, for the tiles around them, in a small pass.
 * The context holds two [4][ny][nx] buffers for modes 1, 2 and 3. Every variant
 * evaluates the same formulas; results agree to rounding (the WENO face
 * arithmetic is grouped per strip of R cells and the moment sums per wave),
 * and a given variant is deterministic. lbm_set_step_variant selects the
 * variant that later lbm_step calls of that context launch. */
int lbm_step_variant_count(void);
int lbm_step_variant_info(int32_t variant, int32_t* info6);
int lbm_set_step_variant(lbm_ctx* ctx, int32_t variant);
int lbm_get_step_variant(lbm_ctx* ctx, int32_t* variant);

/* Autotuner. Times the step variants variants[0..nv) (nv = 0: all of them)
 * on this context's grid: 2 warm-up steps, then one call of nsteps >= 1 and
 * one of 2 nsteps steps of lbm_step from f_in into f_tmp (f_in is not
 * modified), each bracketed by HIP events on `stream`; the time per step is
 * the difference of the two over nsteps, so that a call's fixed cost does
 * not count. ms_out: NULL or host double[nv or count] receiving
 * milliseconds per step. Leaves the fastest variant selected. Synchronous
 * (waits for the timed work); on error the previous variant is kept.
 * LBM_EUNSUPPORTED when the context's scheme is not WENO5 (the variants are
 * WENO5 kernels). */
int lbm_tune_step(lbm_ctx* ctx, const double* f_in, double* f_tmp, int32_t nsteps,
                  const int32_t* variants, int32_t nv, double* ms_out, lbm_stream stream);

/* ---- Batches of independent grids -------------------------------------
 *
 * A batch advances n independent grids ("instances") of possibly different
 * sizes, boundary rules, dx, dy, dt, tau and fixed-side states by the same
 * forward step as lbm_step, all instances in each launch: the work items of
 * every instance form one list that one kernel launch covers. Instances must
 * share vk and weno_eps (they share the velocity set and weights).
 *
 * Layout. A batch distribution field holds instance i's 19-plane field
 * ([19][ny_i][nx_i], as above) at element offset f_offset[i]; blocks must not
 * overlap (gaps are allowed and left untouched). The field's extent is
 * max_i (f_offset[i] + 19 nx_i ny_i) elements (lbm_batch_info). A batch
 * scalar field packs the instances back to back in instance order: instance
 * i's plane starts at element sum_{j<i} nx_j ny_j.
 */
typedef struct lbm_batch lbm_batch;

/* Validate the n >= 1 parameter sets and create a batch on the current
 * device. f_offset: host int64[n], or NULL for back-to-back packing in
 * instance order. Allocates one ping-pong field of the batch's extent,
 * per-tile partials, the device descriptor table and the work list, and a
 * private stream used only to capture graphs. Synchronous.
 * Errors: LBM_EINVAL (invalid instance, differing vk or weno_eps,
 * overlapping or negative offsets), LBM_EUNSUPPORTED (an instance with a
 * scheme other than WENO5), LBM_ENOMEM, LBM_EHIP. */
int lbm_batch_create(const lbm_params* inst, int32_t n, const int64_t* f_offset,
                     lbm_batch** out);

/* Free a batch, its captured graphs and device buffers (synchronises the
 * device). NULL is a no-op. */
void lbm_batch_destroy(lbm_batch* b);

/* out4 (host int64[4]) = (n, extent of a batch distribution field in
 * elements, total cells = length of a batch scalar field, work items per
 * launch of the current variant). */
int lbm_batch_info(lbm_batch* b, int64_t* out4);

/* lbm_init for every instance: batch scalar fields in, batch field out. */
int lbm_batch_init(lbm_batch* b, const double* rho, const double* ux, const double* uy,
                   const double* T, double* f_out, lbm_stream stream);

/* lbm_moments for every instance: batch field in, batch scalar fields out. */
int lbm_batch_moments(lbm_batch* b, const double* f, double* rho, double* ux, double* uy,
                      double* T, lbm_stream stream);

/* lbm_step for every instance (Eq. (47)), nsteps >= 1, f_in unchanged, the
 * result in f_out. ke_log: NULL, or device double[n * nsteps * 2] with
 * ke_log[(i*nsteps + s)*2 + 0/1] = (sum_cells rho u_y^2/2 dx dy, max_cells
 * rho u_y^2/2) of instance i in the state step s starts from. Each instance's
 * result is identical to lbm_step's for that instance alone with the same
 * variant. With a graph chunk C set (lbm_batch_set_schedule), steps after the
 * first run as replays of a captured graph of C steps (cached per buffer
 * pair; recaptured when the variant, the schedule or the buffers change). */
int lbm_batch_step(lbm_batch* b, const double* f_in, double* f_out, int32_t nsteps,
                   double* ke_log, lbm_stream stream);

/* Step variant of the batch kernel (same table as lbm_step_variant_info).
 * Setting it rebuilds the device work list (synchronises the device). */
int lbm_batch_set_step_variant(lbm_batch* b, int32_t variant);
int lbm_batch_get_step_variant(lbm_batch* b, int32_t* variant);

/* Launch schedule. slots_per_xcd = 0: one workgroup per work item; s > 0:
 * a persistent grid of 8 s workgroups, each looping over its XCD's band of
 * the work list. graph_chunk = 0: one launch per step; an even C >= 2:
 * graph replays of C steps. out2 = (slots_per_xcd, graph_chunk). */
int lbm_batch_set_schedule(lbm_batch* b, int32_t slots_per_xcd, int32_t graph_chunk);
int lbm_batch_get_schedule(lbm_batch* b, int32_t* out2);

/* Autotuner of a batch: times every (variant, slots_per_xcd) pair of
 * variants[0..nv) x slots[0..ns) (nv = 0: all variants; ns = 0: the current
 * slot count) like lbm_tune_step, without graphs; ms_out: NULL or host
 * double[nv * ns] (row = variant). Leaves the fastest pair selected and the
 * graph chunk unchanged. Synchronous. */
int lbm_batch_tune(lbm_batch* b, const double* f_in, double* f_tmp, int32_t nsteps,
                   const int32_t* variants, int32_t nv, const int32_t* slots, int32_t ns,
                   double* ms_out, lbm_stream stream);

/* Message of the last failed call on this thread ("" if none). */
const char* lbm_last_error(void);

/* Library version string. */
const char* lbm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
