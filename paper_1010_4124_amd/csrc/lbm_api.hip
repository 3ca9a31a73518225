// lbm_api.hip -- host side of the C-ABI declared in include/lbm.h:
// parameter validation, context ownership, launch sequencing and errors.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>

#include "lbm.h"
#include "lbm_device.h"
#include "lbm_internal.h"

using namespace lbmd;

namespace {
thread_local std::string g_err;

// Stores the message of the calling thread's last failure; never throws (on
// a host allocation failure the previous message stays).
void set_error(const char* msg) noexcept
{
    try {
        g_err = msg;
    } catch (...) {
    }
}

int fail(int code, const char* fmt, const char* a = "", long long b = 0)
{
    char buf[512];
    std::snprintf(buf, sizeof(buf), fmt, a, b);
    set_error(buf);
    return code;
}

int hip_fail(hipError_t e, const char* where)
{
    char buf[512];
    std::snprintf(buf, sizeof(buf), "%s: %s", where, hipGetErrorString(e));
    set_error(buf);
    return LBM_EHIP;
}
}  // namespace

const char* lbm_last_error(void) { return g_err.c_str(); }

void lbmi_set_error(const char* msg) { set_error(msg); }

const char* lbm_version(void) { return "lbm_hip 0.1 gfx950 d2v19-weno5"; }

int lbmi_validate(const lbm_params* p)
{
    if (!p) return fail(LBM_EINVAL, "params is null%s%lld");
    if (p->nx < 1 || p->ny < 1) return fail(LBM_EINVAL, "nx, ny must be >= 1%s%lld");
    if ((long long)p->nx * p->ny * NV >= (1ll << 31) * 8ll)
        return fail(LBM_EINVAL, "grid too large%s%lld");
    if (!(p->dx > 0) || !(p->dy > 0) || !(p->dt > 0) || !(p->tau > 0))
        return fail(LBM_EINVAL, "dx, dy, dt, tau must be > 0%s%lld");
    if (!(p->weno_eps > 0)) return fail(LBM_EINVAL, "weno_eps must be > 0%s%lld");
    for (int k = 0; k < 3; ++k)
        if (!(p->vk[k] > 0)) return fail(LBM_EINVAL, "vk must be > 0%s%lld");
    if (p->vk[0] == p->vk[1] || p->vk[1] == p->vk[2] || p->vk[0] == p->vk[2])
        return fail(LBM_EINVAL, "vk must be distinct%s%lld");
    for (int s = 0; s < 4; ++s) {
        if (p->bc[s] < 0 || p->bc[s] > 3) return fail(LBM_EINVAL, "unknown boundary code%s%lld");
        const int n = s < 2 ? p->nx : p->ny;
        if (p->bc[s] != LBM_BC_PERIODIC && n < HALO)
            return fail(LBM_EINVAL, "a non-periodic axis needs at least 3 cells%s%lld");
        if (p->bc[s] == LBM_BC_FIXED_EQ && (!(p->side_state[s][0] > 0) || !(p->side_state[s][3] > 0)))
            return fail(LBM_EINVAL, "fixed-equilibrium side needs rho > 0 and T > 0%s%lld");
    }
    if (p->ke_axis != 0 && p->ke_axis != 1) return fail(LBM_EINVAL, "ke_axis must be 0 or 1%s%lld");
    if (p->scheme < LBM_SCHEME_WENO5 || p->scheme > LBM_SCHEME_UPWIND2)
        return fail(LBM_EINVAL, "unknown scheme%s%lld");
    if ((p->bc[0] == LBM_BC_PERIODIC) != (p->bc[1] == LBM_BC_PERIODIC) ||
        (p->bc[2] == LBM_BC_PERIODIC) != (p->bc[3] == LBM_BC_PERIODIC))
        return fail(LBM_EINVAL, "periodic must be set on both sides of an axis%s%lld");
    return LBM_OK;
}

// Host image of the per-context constants: velocity components from the
// exact direction tables, |v|^2/2, the coefficients of the weights of
// Eqs. (44)-(46) and the mirror partners.
void lbmi_fill_consts(const lbm_params* p, Consts* h)
{
    std::memset(h, 0, sizeof(*h));
    h->vx[0] = h->vy[0] = h->hv2[0] = 0.0;
    h->mirx[0] = h->miry[0] = 0;
    for (int k = 0; k < 3; ++k)
        for (int d = 0; d < 6; ++d) {
            const int i = 1 + 6 * k + d;
            h->vx[i] = p->vk[k] * dir_cos(d);
            h->vy[i] = p->vk[k] * (dir_sin_sign(d) * SIN60);
            h->hv2[i] = 0.5 * (p->vk[k] * p->vk[k]);
            h->mirx[i] = 1 + 6 * k + mirror_x_dir(d);
            h->miry[i] = 1 + 6 * k + mirror_y_dir(d);
        }
    for (int k = 0; k < 3; ++k) {
        const double a = p->vk[k] * p->vk[k];
        const double b = p->vk[(k + 1) % 3] * p->vk[(k + 1) % 3];
        const double c = p->vk[(k + 2) % 3] * p->vk[(k + 2) % 3];
        const double den = 3.0 * a * (a - b) * (a - c);
        h->Fc4[k] = 4.0 * (b + c);
        h->Fbc[k] = b * c;
        h->Fden[k] = den;
        h->Frden[k] = 1.0 / den;
    }
    h->eps = p->weno_eps;
    for (int i = 0; i < NV; ++i) {
        h->epsx[i] = h->vx[i] != 0.0 ? p->weno_eps / (h->vx[i] * h->vx[i]) : 0.0;
        h->epsy[i] = h->vy[i] != 0.0 ? p->weno_eps / (h->vy[i] * h->vy[i]) : 0.0;
    }
}

int lbm_create(const lbm_params* p, lbm_ctx** out)
{
    if (!out) return fail(LBM_EINVAL, "out is null%s%lld");
    *out = nullptr;
    int rc = lbmi_validate(p);
    if (rc) return rc;
    lbm_ctx* c = new (std::nothrow) lbm_ctx();
    if (!c) return fail(LBM_ENOMEM, "host allocation failed%s%lld");
    c->p = *p;
    hipError_t e = hipGetDevice(&c->device);
    if (e != hipSuccess) {
        delete c;
        return hip_fail(e, "hipGetDevice");
    }
    lbmi_fill_consts(p, &c->k);
    const size_t n = (size_t)p->nx * p->ny;
    c->variant = lbmi_default_variant(p->nx, p->ny);
    c->adj_variant = lbmi_default_adj_variant((int64_t)p->nx * p->ny);
    int maxtiles = 0;
    for (int v = 0; v < step_variant_count(); ++v) {
        const int t = step_ntiles(v, p->nx, p->ny);
        if (t > maxtiles) maxtiles = t;
    }
    c->ke_cap = maxtiles > (int)((n + 255) / 256) ? maxtiles : (int)((n + 255) / 256);
    // the same buffer first receives the 4 x 19 fixed-side equilibria
    if (2 * c->ke_cap < 4 * NV) c->ke_cap = 2 * NV;
    // energy partials of up to KE_ROWS steps, reduced by one launch (fewer
    // rows where that would take more than 64 MiB)
    constexpr int KE_ROWS = 32;
    const size_t row_bytes = 2 * (size_t)c->ke_cap * sizeof(double);
    c->ke_rows = (int)std::max<size_t>(1, std::min<size_t>(KE_ROWS, (64u << 20) / row_bytes));
    if ((e = hipMalloc(&c->scratch, NV * n * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&c->ke_part, row_bytes * c->ke_rows)) != hipSuccess ||
        (e = hipMalloc(&c->colbuf, (size_t)p->nx * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&c->msum, 8 * n * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&c->gbuf, NV * 2 * ((size_t)p->nx + p->ny) * sizeof(double))) !=
            hipSuccess ||
        (e = hipMalloc(&c->chk, 4 * sizeof(unsigned long long))) != hipSuccess) {
        lbm_destroy(c);
        hip_fail(e, "hipMalloc");
        return LBM_ENOMEM;
    }
    {
        size_t o = 0;
        for (int sd = 0; sd < 4; ++sd) {
            const size_t len = sd < 2 ? (size_t)p->ny : (size_t)p->nx;
            c->gb[sd] = p->bc[sd] == LBM_BC_OUTFLOW ? c->gbuf + o : nullptr;
            o += NV * len;
        }
    }
    // f^eq of the fixed sides, evaluated on the device by the same
    // equilibrium code as every other cell, then kept in the constants
    if ((e = launch_side_eq(c->ke_part, p->side_state, c->k, nullptr)) != hipSuccess ||
        (e = hipDeviceSynchronize()) != hipSuccess ||
        (e = hipMemcpy(&c->k.side_eq[0][0], c->ke_part, sizeof(c->k.side_eq),
                       hipMemcpyDeviceToHost)) != hipSuccess) {
        lbm_destroy(c);
        return hip_fail(e, "side equilibria");
    }
    *out = c;
    return LBM_OK;
}

void lbm_destroy(lbm_ctx* c)
{
    if (!c) return;
    hipDeviceSynchronize();
    if (c->scratch) hipFree(c->scratch);
    if (c->ke_part) hipFree(c->ke_part);
    if (c->colbuf) hipFree(c->colbuf);
    if (c->msum) hipFree(c->msum);
    if (c->gbuf) hipFree(c->gbuf);
    if (c->chk) hipFree(c->chk);
    delete c;
}

static bool overlaps(const void* a, size_t na, const void* b, size_t nb)
{
    const char* x = (const char*)a;
    const char* y = (const char*)b;
    return x < y + nb && y < x + na;
}

int lbm_init(lbm_ctx* c, const double* rho, const double* ux, const double* uy, const double* T,
             double* f_out, lbm_stream stream)
{
    if (!c || !rho || !ux || !uy || !T || !f_out) return fail(LBM_EINVAL, "null argument%s%lld");
    const int64_t n = (int64_t)c->p.nx * c->p.ny;
    const size_t fb = NV * n * sizeof(double), sb = n * sizeof(double);
    const double* ins[4] = {rho, ux, uy, T};
    for (auto q : ins)
        if (overlaps(q, sb, f_out, fb)) return fail(LBM_EINVAL, "input overlaps f_out%s%lld");
    hipError_t e = launch_init(rho, ux, uy, T, f_out, c->k, n, (hipStream_t)stream);
    return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_init");
}

// Row of the energy partials that step s of a call writes.
static double* ke_row(lbm_ctx* c, int s)
{
    return c->ke_part + 2 * (int64_t)c->ke_cap * (s % c->ke_rows);
}

// After step s of nsteps: when s fills the last row or is the last step,
// reduce the rows written since the previous reduction into their ke_log
// entries, one workgroup per row (each row as a single step's would be).
static hipError_t reduce_ke_rows(lbm_ctx* c, int s, int nsteps, int nparts, double* ke_log,
                                 hipStream_t st)
{
    if ((s + 1) % c->ke_rows != 0 && s != nsteps - 1) return hipSuccess;
    const int rows = s % c->ke_rows + 1;
    return launch_reduce_pairs(c->ke_part, nparts, rows, 2 * (int64_t)c->ke_cap,
                               c->p.dx * c->p.dy, ke_log + 2 * (s + 1 - rows), st);
}

int lbm_step(lbm_ctx* c, const double* f_in, double* f_out, int32_t nsteps, double* ke_log,
             lbm_stream stream)
{
    if (!c || !f_in || !f_out) return fail(LBM_EINVAL, "null argument%s%lld");
    if (nsteps < 1) return fail(LBM_EINVAL, "nsteps must be >= 1%s%lld");
    const int64_t n = (int64_t)c->p.nx * c->p.ny;
    const size_t fb = NV * n * sizeof(double);
    if (overlaps(f_in, fb, f_out, fb)) return fail(LBM_EINVAL, "f_in overlaps f_out%s%lld");
    if (ke_log && (overlaps(ke_log, 16 * (size_t)nsteps, f_out, fb) ||
                   overlaps(ke_log, 16 * (size_t)nsteps, f_in, fb)))
        return fail(LBM_EINVAL, "ke_log overlaps a field%s%lld");
    hipStream_t st = (hipStream_t)stream;
    const lbm_params& p = c->p;
    const double cx = p.dt / p.dx, cy = p.dt / p.dy, ct = p.dt / p.tau;
    if (p.scheme != LBM_SCHEME_WENO5) {
        // comparison schemes: one cell-parallel kernel per step
        for (int s = 0; s < nsteps; ++s) {
            const double* src = s == 0 ? f_in : (((nsteps - s) % 2 == 0) ? f_out : c->scratch);
            double* dst = ((nsteps - 1 - s) % 2 == 0) ? f_out : c->scratch;
            hipError_t e = hipSuccess;
            if (c->gb[0] || c->gb[1] || c->gb[2] || c->gb[3])
                e = launch_outflow(src, p.nx, p.ny, c->gb, c->k, st);
            if (e != hipSuccess) return hip_fail(e, "lbm_step outflow");
            int nparts = 0;
            e = launch_step_lo(p.scheme, src, dst, c->k, ke_log ? ke_row(c, s) : nullptr, &nparts,
                               p.nx, p.ny, p.bc, cx, cy, ct, p.ke_axis, c->gb, st);
            if (e != hipSuccess) return hip_fail(e, "lbm_step");
            if (ke_log && (e = reduce_ke_rows(c, s, nsteps, nparts, ke_log, st)) != hipSuccess)
                return hip_fail(e, "lbm_step ke");
        }
        return LBM_OK;
    }
    const int ntiles = step_ntiles(c->variant, p.nx, p.ny);
    int info[6];
    step_variant_desc(c->variant, info);
    const int mode = info[5];
    const bool carry = mode == 1 || mode == 3;  // carried moment sums
    // carried sums: the first step forms those of f_in (the fast-tile kernel
    // in its tiles, the others by a sums pass first); each step then reads
    // one set and writes the other
    for (int s = 0; s < nsteps; ++s) {
        // step s writes f_out when (nsteps - 1 - s) is even, else the scratch
        const double* src = s == 0 ? f_in : (((nsteps - s) % 2 == 0) ? f_out : c->scratch);
        double* dst = ((nsteps - 1 - s) % 2 == 0) ? f_out : c->scratch;
        const double* m_in = nullptr;
        double* m_out = nullptr;
        int nparts = ntiles;
        if ((c->gb[0] || c->gb[1] || c->gb[2] || c->gb[3]) && mode != 2) {
            // outflow ghosts of the state this step starts from (the state
            // pass writes them itself)
            hipError_t e = launch_outflow(src, p.nx, p.ny, c->gb, c->k, st);
            if (e != hipSuccess) return hip_fail(e, "lbm_step outflow");
        }
        if (carry) {
            m_in = c->msum + 4 * n * (s % 2);
            m_out = c->msum + 4 * n * ((s + 1) % 2);
        } else if (mode == 2) {
            // state pass: cell state, rest particle and energy partials
            hipError_t e = launch_state(src, dst, c->msum, p.nx, p.ny, ct, p.ke_axis,
                                        ke_log ? ke_row(c, s) : nullptr, &nparts, c->k, c->gb, st);
            if (e != hipSuccess) return hip_fail(e, "lbm_step state");
            m_in = c->msum;
        }
        hipError_t e = launch_step(c->variant, src, dst, c->k,
                                   ke_log && mode != 2 ? ke_row(c, s) : nullptr, p.nx, p.ny, p.bc,
                                   cx, cy, ct, p.ke_axis, c->gb, m_in, m_out, st,
                                   carry && s == 0);
        if (e != hipSuccess) return hip_fail(e, "lbm_step");
        if (ke_log && (e = reduce_ke_rows(c, s, nsteps, nparts, ke_log, st)) != hipSuccess)
            return hip_fail(e, "lbm_step ke");
    }
    return LBM_OK;
}

int lbm_sums(lbm_ctx* c, const double* f, double* sums, lbm_stream stream)
{
    if (!c || !f || !sums) return fail(LBM_EINVAL, "null argument%s%lld");
    const int64_t n = (int64_t)c->p.nx * c->p.ny;
    if (overlaps(sums, 4 * n * sizeof(double), f, NV * n * sizeof(double)))
        return fail(LBM_EINVAL, "sums overlaps f%s%lld");
    hipError_t e = launch_sums(f, sums, c->k, n, (hipStream_t)stream);
    return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_sums");
}

int lbm_step_sums(lbm_ctx* c, const double* f_in, const double* sums_in, double* f_out,
                  double* sums_out, lbm_stream stream)
{
    if (!c || !f_in || !f_out || !sums_out) return fail(LBM_EINVAL, "null argument%s%lld");
    const int64_t n = (int64_t)c->p.nx * c->p.ny;
    const size_t fb = NV * n * sizeof(double), sb = 4 * n * sizeof(double);
    if (overlaps(f_in, fb, f_out, fb) || overlaps(sums_out, sb, f_in, fb) ||
        overlaps(sums_out, sb, f_out, fb) || (sums_in && (overlaps(sums_in, sb, sums_out, sb) ||
                                                          overlaps(sums_in, sb, f_out, fb))))
        return fail(LBM_EINVAL, "an output overlaps an input or another output%s%lld");
    hipStream_t st = (hipStream_t)stream;
    const lbm_params& p = c->p;
    int info[6];
    step_variant_desc(c->variant, info);
    const bool carry = p.scheme == LBM_SCHEME_WENO5 && (info[5] == 1 || info[5] == 3);
    if (!carry) {
        // the step as lbm_step takes it, then the sums of its result
        const int rc = lbm_step(c, f_in, f_out, 1, nullptr, stream);
        if (rc != LBM_OK) return rc;
        hipError_t e = launch_sums(f_out, sums_out, c->k, n, st);
        return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_step_sums");
    }
    hipError_t e = hipSuccess;
    // without the sums of f_in the step forms them itself (into c->msum)
    const bool own = !sums_in;
    if (own) sums_in = c->msum;
    if (c->gb[0] || c->gb[1] || c->gb[2] || c->gb[3]) {
        e = launch_outflow(f_in, p.nx, p.ny, c->gb, c->k, st);
        if (e != hipSuccess) return hip_fail(e, "lbm_step_sums outflow");
    }
    e = launch_step(c->variant, f_in, f_out, c->k, nullptr, p.nx, p.ny, p.bc, p.dt / p.dx,
                    p.dt / p.dy, p.dt / p.tau, p.ke_axis, c->gb, sums_in, sums_out, st, own);
    return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_step_sums");
}

int lbm_moments(lbm_ctx* c, const double* f, double* rho, double* ux, double* uy, double* T,
                lbm_stream stream)
{
    if (!c || !f || !rho || !ux || !uy || !T) return fail(LBM_EINVAL, "null argument%s%lld");
    const int64_t n = (int64_t)c->p.nx * c->p.ny;
    const size_t fb = NV * n * sizeof(double), sb = n * sizeof(double);
    double* outs[4] = {rho, ux, uy, T};
    for (auto q : outs)
        if (overlaps(q, sb, f, fb)) return fail(LBM_EINVAL, "output overlaps f%s%lld");
    hipError_t e = launch_moments(f, rho, ux, uy, T, c->k, n, (hipStream_t)stream);
    return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_moments");
}

int lbm_kinetic_y(lbm_ctx* c, const double* f, double* out2, lbm_stream stream)
{
    if (!c || !f || !out2) return fail(LBM_EINVAL, "null argument%s%lld");
    const int64_t n = (int64_t)c->p.nx * c->p.ny;
    int np = 0;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = launch_kinetic_part(f, c->k, n, c->p.ke_axis, c->ke_part, &np, st);
    if (e == hipSuccess) e = launch_reduce_pairs(c->ke_part, np, 1, 0, c->p.dx * c->p.dy, out2, st);
    return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_kinetic_y");
}

int lbm_check_state(lbm_ctx* c, const double* f, int64_t* out4, lbm_stream stream)
{
    if (!c || !f) return fail(LBM_EINVAL, "null argument%s%lld");
    const int64_t n = (int64_t)c->p.nx * c->p.ny;
    hipStream_t st = (hipStream_t)stream;
    unsigned long long h[4];
    hipError_t e = launch_check(f, c->k, n, c->chk, st);
    if (e == hipSuccess) e = hipMemcpyAsync(h, c->chk, sizeof(h), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "lbm_check_state");
    const int64_t r[4] = {(int64_t)h[0], (int64_t)h[1], h[2] == ~0ull ? -1 : (int64_t)h[2],
                          h[3] == ~0ull ? -1 : (int64_t)h[3]};
    if (out4)
        for (int j = 0; j < 4; ++j) out4[j] = r[j];
    const int nx = c->p.nx;
    char buf[256];
    if (r[0] > 0) {
        std::snprintf(buf, sizeof(buf), "non-finite state: %lld cells, first at x=%lld y=%lld",
                      (long long)r[0], (long long)(r[2] % nx), (long long)(r[2] / nx));
        set_error(buf);
        return LBM_ENONFINITE;
    }
    if (r[1] > 0) {
        std::snprintf(buf, sizeof(buf),
                      "non-physical state (rho <= 0 or T <= 0): %lld cells, first at x=%lld y=%lld",
                      (long long)r[1], (long long)(r[3] % nx), (long long)(r[3] / nx));
        set_error(buf);
        return LBM_ENONPHYS;
    }
    return LBM_OK;
}

int lbm_step_variant_count(void) { return step_variant_count(); }

int lbm_step_variant_info(int32_t v, int32_t* info6)
{
    int d[6];
    if (!info6 || step_variant_desc(v, d)) return fail(LBM_EINVAL, "bad variant%s%lld");
    for (int j = 0; j < 6; ++j) info6[j] = d[j];
    return LBM_OK;
}

int lbm_set_step_variant(lbm_ctx* c, int32_t v)
{
    if (!c || v < 0 || v >= step_variant_count()) return fail(LBM_EINVAL, "bad variant%s%lld");
    c->variant = v;
    return LBM_OK;
}

int lbm_get_step_variant(lbm_ctx* c, int32_t* v)
{
    if (!c || !v) return fail(LBM_EINVAL, "null argument%s%lld");
    *v = c->variant;
    return LBM_OK;
}

// Default step variant (the autotuner can override it per context or batch),
// the fastest measured on MI355X: on small grids a state pass and one
// velocity per workgroup; on large grids (or batches) carried moment sums
// with the fast-tile kernel and non-temporal stores.
int lbmi_default_variant(int nx, int ny) { return lbmi_default_variant_cells((int64_t)nx * ny); }

int lbmi_default_variant_cells(int64_t cells)
{
    const bool large = cells >= (1ll << 21);
    const int small_v[6] = {4, 18, 4, 1, 0, 2}, large_v[6] = {4, 1, 2, 1, 1, 3};
    const int* want = large ? large_v : small_v;
    for (int v = 0; v < step_variant_count(); ++v) {
        int d[6];
        step_variant_desc(v, d);
        bool same = true;
        for (int j = 0; j < 6; ++j) same = same && d[j] == want[j];
        if (same) return v;
    }
    return 0;
}

static int adjoint_step(lbm_ctx* c, const double* f_n, const double* sums_n,
                        const double* lam_np1, double w, double* lam_n, lbm_stream stream)
{
    if (!c || !f_n || !lam_np1 || !lam_n) return fail(LBM_EINVAL, "null argument%s%lld");
    const lbm_params& p = c->p;
    for (int sd = 0; sd < 4; ++sd)
        if (p.bc[sd] == LBM_BC_OUTFLOW)
            return fail(LBM_EUNSUPPORTED, "the reverse step has no outflow sides%s%lld");
    if (p.ke_axis != 0)
        return fail(LBM_EUNSUPPORTED, "the reverse step's objective is E_y (ke_axis 0)%s%lld");
    if (p.scheme != LBM_SCHEME_WENO5)
        return fail(LBM_EUNSUPPORTED, "the reverse step is the WENO5 scheme's%s%lld");
    const size_t fb = NV * (size_t)p.nx * p.ny * sizeof(double);
    const size_t sb = 4 * (size_t)p.nx * p.ny * sizeof(double);
    if (overlaps(lam_n, fb, lam_np1, fb) || overlaps(lam_n, fb, f_n, fb) ||
        (sums_n && overlaps(lam_n, fb, sums_n, sb)))
        return fail(LBM_EINVAL, "lam_n overlaps an input%s%lld");
    hipError_t e = launch_adjoint(c->adj_variant, f_n, sums_n, lam_np1, lam_n, c->msum, c->k, p.nx,
                                  p.ny, p.bc, p.dt / p.dx, p.dt / p.dy, p.dt / p.tau,
                                  w * p.dx * p.dy, (hipStream_t)stream);
    return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_adjoint_step");
}

int lbm_adjoint_step(lbm_ctx* c, const double* f_n, const double* lam_np1, double w, double* lam_n,
                     lbm_stream stream)
{
    return adjoint_step(c, f_n, nullptr, lam_np1, w, lam_n, stream);
}

int lbm_adjoint_step_sums(lbm_ctx* c, const double* f_n, const double* sums_n,
                          const double* lam_np1, double w, double* lam_n, lbm_stream stream)
{
    if (!sums_n) return fail(LBM_EINVAL, "null argument%s%lld");
    return adjoint_step(c, f_n, sums_n, lam_np1, w, lam_n, stream);
}

int lbm_init_vjp(lbm_ctx* c, const double* rho, const double* ux, const double* uy, const double* T,
                 const double* lam0, double* g_rho, double* g_ux, double* g_uy, double* g_T,
                 lbm_stream stream)
{
    if (!c || !rho || !ux || !uy || !T || !lam0 || !g_rho || !g_ux || !g_uy || !g_T)
        return fail(LBM_EINVAL, "null argument%s%lld");
    const int64_t n = (int64_t)c->p.nx * c->p.ny;
    const size_t sb = n * sizeof(double), fb = NV * sb;
    const double* ins[5] = {rho, ux, uy, T, lam0};
    const size_t insz[5] = {sb, sb, sb, sb, fb};
    double* outs[4] = {g_rho, g_ux, g_uy, g_T};
    for (int o = 0; o < 4; ++o) {
        for (int q = 0; q < 5; ++q)
            if (overlaps(outs[o], sb, ins[q], insz[q]))
                return fail(LBM_EINVAL, "an output overlaps an input%s%lld");
        for (int q = o + 1; q < 4; ++q)
            if (overlaps(outs[o], sb, outs[q], sb)) return fail(LBM_EINVAL, "outputs overlap%s%lld");
    }
    hipError_t e = launch_init_vjp(rho, ux, uy, T, lam0, g_rho, g_ux, g_uy, g_T, c->k, n,
                                   (hipStream_t)stream);
    return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_init_vjp");
}

int lbm_sep_project(lbm_ctx* c, const double* g, const double* A, int32_t M, const double* B,
                    double* out, lbm_stream stream)
{
    if (!c || !g || !A || !B || !out || M < 1) return fail(LBM_EINVAL, "bad argument%s%lld");
    const lbm_params& p = c->p;
    hipError_t e = launch_sep_project(g, A, B, p.nx, p.ny, M, c->colbuf, out, (hipStream_t)stream);
    return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_sep_project");
}

// Autotuner: time each listed variant on this grid with HIP events on
// `stream` (warm-up steps first), keep the fastest.
int lbm_tune_step(lbm_ctx* c, const double* f_in, double* f_tmp, int32_t nsteps,
                  const int32_t* variants, int32_t nv, double* ms_out, lbm_stream stream)
{
    if (!c || !f_in || !f_tmp || nsteps < 1 || nv < 0 || (nv > 0 && !variants))
        return fail(LBM_EINVAL, "bad argument%s%lld");
    if (c->p.scheme != LBM_SCHEME_WENO5)
        return fail(LBM_EUNSUPPORTED, "step variants are WENO5 kernels%s%lld");
    const int count = nv > 0 ? nv : step_variant_count();
    for (int j = 0; j < count; ++j) {
        const int v = nv > 0 ? variants[j] : j;
        if (v < 0 || v >= step_variant_count()) return fail(LBM_EINVAL, "bad variant%s%lld");
    }
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e;
    if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
        if (e0) hipEventDestroy(e0);
        return hip_fail(e, "lbm_tune_step");
    }
    const int keep = c->variant;
    int best = keep, rc = LBM_OK;
    double best_ms = 0.0;
    // milliseconds of one call of n steps
    auto timed = [&](int32_t n, float& ms) -> int {
        if ((e = hipEventRecord(e0, st)) != hipSuccess) return hip_fail(e, "tune");
        const int r = lbm_step(c, f_in, f_tmp, n, nullptr, stream);
        if (r != LBM_OK) return r;
        if ((e = hipEventRecord(e1, st)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess ||
            (e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess)
            return hip_fail(e, "tune");
        return LBM_OK;
    };
    const int32_t n2 = nsteps <= INT32_MAX / 2 ? 2 * nsteps : nsteps;
    for (int j = 0; j < count && rc == LBM_OK; ++j) {
        c->variant = nv > 0 ? variants[j] : j;
        float t1 = 0.f, t2 = 0.f;
        if ((rc = lbm_step(c, f_in, f_tmp, 2, nullptr, stream)) != LBM_OK) break;
        if ((rc = timed(nsteps, t1)) != LBM_OK || (rc = timed(n2, t2)) != LBM_OK) break;
        // per step from the difference of the two calls: a call's fixed cost
        // (the carried-moment mode's sums pass over f_in) cancels
        const double per = n2 > nsteps && t2 > t1 ? (double)(t2 - t1) / (n2 - nsteps)
                                                  : (double)t2 / n2;
        if (ms_out) ms_out[j] = per;
        if (j == 0 || per < best_ms) {
            best_ms = per;
            best = c->variant;
        }
    }
    c->variant = rc == LBM_OK ? best : keep;
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return rc;
}

// Default reverse-step variant: one velocity per workgroup after a state
// pass, so that small grids still fill the chip; from 2^20 cells on, the
// marching variant in chunks of 64 rows.
int lbmi_default_adj_variant(int64_t cells)
{
    const int want[4] = {cells >= (1 << 20) ? 64 : 4, 18, 2, cells >= (1 << 20) ? 2 : 1};
    for (int v = 0; v < adj_variant_count(); ++v) {
        int d[4];
        adj_variant_desc(v, d);
        if (d[0] == want[0] && d[1] == want[1] && d[2] == want[2] && d[3] == want[3]) return v;
    }
    return 0;
}

int lbm_adjoint_variant_count(void) { return adj_variant_count(); }

int lbm_adjoint_variant_info(int32_t v, int32_t* info4)
{
    int d[4];
    if (!info4 || adj_variant_desc(v, d)) return fail(LBM_EINVAL, "bad adjoint variant%s%lld");
    for (int j = 0; j < 4; ++j) info4[j] = d[j];
    return LBM_OK;
}

int lbm_set_adjoint_variant(lbm_ctx* c, int32_t v)
{
    if (!c || v < 0 || v >= adj_variant_count())
        return fail(LBM_EINVAL, "bad adjoint variant%s%lld");
    c->adj_variant = v;
    return LBM_OK;
}

int lbm_get_adjoint_variant(lbm_ctx* c, int32_t* v)
{
    if (!c || !v) return fail(LBM_EINVAL, "null argument%s%lld");
    *v = c->adj_variant;
    return LBM_OK;
}

int lbm_tune_adjoint(lbm_ctx* c, const double* f_n, const double* lam_np1, double* lam_tmp,
                     int32_t nsteps, const int32_t* variants, int32_t nv, double* ms_out,
                     lbm_stream stream)
{
    if (!c || !f_n || !lam_np1 || !lam_tmp || nsteps < 1 || nv < 0 || (nv > 0 && !variants))
        return fail(LBM_EINVAL, "bad argument%s%lld");
    const int count = nv > 0 ? nv : adj_variant_count();
    for (int j = 0; j < count; ++j) {
        const int v = nv > 0 ? variants[j] : j;
        if (v < 0 || v >= adj_variant_count()) return fail(LBM_EINVAL, "bad adjoint variant%s%lld");
    }
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e;
    if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
        if (e0) hipEventDestroy(e0);
        return hip_fail(e, "lbm_tune_adjoint");
    }
    const int keep = c->adj_variant;
    int best = keep, rc = LBM_OK;
    double best_ms = 0.0;
    for (int j = 0; j < count && rc == LBM_OK; ++j) {
        c->adj_variant = nv > 0 ? variants[j] : j;
        float ms = 0.f;
        if ((rc = lbm_adjoint_step(c, f_n, lam_np1, 1.0, lam_tmp, stream)) != LBM_OK) break;
        if ((e = hipEventRecord(e0, st)) != hipSuccess) { rc = hip_fail(e, "tune"); break; }
        for (int s = 0; s < nsteps && rc == LBM_OK; ++s)
            rc = lbm_adjoint_step(c, f_n, lam_np1, 1.0, lam_tmp, stream);
        if (rc != LBM_OK) break;
        if ((e = hipEventRecord(e1, st)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess ||
            (e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) {
            rc = hip_fail(e, "tune");
            break;
        }
        const double per = ms / nsteps;
        if (ms_out) ms_out[j] = per;
        if (j == 0 || per < best_ms) {
            best_ms = per;
            best = c->adj_variant;
        }
    }
    c->adj_variant = rc == LBM_OK ? best : keep;
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return rc;
}
