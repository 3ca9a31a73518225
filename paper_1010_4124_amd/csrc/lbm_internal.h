// lbm_internal.h -- declarations shared by the host-side translation units of
// liblbm_hip (not part of the public C-ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm.h"
#include "lbm_device.h"

struct lbm_ctx {
    lbm_params p;
    int device = 0;
    int variant = 0;
    int adj_variant = 0;
    int ke_cap = 0;   // partials per row of ke_part
    int ke_rows = 1;  // rows of ke_part: steps whose energy partials one launch reduces
    lbmd::Consts k;                // per-context constants (kernel arguments)
    double* scratch = nullptr;     // 19 planes: ping-pong state of multi-step calls
    double* ke_part = nullptr;     // [ke_rows][ke_cap][2] diagnostic partials
    double* colbuf = nullptr;      // nx doubles: column sums of lbm_sep_project
    double* msum = nullptr;        // 2 x [4][ny][nx]: carried moment sums (ping-pong)
    double* gbuf = nullptr;        // outflow ghosts: [19][ny] per x side, [19][nx] per y side
    double* gb[4] = {nullptr, nullptr, nullptr, nullptr};  // per side into gbuf, or null
    unsigned long long* chk = nullptr;  // 4 counters of lbm_check_state
};

int lbmi_validate(const lbm_params* p);
void lbmi_fill_consts(const lbm_params* p, lbmd::Consts* h);
int lbmi_default_variant(int nx, int ny);
int lbmi_default_variant_cells(int64_t cells);
int lbmi_default_adj_variant(int64_t cells);
void lbmi_set_error(const char* msg);

namespace lbmd {
int step_variant_count();
int step_variant_desc(int v, int info[6]);
int step_ntiles(int variant, int nx, int ny);
hipError_t launch_step(int variant, const double* fin, double* fout, const Consts& k,
                       double* ke_part, int nx, int ny, const int bc[4], double cx, double cy,
                       double ct, int ke_axis, const double* const gb[4], const double* m_in,
                       double* m_out, hipStream_t st, bool own_sums = false);
// own_sums (carried-sum variants): m_in is to receive the moment sums of fin
// (launch_sums' layout) before the step reads them; the fast-tile kernel
// forms them in its tiles and writes only those of the band tiles to m_in
hipError_t launch_step_lo(int scheme, const double* fin, double* fout, const Consts& k,
                          double* ke_part, int* nparts, int nx, int ny, const int bc[4],
                          double cx, double cy, double ct, int ke_axis,
                          const double* const gb[4], hipStream_t st);
hipError_t launch_outflow(const double* f, int nx, int ny, double* const g[4], const Consts& k,
                          hipStream_t st);
hipError_t launch_sums(const double* f, double* m, const Consts& k, int64_t n, hipStream_t st);
hipError_t launch_state(const double* f, double* fout, double* state, int nx, int ny, double ct,
                        int ke_axis, double* part, int* nparts, const Consts& k,
                        double* const gb[4], hipStream_t st);
hipError_t launch_reduce_pairs(const double* part, int n, int rows, int64_t stride, double dxdy,
                               double* out2, hipStream_t st);
hipError_t launch_init(const double* rho, const double* ux, const double* uy, const double* T,
                       double* f, const Consts& k, int64_t n, hipStream_t st);
hipError_t launch_side_eq(double* out, const double s[4][4], const Consts& k, hipStream_t st);
hipError_t launch_moments(const double* f, double* rho, double* ux, double* uy, double* T,
                          const Consts& k, int64_t n, hipStream_t st);
hipError_t launch_check(const double* f, const Consts& k, int64_t n, unsigned long long* cnt,
                        hipStream_t st);
hipError_t launch_kinetic_part(const double* f, const Consts& k, int64_t n, int ke_axis,
                               double* part, int* nparts, hipStream_t st);
int adj_variant_count();
int adj_variant_desc(int v, int info[4]);
// sums: NULL, or the moment sums of f ([4][ny][nx], as launch_sums writes
// them), which the state pass of PS >= 1 variants then reads instead of f
hipError_t launch_adjoint(int variant, const double* f, const double* sums, const double* lam1,
                          double* lam0, double* kst, const Consts& k, int nx, int ny,
                          const int bc[4], double cx, double cy, double ct, double wdxdy,
                          hipStream_t st);
hipError_t launch_init_vjp(const double* rho, const double* ux, const double* uy, const double* T,
                           const double* lam, double* grho, double* gux, double* guy, double* gT,
                           const Consts& k, int64_t n, hipStream_t st);
hipError_t launch_sep_project(const double* g, const double* A, const double* B, int nx, int ny,
                              int M, double* col, double* out, hipStream_t st);
}  // namespace lbmd
