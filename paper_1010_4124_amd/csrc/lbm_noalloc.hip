// lbm_noalloc.hip -- the allocation-free entry point of liblbm_hip.
//
// lbm_kinetic_y_noalloc computes what lbm_kinetic_y computes (the transverse
// kinetic energy sum and maximum, the growth diagnostic of Sec. IV of
// arXiv:1010.4124) with the same two kernels, but takes the grid's
// parameters instead of a context and keeps the kernels' per-block partials
// in a file-scope device array rather than in context buffers. It calls no
// hipMalloc, hipFree or allocating library routine, so callers that cannot
// allocate device memory (code under stream capture, serving loops,
// harnesses that forbid it) can call it.
//
// The array is a host-side stand-in in host code: kernels receive its device
// address, looked up once per device with hipGetSymbolAddress and kept per
// device ordinal. Every call on a device shares that device's array, so
// calls that overlap on one device race (calls on different devices do not).
// Nothing in it needs clearing: the partial kernel writes every entry the
// reduction reads.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>

#include "lbm.h"
#include "lbm_device.h"
#include "lbm_internal.h"

using namespace lbmd;

namespace {

// (sum, max) partials of one 256-cell block each, for up to
// LBM_NOALLOC_MAX_CELLS cells: 2 doubles per block, 1 MiB in all.
constexpr long long kMaxCells = 1ll << 24;
constexpr long long kMaxBlocks = kMaxCells / 256;

__device__ __align__(256) double scratch[2 * kMaxBlocks];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call there), or null with the error recorded.
double* scratch_ptr()
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        char buf[256];
        std::snprintf(buf, sizeof(buf), "lbm_kinetic_y_noalloc: hipGetDevice: %s",
                      hipGetErrorString(e));
        lbmi_set_error(buf);
        return nullptr;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        lbmi_set_error("lbm_kinetic_y_noalloc: device ordinal out of range");
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            char buf[256];
            std::snprintf(buf, sizeof(buf), "lbm_kinetic_y_noalloc: hipGetSymbolAddress: %s",
                          hipGetErrorString(e));
            lbmi_set_error(buf);
            return nullptr;
        }
        g_ptr[dev] = static_cast<double*>(p);
    }
    return g_ptr[dev];
}

}  // namespace

int lbm_kinetic_y_noalloc(const lbm_params* p, const double* f, double* out2,
                          lbm_stream stream)
{
    int rc = lbmi_validate(p);
    if (rc) return rc;
    if (!f || !out2) {
        lbmi_set_error("lbm_kinetic_y_noalloc: null argument");
        return LBM_EINVAL;
    }
    const long long n = (long long)p->nx * p->ny;
    if (n > kMaxCells) {
        char buf[256];
        std::snprintf(buf, sizeof(buf),
                      "lbm_kinetic_y_noalloc: %lld cells exceed the fixed scratch of %lld cells "
                      "(use lbm_kinetic_y with a context)",
                      n, kMaxCells);
        lbmi_set_error(buf);
        return LBM_EINVAL;
    }
    double* part = scratch_ptr();
    if (!part) return LBM_EHIP;
    Consts k;
    lbmi_fill_consts(p, &k);
    hipStream_t st = (hipStream_t)stream;
    int np = 0;
    hipError_t e = launch_kinetic_part(f, k, n, p->ke_axis, part, &np, st);
    if (e == hipSuccess) e = launch_reduce_pairs(part, np, 1, 0, p->dx * p->dy, out2, st);
    if (e != hipSuccess) {
        char buf[256];
        std::snprintf(buf, sizeof(buf), "lbm_kinetic_y_noalloc: %s", hipGetErrorString(e));
        lbmi_set_error(buf);
        return LBM_EHIP;
    }
    return LBM_OK;
}
