// lbm_batch.hip -- batched forward steps of many independent grids of uneven
// sizes (one D2V19 FDLB step, Eq. (47) of arXiv:1010.4124, per grid per
// launch) and the lbm_batch_* entry points of the C-ABI.
//
// The tiles of all instances form one flat work list, instance-major. A
// launch has 8 * slots workgroups (G wavefronts each, as the step variant
// says); workgroup b runs on XCD b % 8 and walks the band of the list
// that belongs to that XCD with stride `slots`, so each XCD sweeps one
// contiguous range of tiles (neighbouring tiles share halos in that XCD's
// L2). With slots equal to the band length every workgroup takes exactly one
// item; fewer slots give a persistent grid that stays resident and loops.
//
// Per-instance data (shape, boundary rules, dt/dx, dt/dy, dt/tau, fixed-side
// equilibria, offsets) live in a device-resident descriptor table; the
// velocity set, weights and WENO epsilon are shared by all instances and
// travel by value. Multi-step calls can replay a captured HIP graph of a
// fixed number of steps instead of launching each step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "lbm.h"
#include "lbm_device.h"
#include "lbm_fast.h"
#include "lbm_internal.h"
#include "lbm_stage.h"
#include "lbm_step.h"

namespace lbmd {

// Device-resident description of one instance.
struct BatchInst {
    int64_t off;     // element offset of the instance's [19][ny][nx] block
    int64_t moff;    // element offset of its [4][ny][nx] moment sums
    int64_t goff[4]; // element offsets of its outflow ghost arrays, or -1
    int nx, ny;
    int ke_axis;
    int bc[4];
    int tiles_x;
    int ntiles;      // tiles of the current variant
    int ke_off;      // first per-tile (sum, max) partial of the instance
    int kp_off, kp_n;  // partials the energy reduction adds up: per tile, or per
                       // 256-cell block when a state pass forms them
    int blk_off;       // first 256-cell block of the instance in the batch's block list
    double cx, cy, ct, dxdy;
    double side_eq[4 * NV];  // fixed-side equilibria [side][i]
};

struct BatchArgs {
    const double* __restrict__ fin;
    double* __restrict__ fout;
    double* __restrict__ ke_part;          // [sum of ntiles][2] or null
    const double* gbuf;                    // outflow ghost arrays of all instances
    const BatchInst* __restrict__ inst;
    const int2* __restrict__ work;         // item -> (instance, tile x groups or tile)
    const double* __restrict__ m_in;       // carried moment sums (M variants)
    double* __restrict__ m_out;
    int nwork, per_xcd, slots;
    Consts k;
};

template <int R, int G, int W, int DEPTH, bool NT, int MODE>
__global__ __launch_bounds__((64 * Waves<G, MODE>::N)) __attribute__((amdgpu_waves_per_eu(W)))
void k_step_batch(BatchArgs a)
{
    // PH_FAST: fast tiles take the fast-tile body (lbm_fast.h), the others
    // the PH_CARRY body, tile by tile as the single-grid launch divides them
    constexpr int ML = MODE == PH_FAST ? PH_CARRY : MODE;
    constexpr int NL0 = Waves<G, ML>::N * WaveLds<R, ML>::SIZE;
    constexpr int NL = MODE == PH_FAST && FastStage<R>::LDS > NL0 ? FastStage<R>::LDS : NL0;
    __shared__ double lds[NL];

    const int b = blockIdx.x;
    const int lo = (b & 7) * a.per_xcd;
    const int hi = min(lo + a.per_xcd, a.nwork);
    for (int w = lo + (b >> 3); w < hi; w += a.slots) {
        const int2 it = a.work[w];
        const BatchInst& d = a.inst[it.x];
        StepGrid s;
        s.fin = a.fin + d.off;
        s.fout = a.fout + d.off;
        s.nx = d.nx;
        s.ny = d.ny;
        s.bc[0] = d.bc[0];
        s.bc[1] = d.bc[1];
        s.bc[2] = d.bc[2];
        s.bc[3] = d.bc[3];
        s.tiles_x = d.tiles_x;
        s.ke_axis = d.ke_axis;
#pragma unroll
        for (int q = 0; q < 4; ++q) s.gb[q] = d.goff[q] >= 0 ? a.gbuf + d.goff[q] : nullptr;
        s.cx = d.cx;
        s.cy = d.cy;
        s.ct = d.ct;
        constexpr int GW = ML == PH_CARRY ? 1 : G;
        const int tile = it.y / GW, grp = it.y - tile * GW;
        double* ke = a.ke_part ? a.ke_part + 2 * ((int64_t)d.ke_off + tile) : nullptr;
        if constexpr (MODE == PH_FAST) {
            const int ty = tile / s.tiles_x, tx = tile - ty * s.tiles_x;
            if (fast_tile(grid_bc(s), tx * TX, ty * R, TX, R, HALO)) {
                fast_tile_work<R, DEPTH, NT>(s, a.k, tile, ke, lds, a.m_in + d.moff,
                                             a.m_out + d.moff);
                __syncthreads();  // LDS is reused by the next item
                continue;
            }
        }
        step_work<R, G, DEPTH, NT, ML>(s, a.k, SideEqPtr{d.side_eq}, tile, grp, ke, lds,
                                       ML != PH_SUMS ? a.m_in + d.moff : nullptr,
                                       ML == PH_CARRY ? a.m_out + d.moff : nullptr);
        __syncthreads();  // LDS is reused by the next item
    }
}

// Per-instance reduction of the tile partials: block i writes
// out[i * stride + pos + {0, 1}] = (dxdy * sum, max).
// State pass of a batch in one launch: block b is block b - blk_off of the
// instance blk_inst[b] (state_block; its energy partial lands at global
// block b, where the instance's kp_off points for the state-pass variants;
// cells on outflow sides also write the instance's ghost values).
__global__ __launch_bounds__(256) void k_state_batch(const double* __restrict__ fin,
                                                     double* __restrict__ fout,
                                                     double* __restrict__ msum,
                                                     const int* __restrict__ blk_inst,
                                                     const BatchInst* __restrict__ inst,
                                                     double* __restrict__ ke_part, double* gbuf,
                                                     Consts k)
{
    __shared__ double sr[8];
    const BatchInst& d = inst[blk_inst[blockIdx.x]];
    Ghosts gh;
#pragma unroll
    for (int q = 0; q < 4; ++q) gh.g[q] = d.goff[q] >= 0 ? gbuf + d.goff[q] : nullptr;
    gh.nx = d.nx;
    gh.ny = d.ny;
    state_block(fin + d.off, fout + d.off, msum + d.moff, (int64_t)d.nx * d.ny, d.ct, d.ke_axis,
                ke_part ? ke_part + 2 * (int64_t)d.blk_off : nullptr, k,
                (int64_t)blockIdx.x - d.blk_off, sr, gh);
}

// Outflow ghosts of every outflow side of a batch in one launch: entry b of
// oflow is (instance, side + 4 * block along the side).
__global__ __launch_bounds__(256) void k_outflow_batch(const double* __restrict__ fin,
                                                       const int2* __restrict__ oflow,
                                                       const BatchInst* __restrict__ inst,
                                                       double* gbuf, Consts k)
{
    const int2 e = oflow[blockIdx.x];
    const BatchInst& d = inst[e.x];
    const int side = e.y & 3;
    outflow_point(fin + d.off, d.nx, d.ny, gbuf + d.goff[side], side,
                  (e.y >> 2) * 256 + (int)threadIdx.x, k);
}

__global__ __launch_bounds__(256) void k_reduce_batch(const double* __restrict__ part,
                                                      const BatchInst* __restrict__ inst,
                                                      double* __restrict__ out, int64_t stride,
                                                      int64_t pos, int64_t row_stride)
{
    __shared__ double sr[8];
    const BatchInst& d = inst[blockIdx.x];
    const double* p = part + blockIdx.y * row_stride + 2 * (int64_t)d.kp_off;
    double s = 0.0, mx = 0.0;
    for (int j = threadIdx.x; j < d.kp_n; j += 256) {
        s += p[2 * j];
        mx = fmax(mx, p[2 * j + 1]);
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
        double* o = out + blockIdx.x * stride + pos + 2 * blockIdx.y;
        o[0] = (sr[0] + sr[2] + sr[4] + sr[6]) * d.dxdy;
        o[1] = fmax(fmax(sr[1], sr[3]), fmax(sr[5], sr[7]));
    }
}

struct BatchVariant {
    int R, G, M;
    void (*kernel)(BatchArgs);
};
// The batched kernel keeps an instance descriptor live as well and takes the
// variant's own batch wave target WB, chosen so that it does not spill. The
// host side treats the fast-tile variants (M = 3) as carried-moment ones:
// same work items, sums and buffers.
#define LBM_BATCH_VARIANT(R, G, W, D, NT, M, WB) \
    {R, G, (M == PH_FAST ? PH_CARRY : M), k_step_batch<R, G, WB, D, NT, M>},
static const BatchVariant kBatchVariants[] = {LBM_STEP_VARIANTS(LBM_BATCH_VARIANT)};
#undef LBM_BATCH_VARIANT

}  // namespace lbmd

using namespace lbmd;

// ---------------------------------------------------------------------------
// Host object.

struct lbm_batch {
    int n = 0;
    int device = 0;
    int variant = 0;
    int slots = 0;        // workgroups per XCD; 0 = one per work item
    int graph_chunk = 0;  // steps per captured graph; 0 = no graphs
    int64_t f_extent = 0, cells = 0;
    std::vector<lbm_params> p;
    std::vector<int64_t> off, cell_off;
    std::vector<BatchInst> hinst;
    Consts k;
    int nwork = 0, ntiles = 0;
    BatchInst* inst = nullptr;
    int2* work = nullptr;
    int work_cap = 0, ke_cap = 0;
    int ke_rows = 1;  // rows of ke_part: steps of a graph whose energy partials one launch reduces
    double* scratch = nullptr;
    double* ke_part = nullptr;  // [ke_rows][ke_cap][2] energy partials
    double* ke_ring = nullptr;  // [n][graph_chunk][2]
    double* msum = nullptr;     // 2 x (4 * cells): carried moment sums, ping-pong
    double* gbuf = nullptr;     // outflow ghost arrays of the instances that have them
    int64_t gcap = 0;
    int* blk_inst = nullptr;    // instance of each 256-cell block (state pass)
    int2* oflow = nullptr;      // (instance, side + 4 block) of each outflow ghost block
    int nblk = 0, noflow = 0;
    int ring_cap = 0;
    hipStream_t cap = nullptr;  // private stream used only for capture
    struct Graph {
        const double* x;
        const double* y;
        bool ke;
        int variant, slots, chunk;
        hipGraphExec_t exec;
        unsigned long long used;
    };
    std::vector<Graph> graphs;
    unsigned long long tick = 0;
};

namespace {
int bfail(int code, const char* msg)
{
    lbmi_set_error(msg);
    return code;
}
int bhip(hipError_t e, const char* where)
{
    char buf[512];
    std::snprintf(buf, sizeof(buf), "%s: %s", where, hipGetErrorString(e));
    return bfail(LBM_EHIP, buf);
}

// Entry points that use host containers turn an allocation failure into
// LBM_ENOMEM: no C++ exception crosses the C interface.
template <class F>
int guarded(F&& f) noexcept
{
    try {
        return f();
    } catch (const std::bad_alloc&) {
        lbmi_set_error("host allocation failed");
        return LBM_ENOMEM;
    } catch (...) {
        lbmi_set_error("unexpected host exception");
        return LBM_EHIP;
    }
}

void drop_graphs(lbm_batch* b)
{
    for (auto& g : b->graphs) hipGraphExecDestroy(g.exec);
    b->graphs.clear();
}

// Tile counts, descriptor table and work list for the current variant.
int build_tables(lbm_batch* b)
{
    const BatchVariant& V = kBatchVariants[b->variant];
    const int per_tile = V.M == PH_CARRY ? 1 : V.G;  // work items per tile
    int64_t nwork = 0, ntiles = 0, nblk = 0;
    for (int i = 0; i < b->n; ++i) {
        BatchInst& d = b->hinst[i];
        d.tiles_x = (d.nx + TX - 1) / TX;
        d.ntiles = d.tiles_x * ((d.ny + V.R - 1) / V.R);
        d.ke_off = (int)ntiles;
        const int blocks = (int)(((int64_t)d.nx * d.ny + 255) / 256);
        d.kp_off = V.M == PH_STATE ? (int)nblk : d.ke_off;
        d.kp_n = V.M == PH_STATE ? blocks : d.ntiles;
        ntiles += d.ntiles;
        nblk += blocks;
        nwork += (int64_t)d.ntiles * per_tile;
    }
    if (nwork > b->work_cap || ntiles > b->ke_cap || nblk > b->ke_cap)
        return bfail(LBM_EINVAL, "batch work list exceeds its allocation");
    std::vector<int2> w((size_t)nwork);
    size_t q = 0;
    for (int i = 0; i < b->n; ++i)
        for (int t = 0; t < b->hinst[i].ntiles * per_tile; ++t) w[q++] = make_int2(i, t);
    hipError_t e;
    if ((e = hipMemcpy(b->inst, b->hinst.data(), sizeof(BatchInst) * b->n,
                       hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(b->work, w.data(), sizeof(int2) * w.size(), hipMemcpyHostToDevice)) !=
            hipSuccess)
        return bhip(e, "batch tables");
    b->nwork = (int)nwork;
    b->ntiles = (int)ntiles;
    return LBM_OK;
}

// Step s of a call reads moment set s % 2 and writes the other one; its
// energy partials (ke) go to row `row` of ke_part.
hipError_t launch_batch_step(lbm_batch* b, const double* src, double* dst, bool ke, int parity,
                             hipStream_t st, int row = 0)
{
    double* part = b->ke_part + 2 * (int64_t)b->ke_cap * row;
    const BatchVariant& V = kBatchVariants[b->variant];
    // outflow ghosts of the state this step starts from, all instances at
    // once (with a state pass, that pass writes them)
    if (b->noflow > 0 && V.M != PH_STATE) {
        hipLaunchKernelGGL(k_outflow_batch, dim3((unsigned)b->noflow), dim3(256), 0, st, src,
                           b->oflow, b->inst, b->gbuf, b->k);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    BatchArgs a;
    a.gbuf = b->gbuf;
    a.m_in = nullptr;
    a.m_out = nullptr;
    if (V.M == PH_CARRY) {
        a.m_in = b->msum + 4 * b->cells * parity;
        a.m_out = b->msum + 4 * b->cells * (1 - parity);
    } else if (V.M == PH_STATE) {
        // state pass of every instance in one launch: cell state, rest
        // particle, energy partials
        hipLaunchKernelGGL(k_state_batch, dim3((unsigned)b->nblk), dim3(256), 0, st, src, dst,
                           b->msum, b->blk_inst, b->inst, ke ? part : nullptr, b->gbuf, b->k);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        a.m_in = b->msum;
    }
    a.fin = src;
    a.fout = dst;
    a.ke_part = ke && V.M != PH_STATE ? part : nullptr;
    a.inst = b->inst;
    a.work = b->work;
    a.nwork = b->nwork;
    a.per_xcd = (b->nwork + 7) / 8;
    a.slots = b->slots > 0 ? std::min(b->slots, a.per_xcd) : a.per_xcd;
    a.k = b->k;
    hipLaunchKernelGGL(V.kernel, dim3(8 * a.slots), dim3(64 * (V.M == PH_CARRY ? V.G : 1)), 0, st,
                       a);
    return hipGetLastError();
}

// Energy-log entries of `rows` consecutive steps (rows 0..rows-1 of ke_part)
// for every instance: out[i * stride + pos + 2 r].
hipError_t launch_batch_reduce(lbm_batch* b, double* out, int64_t stride, int64_t pos,
                               hipStream_t st, int rows = 1)
{
    hipLaunchKernelGGL(k_reduce_batch, dim3(b->n, rows), dim3(256), 0, st, b->ke_part, b->inst,
                       out, stride, pos, 2 * (int64_t)b->ke_cap);
    return hipGetLastError();
}

bool overlaps(const void* a, size_t na, const void* b, size_t nb)
{
    const char* x = (const char*)a;
    const char* y = (const char*)b;
    return x < y + nb && y < x + na;
}

// Graph of `chunk` steps x -> y -> ... -> x (chunk even), logging into the
// ring when ke is set. Captured on the private stream, cached by its inputs.
int get_graph(lbm_batch* b, const double* x, double* y, bool ke, hipGraphExec_t* out)
{
    for (auto& g : b->graphs)
        if (g.x == x && g.y == y && g.ke == ke && g.variant == b->variant &&
            g.slots == b->slots && g.chunk == b->graph_chunk) {
            g.used = ++b->tick;
            *out = g.exec;
            return LBM_OK;
        }
    if (ke && b->ring_cap < b->graph_chunk) {
        // graphs of a shorter chunk log into the old ring: drop them with it
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return bhip(e, "batch ke ring");
        drop_graphs(b);
        if (b->ke_ring) hipFree(b->ke_ring);
        b->ke_ring = nullptr;
        b->ring_cap = 0;
        e = hipMalloc(&b->ke_ring, sizeof(double) * 2 * (size_t)b->n * b->graph_chunk);
        if (e != hipSuccess) return bhip(e, "batch ke ring");
        b->ring_cap = b->graph_chunk;
    }
    hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return bhip(e, "hipStreamBeginCapture");
    hipError_t le = hipSuccess;
    for (int s = 0; s < b->graph_chunk && le == hipSuccess; ++s) {
        const double* src = (s % 2 == 0) ? x : y;
        double* dst = (s % 2 == 0) ? y : (double*)x;
        // energy partials of up to ke_rows steps, reduced by one node
        const int row = s % b->ke_rows;
        le = launch_batch_step(b, src, dst, ke, (1 + s) % 2, b->cap, row);
        if (le == hipSuccess && ke && (row == b->ke_rows - 1 || s == b->graph_chunk - 1))
            le = launch_batch_reduce(b, b->ke_ring, 2 * b->graph_chunk, 2 * (s - row), b->cap,
                                     row + 1);
    }
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(b->cap, &graph);
    if (le != hipSuccess || e != hipSuccess) {
        if (graph) hipGraphDestroy(graph);
        return bhip(le != hipSuccess ? le : e, "batch graph capture");
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (e != hipSuccess) return bhip(e, "hipGraphInstantiate");
    if (b->graphs.size() >= 4) {
        auto lru = std::min_element(b->graphs.begin(), b->graphs.end(),
                                    [](const lbm_batch::Graph& p, const lbm_batch::Graph& q) {
                                        return p.used < q.used;
                                    });
        hipGraphExecDestroy(lru->exec);
        b->graphs.erase(lru);
    }
    b->graphs.push_back({x, y, ke, b->variant, b->slots, b->graph_chunk, exec, ++b->tick});
    *out = exec;
    return LBM_OK;
}
}  // namespace

extern "C" {

static int batch_create_impl(const lbm_params* inst, int32_t n, const int64_t* f_offset,
                             lbm_batch** out)
{
    if (!out) return bfail(LBM_EINVAL, "out is null");
    *out = nullptr;
    if (!inst || n < 1) return bfail(LBM_EINVAL, "need at least one instance");
    for (int i = 0; i < n; ++i) {
        const int rc = lbmi_validate(&inst[i]);
        if (rc) return rc;
        if (inst[i].scheme != LBM_SCHEME_WENO5)
            return bfail(LBM_EUNSUPPORTED, "the batched step is the WENO5 scheme's");
        if (std::memcmp(inst[i].vk, inst[0].vk, sizeof(inst[0].vk)) != 0 ||
            std::memcmp(&inst[i].weno_eps, &inst[0].weno_eps, sizeof(double)) != 0)
            return bfail(LBM_EINVAL, "instances of a batch must share vk and weno_eps");
    }
    lbm_batch* b = new (std::nothrow) lbm_batch();
    if (!b) return bfail(LBM_ENOMEM, "host allocation failed");
    b->n = n;
    b->p.assign(inst, inst + n);
    b->off.resize(n);
    b->cell_off.resize(n);
    int64_t pos = 0, cells = 0;
    for (int i = 0; i < n; ++i) {
        const int64_t c = (int64_t)inst[i].nx * inst[i].ny;
        b->off[i] = f_offset ? f_offset[i] : pos;
        b->cell_off[i] = cells;
        pos += NV * c;
        cells += c;
    }
    b->cells = cells;
    // offsets: non-negative and non-overlapping blocks
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int x, int y) { return b->off[x] < b->off[y]; });
    int64_t end = 0;
    for (int j = 0; j < n; ++j) {
        const int i = order[j];
        if (b->off[i] < 0 || b->off[i] < end) {
            delete b;
            return bfail(LBM_EINVAL, "instance blocks overlap or have negative offsets");
        }
        end = b->off[i] + NV * (int64_t)inst[i].nx * inst[i].ny;
    }
    b->f_extent = end;
    lbmi_fill_consts(&inst[0], &b->k);
    hipError_t e = hipGetDevice(&b->device);
    if (e != hipSuccess) {
        delete b;
        return bhip(e, "hipGetDevice");
    }
    // capacity for the variant with the most work items and the most tiles
    int64_t wmax = 0, tmax = 0;
    for (int v = 0; v < step_variant_count(); ++v) {
        int64_t w = 0, t = 0;
        for (int i = 0; i < n; ++i) {
            const int64_t nt = (int64_t)((inst[i].nx + TX - 1) / TX) *
                               ((inst[i].ny + kBatchVariants[v].R - 1) / kBatchVariants[v].R);
            t += nt;
            w += nt * (kBatchVariants[v].M == PH_CARRY ? 1 : kBatchVariants[v].G);
        }
        wmax = std::max(wmax, w);
        tmax = std::max(tmax, t);
    }
    int64_t blocks = 0;
    for (int i = 0; i < n; ++i) blocks += ((int64_t)inst[i].nx * inst[i].ny + 255) / 256;
    tmax = std::max(tmax, blocks);
    if (wmax >= (1ll << 31) || tmax >= (1ll << 30)) {
        delete b;
        return bfail(LBM_EINVAL, "batch too large");
    }
    int64_t gtotal = 0;
    for (int i = 0; i < n; ++i)
        for (int q = 0; q < 4; ++q)
            if (inst[i].bc[q] == LBM_BC_OUTFLOW) gtotal += NV * (int64_t)(q < 2 ? inst[i].ny : inst[i].nx);
    b->gcap = gtotal;
    b->work_cap = (int)wmax;
    b->ke_cap = (int)std::max<int64_t>(tmax, 2 * NV);
    // rows of partials for graph steps: up to 32, within 64 MiB
    b->ke_rows = (int)std::max<int64_t>(
        1, std::min<int64_t>(32, (int64_t)(64 << 20) / (16 * (int64_t)b->ke_cap)));
    b->hinst.resize(n);
    if ((e = hipMalloc(&b->scratch, sizeof(double) * (size_t)b->f_extent)) != hipSuccess ||
        (e = hipMalloc(&b->ke_part, sizeof(double) * 2 * (size_t)b->ke_cap * b->ke_rows)) !=
            hipSuccess ||
        (e = hipMalloc(&b->inst, sizeof(BatchInst) * (size_t)n)) != hipSuccess ||
        (e = hipMalloc(&b->work, sizeof(int2) * (size_t)b->work_cap)) != hipSuccess ||
        (e = hipMalloc(&b->msum, sizeof(double) * 8 * (size_t)b->cells)) != hipSuccess ||
        (e = hipMalloc(&b->gbuf, sizeof(double) * (size_t)(b->gcap > 0 ? b->gcap : 1))) !=
            hipSuccess ||
        (e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking)) != hipSuccess) {
        lbm_batch_destroy(b);
        bhip(e, "batch allocation");
        return LBM_ENOMEM;
    }
    int64_t goff = 0;
    for (int i = 0; i < n; ++i) {
        const lbm_params& q = inst[i];
        BatchInst& d = b->hinst[i];
        std::memset(&d, 0, sizeof(d));
        d.off = b->off[i];
        d.moff = 4 * b->cell_off[i];
        d.ke_axis = q.ke_axis;
        d.nx = q.nx;
        d.ny = q.ny;
        for (int s = 0; s < 4; ++s) d.bc[s] = q.bc[s];
        d.cx = q.dt / q.dx;
        d.cy = q.dt / q.dy;
        d.ct = q.dt / q.tau;
        d.dxdy = q.dx * q.dy;
        for (int sd = 0; sd < 4; ++sd) {
            d.goff[sd] = -1;
            if (q.bc[sd] == LBM_BC_OUTFLOW) {
                d.goff[sd] = goff;
                goff += NV * (int64_t)(sd < 2 ? q.ny : q.nx);
            }
        }
        // fixed-side equilibria by the device equilibrium code
        if ((e = launch_side_eq(b->ke_part, q.side_state, b->k, nullptr)) != hipSuccess ||
            (e = hipDeviceSynchronize()) != hipSuccess ||
            (e = hipMemcpy(d.side_eq, b->ke_part, sizeof(d.side_eq), hipMemcpyDeviceToHost)) !=
                hipSuccess) {
            lbm_batch_destroy(b);
            return bhip(e, "batch side equilibria");
        }
    }
    // block and outflow lists of the one-launch state pass and ghost kernel
    std::vector<int> blk;
    std::vector<int2> ofl;
    for (int i = 0; i < n; ++i) {
        BatchInst& d = b->hinst[i];
        d.blk_off = (int)blk.size();
        const int64_t nb = ((int64_t)d.nx * d.ny + 255) / 256;
        blk.insert(blk.end(), (size_t)nb, i);
        for (int sd = 0; sd < 4; ++sd) {
            if (d.goff[sd] < 0) continue;
            const int len = sd < 2 ? d.ny : d.nx;
            for (int q = 0; q < (len + 255) / 256; ++q) ofl.push_back(make_int2(i, sd + 4 * q));
        }
    }
    b->nblk = (int)blk.size();
    b->noflow = (int)ofl.size();
    if ((e = hipMalloc(&b->blk_inst, sizeof(int) * blk.size())) != hipSuccess ||
        (e = hipMemcpy(b->blk_inst, blk.data(), sizeof(int) * blk.size(),
                       hipMemcpyHostToDevice)) != hipSuccess ||
        (b->noflow > 0 &&
         ((e = hipMalloc(&b->oflow, sizeof(int2) * ofl.size())) != hipSuccess ||
          (e = hipMemcpy(b->oflow, ofl.data(), sizeof(int2) * ofl.size(),
                         hipMemcpyHostToDevice)) != hipSuccess))) {
        lbm_batch_destroy(b);
        bhip(e, "batch block lists");
        return LBM_ENOMEM;
    }
    b->variant = lbmi_default_variant_cells(b->cells);
    const int rc = build_tables(b);
    if (rc) {
        lbm_batch_destroy(b);
        return rc;
    }
    *out = b;
    return LBM_OK;
}

void lbm_batch_destroy(lbm_batch* b)
{
    if (!b) return;
    hipDeviceSynchronize();
    drop_graphs(b);
    if (b->cap) hipStreamDestroy(b->cap);
    if (b->scratch) hipFree(b->scratch);
    if (b->ke_part) hipFree(b->ke_part);
    if (b->ke_ring) hipFree(b->ke_ring);
    if (b->inst) hipFree(b->inst);
    if (b->work) hipFree(b->work);
    if (b->msum) hipFree(b->msum);
    if (b->gbuf) hipFree(b->gbuf);
    if (b->blk_inst) hipFree(b->blk_inst);
    if (b->oflow) hipFree(b->oflow);
    delete b;
}

int lbm_batch_info(lbm_batch* b, int64_t* out4)
{
    if (!b || !out4) return bfail(LBM_EINVAL, "null argument");
    out4[0] = b->n;
    out4[1] = b->f_extent;
    out4[2] = b->cells;
    out4[3] = b->nwork;
    return LBM_OK;
}

int lbm_batch_init(lbm_batch* b, const double* rho, const double* ux, const double* uy,
                   const double* T, double* f_out, lbm_stream stream)
{
    if (!b || !rho || !ux || !uy || !T || !f_out) return bfail(LBM_EINVAL, "null argument");
    const size_t fb = sizeof(double) * (size_t)b->f_extent, sb = sizeof(double) * (size_t)b->cells;
    const double* ins[4] = {rho, ux, uy, T};
    for (auto q : ins)
        if (overlaps(q, sb, f_out, fb)) return bfail(LBM_EINVAL, "input overlaps f_out");
    for (int i = 0; i < b->n; ++i) {
        const int64_t c = b->cell_off[i], m = (int64_t)b->p[i].nx * b->p[i].ny;
        hipError_t e = launch_init(rho + c, ux + c, uy + c, T + c, f_out + b->off[i], b->k, m,
                                   (hipStream_t)stream);
        if (e != hipSuccess) return bhip(e, "lbm_batch_init");
    }
    return LBM_OK;
}

int lbm_batch_moments(lbm_batch* b, const double* f, double* rho, double* ux, double* uy,
                      double* T, lbm_stream stream)
{
    if (!b || !f || !rho || !ux || !uy || !T) return bfail(LBM_EINVAL, "null argument");
    const size_t fb = sizeof(double) * (size_t)b->f_extent, sb = sizeof(double) * (size_t)b->cells;
    double* outs[4] = {rho, ux, uy, T};
    for (auto q : outs)
        if (overlaps(q, sb, f, fb)) return bfail(LBM_EINVAL, "output overlaps f");
    for (int i = 0; i < b->n; ++i) {
        const int64_t c = b->cell_off[i], m = (int64_t)b->p[i].nx * b->p[i].ny;
        hipError_t e = launch_moments(f + b->off[i], rho + c, ux + c, uy + c, T + c, b->k, m,
                                      (hipStream_t)stream);
        if (e != hipSuccess) return bhip(e, "lbm_batch_moments");
    }
    return LBM_OK;
}

static int batch_step_impl(lbm_batch* b, const double* f_in, double* f_out, int32_t nsteps,
                           double* ke_log, lbm_stream stream)
{
    if (!b || !f_in || !f_out) return bfail(LBM_EINVAL, "null argument");
    if (nsteps < 1) return bfail(LBM_EINVAL, "nsteps must be >= 1");
    const size_t fb = sizeof(double) * (size_t)b->f_extent;
    const size_t kb = sizeof(double) * 2 * (size_t)b->n * nsteps;
    if (overlaps(f_in, fb, f_out, fb)) return bfail(LBM_EINVAL, "f_in overlaps f_out");
    if (ke_log && (overlaps(ke_log, kb, f_in, fb) || overlaps(ke_log, kb, f_out, fb)))
        return bfail(LBM_EINVAL, "ke_log overlaps a field");
    hipStream_t st = (hipStream_t)stream;
    const bool ke = ke_log != nullptr;
    // step s writes f_out when (nsteps - 1 - s) is even, else the scratch
    auto dst_of = [&](int s) { return ((nsteps - 1 - s) % 2 == 0) ? f_out : b->scratch; };
    if (kBatchVariants[b->variant].M == PH_CARRY) {
        // moment sums of f_in for the first step (set 0)
        for (int i = 0; i < b->n; ++i) {
            hipError_t e = launch_sums(f_in + b->off[i], b->msum + 4 * b->cell_off[i], b->k,
                                       (int64_t)b->p[i].nx * b->p[i].ny, st);
            if (e != hipSuccess) return bhip(e, "lbm_batch_step sums");
        }
    }
    auto eager = [&](int s) -> int {
        const double* src = s == 0 ? f_in : dst_of(s - 1);
        hipError_t e = launch_batch_step(b, src, dst_of(s), ke, s % 2, st);
        if (e == hipSuccess && ke) e = launch_batch_reduce(b, ke_log, 2 * (int64_t)nsteps, 2 * (int64_t)s, st);
        return e == hipSuccess ? LBM_OK : bhip(e, "lbm_batch_step");
    };
    int s = 0;
    int rc = eager(s++);
    if (rc) return rc;
    const int C = b->graph_chunk;
    if (C >= 2) {
        // steps s .. s+C-1 read dst_of(s-1) and end there again (C even)
        const double* x = dst_of(0);
        double* y = x == f_out ? b->scratch : f_out;
        while (nsteps - s >= C) {
            hipGraphExec_t exec;
            rc = get_graph(b, x, y, ke, &exec);
            if (rc) return rc;
            hipError_t e = hipGraphLaunch(exec, st);
            if (e != hipSuccess) return bhip(e, "hipGraphLaunch");
            if (ke) {
                e = hipMemcpy2DAsync(ke_log + 2 * (int64_t)s, sizeof(double) * 2 * (size_t)nsteps,
                                     b->ke_ring, sizeof(double) * 2 * (size_t)C,
                                     sizeof(double) * 2 * (size_t)C, (size_t)b->n,
                                     hipMemcpyDeviceToDevice, st);
                if (e != hipSuccess) return bhip(e, "batch ke copy");
            }
            s += C;
        }
    }
    for (; s < nsteps; ++s)
        if ((rc = eager(s))) return rc;
    return LBM_OK;
}

static int batch_set_variant_impl(lbm_batch* b, int32_t v)
{
    if (!b || v < 0 || v >= step_variant_count()) return bfail(LBM_EINVAL, "bad variant");
    if (v == b->variant) return LBM_OK;
    hipError_t e = hipDeviceSynchronize();  // tables may be in use by queued work
    if (e != hipSuccess) return bhip(e, "lbm_batch_set_step_variant");
    const int old = b->variant;
    b->variant = v;
    const int rc = build_tables(b);
    if (rc) {
        b->variant = old;
        build_tables(b);
    }
    return rc;
}

int lbm_batch_get_step_variant(lbm_batch* b, int32_t* v)
{
    if (!b || !v) return bfail(LBM_EINVAL, "null argument");
    *v = b->variant;
    return LBM_OK;
}

int lbm_batch_set_schedule(lbm_batch* b, int32_t slots_per_xcd, int32_t graph_chunk)
{
    if (!b || slots_per_xcd < 0 || graph_chunk < 0 || graph_chunk == 1 || graph_chunk % 2)
        return bfail(LBM_EINVAL, "slots must be >= 0 and graph_chunk 0 or even");
    b->slots = slots_per_xcd;
    b->graph_chunk = graph_chunk;
    return LBM_OK;
}

int lbm_batch_get_schedule(lbm_batch* b, int32_t* out2)
{
    if (!b || !out2) return bfail(LBM_EINVAL, "null argument");
    out2[0] = b->slots;
    out2[1] = b->graph_chunk;
    return LBM_OK;
}

}  // extern "C"

static int batch_tune_impl(lbm_batch* b, const double* f_in, double* f_tmp, int32_t nsteps,
                           const int32_t* variants, int32_t nv, const int32_t* slots, int32_t ns,
                           double* ms_out, lbm_stream stream)
{
    if (!b || !f_in || !f_tmp || nsteps < 1 || nv < 0 || ns < 0 || (nv > 0 && !variants) ||
        (ns > 0 && !slots))
        return bfail(LBM_EINVAL, "bad argument");
    const int cv = nv > 0 ? nv : step_variant_count();
    const int cs = ns > 0 ? ns : 1;
    for (int j = 0; j < cv; ++j) {
        const int v = nv > 0 ? variants[j] : j;
        if (v < 0 || v >= step_variant_count()) return bfail(LBM_EINVAL, "bad variant");
    }
    for (int q = 0; q < cs; ++q)
        if (ns > 0 && slots[q] < 0) return bfail(LBM_EINVAL, "bad slot count");
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e;
    if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
        if (e0) hipEventDestroy(e0);
        return bhip(e, "lbm_batch_tune");
    }
    const int keep_v = b->variant, keep_s = b->slots, keep_c = b->graph_chunk;
    int best_v = keep_v, best_s = keep_s, rc = LBM_OK;
    double best_ms = 0.0;
    b->graph_chunk = 0;
    // milliseconds of one call of n steps
    auto timed = [&](int32_t n, float& ms) -> int {
        if ((e = hipEventRecord(e0, st)) != hipSuccess) return bhip(e, "tune");
        const int r = lbm_batch_step(b, f_in, f_tmp, n, nullptr, stream);
        if (r != LBM_OK) return r;
        if ((e = hipEventRecord(e1, st)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess ||
            (e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess)
            return bhip(e, "tune");
        return LBM_OK;
    };
    const int32_t n2 = nsteps <= INT32_MAX / 2 ? 2 * nsteps : nsteps;
    for (int j = 0; j < cv && rc == LBM_OK; ++j) {
        if ((rc = lbm_batch_set_step_variant(b, nv > 0 ? variants[j] : j)) != LBM_OK) break;
        for (int q = 0; q < cs && rc == LBM_OK; ++q) {
            b->slots = ns > 0 ? slots[q] : keep_s;
            float t1 = 0.f, t2 = 0.f;
            if ((rc = lbm_batch_step(b, f_in, f_tmp, 2, nullptr, stream)) != LBM_OK) break;
            if ((rc = timed(nsteps, t1)) != LBM_OK || (rc = timed(n2, t2)) != LBM_OK) break;
            // per step from the difference of the two calls: a call's fixed
            // cost (the carried-moment mode's sums pass over f_in) cancels
            const double per = n2 > nsteps && t2 > t1 ? (double)(t2 - t1) / (n2 - nsteps)
                                                      : (double)t2 / n2;
            if (ms_out) ms_out[j * cs + q] = per;
            if ((j == 0 && q == 0) || per < best_ms) {
                best_ms = per;
                best_v = b->variant;
                best_s = b->slots;
            }
        }
    }
    b->graph_chunk = keep_c;
    if (rc == LBM_OK) {
        rc = lbm_batch_set_step_variant(b, best_v);
        b->slots = best_s;
    } else {
        lbm_batch_set_step_variant(b, keep_v);
        b->slots = keep_s;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return rc;
}

// The C entry points of the allocating calls, behind the exception guard.
extern "C" {

int lbm_batch_create(const lbm_params* inst, int32_t n, const int64_t* f_offset, lbm_batch** out)
{
    return guarded([&] { return batch_create_impl(inst, n, f_offset, out); });
}

int lbm_batch_step(lbm_batch* b, const double* f_in, double* f_out, int32_t nsteps,
                   double* ke_log, lbm_stream stream)
{
    return guarded([&] { return batch_step_impl(b, f_in, f_out, nsteps, ke_log, stream); });
}

int lbm_batch_set_step_variant(lbm_batch* b, int32_t v)
{
    return guarded([&] { return batch_set_variant_impl(b, v); });
}

int lbm_batch_tune(lbm_batch* b, const double* f_in, double* f_tmp, int32_t nsteps,
                   const int32_t* variants, int32_t nv, const int32_t* slots, int32_t ns,
                   double* ms_out, lbm_stream stream)
{
    return guarded([&] {
        return batch_tune_impl(b, f_in, f_tmp, nsteps, variants, nv, slots, ns, ms_out, stream);
    });
}

}  // extern "C"
