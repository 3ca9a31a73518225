// lbm_stage.h -- staging of one distribution plane of a 64 x R tile, with a
// cross-shaped halo of depth H, from global memory into LDS. Shared by the
// forward and adjoint step kernels of liblbm_hip.
//
// The staged image has R+2H rows of PITCH doubles; tile column lx (-H..63+H)
// sits at lx+H. Every row is one 64-lane load (lane = column 0..63) from a
// wavefront-uniform row base; the 2H halo columns of the R centre rows come
// from one more load in which lane l < 2HR takes row l/(2H) and one of the
// halo columns. A plane costs R+2H+1 loads per lane.
//
// Fast tiles (tile plus halo inside the domain, or halo columns wrapping
// once around a periodic x axis: fast_tile) need nothing else. A tile
// touching the boundary gets a per-lane column map once (source column and
// kind of the row-load lane and of the halo lane) and resolves ghost rows with
// uniform logic: a row outside the domain is a periodic wrap, a mirror row of
// the y-mirrored velocity (reflecting wall), a constant (fixed equilibrium)
// or unused, or (outflow) a row of the per-step ghost array. Constants and
// unused slots are substituted when the staged values are written to LDS, so
// no load result is consumed before it is needed. Outflow ghosts are loaded
// from the ghost arrays, which hold f^eq of the nearest interior cell per
// position along the side.
//
// ZG ("zero ghosts") stages an adjoint field instead: outside the domain it is
// the periodic image on periodic axes and zero elsewhere, since ghost cells
// have no update of their own whose adjoint could be non-zero.
#pragma once

#include "lbm_device.h"

namespace lbmd {

enum { CK_NORM = 0, CK_MIRX = 1, CK_CXLO = 2, CK_CXHI = 3, CK_NONE = 4, CK_OUTLO = 5, CK_OUTHI = 6 };
enum { RM_NORM = 0, RM_MIRY = 1, RM_CONST = 2, RM_NONE = 3, RM_OUT = 4 };

// Boundary description of the grid being staged. gb[s]: the outflow ghost
// array of side s ([19][ny] for x sides, [19][nx] for y sides), or null.
struct GridBC {
    int nx, ny;
    int bc[4];
    const double* gb[4];
};

template <int R, int H, int PITCH>
struct StageG {
    static constexpr int ROWS = R + 2 * H;
    static constexpr int NPRE = ROWS + 1;
    // one pad slot per idle halo lane (lanes 2HR..63), which keeps the
    // staged image within 8 KB per wave for R = 4
    static constexpr int PAD = ROWS * PITCH;
    static constexpr int NPAD = 64 - 2 * H * R > 0 ? 64 - 2 * H * R : 1;
    static constexpr int SLOTS = PAD + NPAD;
    static_assert(2 * H * R <= 64, "the x-halo of the tile must fit one 64-lane load");
    static_assert(PITCH >= 64 + 2 * H, "row pitch too small");
};

struct TileMapG {
    int hrow, hlx;    // halo lane: tile row and column (-H..-1, 64..63+H)
    int mcol, mkind;  // row-load lane: source column and kind (boundary tiles)
    int hcol, hkind;  // halo lane: source column and kind (boundary tiles);
                      // fast tiles: hcol = offset of the halo value from the
                      // start of the tile's first row (periodic image)
};

// Source column of global column gx for a row inside the domain. Ghost
// layers deeper than three cells exist only for adjoint staging and only
// matter on periodic axes (elsewhere the faces that reach them carry no
// adjoint), so they are unused there.
template <bool ZG>
__device__ __forceinline__ void x_source_g(const GridBC& g, int gx, int& col, int& kind)
{
    if (gx >= 0 && gx < g.nx) {
        col = gx;
        kind = CK_NORM;
        return;
    }
    const bool lo = gx < 0;
    const int m = lo ? -1 - gx : gx - g.nx;
    const int bc = lo ? g.bc[XLO] : g.bc[XHI];
    col = 0;
    kind = CK_NONE;
    if (bc == PERIODIC) {
        col = wrap_index(gx, g.nx);
        kind = CK_NORM;
        return;
    }
    if (ZG || m >= HALO) return;
    if (bc == REFLECT) {
        col = lo ? m : g.nx - 1 - m;
        kind = CK_MIRX;
    } else if (bc == OUTFLOW) {
        kind = lo ? CK_OUTLO : CK_OUTHI;
    } else {
        kind = lo ? CK_CXLO : CK_CXHI;
    }
}

// Tile walk of the tile-parallel kernels: the tiles_x x tiles_y tile grid is
// cut into strips of STRIP tile columns (the last one possibly narrower), each
// walked row by row. Work items that follow each other are then vertical
// neighbours within a strip and find the halo rows they share in L2; on a
// wide grid a row-major walk moves on before they are reused (at 2048 cells
// wide and 4-row tiles, one tile row of the reverse step touches ~6.5 MB,
// more than an XCD's 4 MB L2). Grids at most STRIP tiles wide are walked row
// by row. Returns the tile's row-major index ty * tiles_x + tx.
// The fast-tile forward step walks strips of FAST_STRIP tile columns (2048
// cells): on the 2048-wide grid that is a row-by-row walk, which measured
// faster for it than strips of 8 or 16 tile columns.
constexpr int STRIP = 8;
constexpr int FAST_STRIP = 32;

template <int SW = STRIP>
__device__ __forceinline__ int strip_walk(int t, int tiles_x, int tiles_y)
{
    const int s = t / (SW * tiles_y);
    const int w = min(SW, tiles_x - s * SW);
    const int i = t - s * SW * tiles_y;
    const int ty = i / w;
    return ty * tiles_x + s * SW + (i - ty * w);
}

// v mapped once around a periodic axis of n >= the halo depth: the column
// of every halo value a fast tile (fast_tile) stages.
__device__ __forceinline__ int wrap_once(int v, int n)
{
    return v < 0 ? v + n : (v >= n ? v - n : v);
}

// A tile of columns x0 .. x0+TXW-1 and rows y0 .. y0+R-1 stages without
// boundary logic when it lies in the domain and so do the rows of its halo of
// depth H, and its halo columns do too or lie at most one period away around
// a periodic x axis. (Periodic x is the common case of a boundary strip:
// handling it here keeps whole tile columns off the boundary path. Rows are
// not wrapped: a per-row wrap costs scalar registers the kernels need.)
__device__ __forceinline__ bool fast_tile(const GridBC& g, int x0, int y0, int TXW, int R, int H)
{
    const bool xok = x0 + TXW <= g.nx &&
                     (g.bc[XLO] == PERIODIC ? g.nx >= H : (x0 >= H && x0 + TXW + H <= g.nx));
    return xok && y0 >= H && y0 + R + H <= g.ny;
}

// bnd false: a fast tile; the halo lane's column is then its periodic image.
template <int R, int H, bool ZG>
__device__ __forceinline__ TileMapG tile_map_g(const GridBC& g, int x0, int y0, int lane, bool bnd)
{
    TileMapG t;
    const bool hl = lane < 2 * H * R;
    const int r = lane / (2 * H), c = lane - 2 * H * (lane / (2 * H));
    t.hrow = hl ? r : 0;
    t.hlx = hl ? (c < H ? c - H : c + 64 - H) : 0;
    t.mcol = lane;
    t.mkind = CK_NORM;
    t.hcol = 0;
    t.hkind = CK_NONE;
    if (bnd) {
        x_source_g<ZG>(g, x0 + lane, t.mcol, t.mkind);
        if (hl && y0 + r < g.ny) x_source_g<ZG>(g, x0 + t.hlx, t.hcol, t.hkind);
    } else {
        // fast tile: the halo value's offset from the start of row y0
        t.hcol = t.hrow * g.nx + wrap_once(x0 + t.hlx, g.nx);
    }
    return t;
}

// Uniform description of global row gy: mode, source row and side.
struct RowDesc {
    int mode, src, side;
};

template <bool ZG>
__device__ __forceinline__ RowDesc row_desc_g(const GridBC& g, int gy)
{
    RowDesc d{RM_NORM, gy, 0};
    if (gy >= 0 && gy < g.ny) return d;
    const bool lo = gy < 0;
    const int m = lo ? -1 - gy : gy - g.ny;
    const int bc = lo ? g.bc[YLO] : g.bc[YHI];
    d.side = lo ? YLO : YHI;
    d.src = 0;
    if (bc == PERIODIC) {
        d.src = wrap_index(gy, g.ny);
        return d;
    }
    d.mode = RM_NONE;
    if (ZG || m >= HALO) return d;
    if (bc == REFLECT) {
        d.mode = RM_MIRY;
        d.src = lo ? m : g.ny - 1 - m;
    } else if (bc == OUTFLOW) {
        d.mode = RM_OUT;
    } else {
        d.mode = RM_CONST;
    }
    return d;
}

// Issue the loads of plane `i` (base = start of the 19-plane field) into pre.
template <int R, int H, int PITCH, bool BND, bool ZG>
__device__ __forceinline__ void stage_load_g(const double* __restrict__ field, const GridBC& g,
                                             const Consts& k, int i, int x0, int y0, int lane,
                                             const TileMapG& t, int64_t plane,
                                             double (&pre)[StageG<R, H, PITCH>::NPRE])
{
    using S = StageG<R, H, PITCH>;
    if (!BND) {
        // fast tile: rows in the domain, halo columns in it or one period away
        const unsigned ul = (unsigned)lane;
#pragma unroll
        for (int r = 0; r < S::ROWS; ++r) {
            const double* row = field + i * plane + (int64_t)(y0 - H + r) * g.nx + x0;
            pre[r] = row[ul];
        }
        const double* hb = field + i * plane + (int64_t)y0 * g.nx;
        pre[S::ROWS] = hb[(unsigned)t.hcol];
    } else {
        const int64_t pi = i * plane, px = k.mirx[i] * plane, py = k.miry[i] * plane;
        const bool mout = t.mkind == CK_OUTLO || t.mkind == CK_OUTHI;
        const double* xg = t.mkind == CK_OUTLO ? g.gb[XLO] : g.gb[XHI];
#pragma unroll
        for (int r = 0; r < S::ROWS; ++r) {
            const RowDesc d = row_desc_g<ZG>(g, y0 - H + r);
            const double* base = field;
            int64_t off = 0;
            if (d.mode == RM_NORM) {
                if (mout) {
                    base = xg;
                    off = (int64_t)i * g.ny + d.src;
                } else {
                    off = (t.mkind == CK_MIRX ? px : pi) + (int64_t)d.src * g.nx + t.mcol;
                }
            } else if (d.mode == RM_MIRY) {
                off = py + (int64_t)d.src * g.nx + t.mcol;
            } else if (d.mode == RM_OUT && t.mkind == CK_NORM) {
                // (a select, not g.gb[d.side]: a run-time index would put the
                // descriptor in scratch memory)
                base = d.side == YLO ? g.gb[YLO] : g.gb[YHI];
                off = (int64_t)i * g.nx + t.mcol;
            }
            pre[r] = base[off];
        }
        const double* hbase = field;
        int64_t hoff = 0;
        if (t.hkind == CK_OUTLO || t.hkind == CK_OUTHI) {
            hbase = t.hkind == CK_OUTLO ? g.gb[XLO] : g.gb[XHI];
            hoff = (int64_t)i * g.ny + y0 + t.hrow;
        } else if (t.hkind != CK_NONE) {
            hoff = (t.hkind == CK_MIRX ? px : pi) + (int64_t)(y0 + t.hrow) * g.nx + t.hcol;
        }
        pre[S::ROWS] = hbase[hoff];
    }
}

// Fixed-equilibrium ghost values of a context, held in its by-value
// constants. Stateless on purpose: a functor holding a pointer to by-value
// kernel arguments makes the compiler copy them to scratch memory.
struct SideEqConsts {
    __device__ __forceinline__ double operator()(const Consts& k, int side, int i) const
    {
        return k.side_eq[side][i];
    }
};

// Fixed-equilibrium ghost values read from global memory laid out [4][NV].
struct SideEqPtr {
    const double* p;
    __device__ __forceinline__ double operator()(const Consts&, int side, int i) const
    {
        return p[side * NV + i];
    }
};

// Write the staged plane `i` to LDS, substituting constants and unused slots;
// se(k, side, i) gives the fixed-equilibrium ghost value of velocity i on a
// side.
template <int R, int H, int PITCH, bool BND, bool ZG, class SE>
__device__ __forceinline__ void stage_store_g(const GridBC& g, const Consts& k, SE se, int i, int y0,
                                              int lane, const TileMapG& t, double* s_pl,
                                              const double (&pre)[StageG<R, H, PITCH>::NPRE])
{
    using S = StageG<R, H, PITCH>;
    if (!BND) {
#pragma unroll
        for (int r = 0; r < S::ROWS; ++r) s_pl[r * PITCH + lane + H] = pre[r];
    } else {
        const double cxl = se(k, XLO, i), cxh = se(k, XHI, i);
#pragma unroll
        for (int r = 0; r < S::ROWS; ++r) {
            const RowDesc d = row_desc_g<ZG>(g, y0 - H + r);
            double v = pre[r];
            if (d.mode == RM_CONST)
                v = se(k, d.side, i);
            else if (d.mode == RM_NONE)
                v = 0.0;
            else if (d.mode == RM_NORM)
                v = t.mkind == CK_CXLO ? cxl
                    : t.mkind == CK_CXHI ? cxh
                    : t.mkind == CK_NONE ? 0.0
                                         : v;
            s_pl[r * PITCH + lane + H] = v;
        }
    }
    double h = pre[S::ROWS];
    if (BND)
        h = t.hkind == CK_CXLO ? se(k, XLO, i)
            : t.hkind == CK_CXHI ? se(k, XHI, i)
            : t.hkind == CK_NONE ? 0.0
                                 : h;
    const int slot =
        lane < 2 * H * R ? (t.hrow + H) * PITCH + t.hlx + H : S::PAD + (lane - 2 * H * R);
    s_pl[slot] = h;
}

}  // namespace lbmd
