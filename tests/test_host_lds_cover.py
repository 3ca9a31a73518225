"""Host-side model of the forward tile kernels' LDS use: for every tile of
a grid, the slots that the staging of one distribution plane writes
(stage_store_g, lbm_stage.h, with tile_map_g's halo lanes) and the slots the
x pass and the y pass then read (x_pass, y_pass, lbm_step.h; the update's
reads of the x flux differences). Every slot read must have been written by
the same plane's staging, and no two lanes may write one slot. The index
arithmetic is the kernels' own, restated here for the CPU; the check runs
on every grid shape and boundary set of the GPU parity cases and on the tile
heights the variants use (R = 2, 4, 8). It needs no GPU.

This is the check of the hypothesis that a value is read from LDS before it
is written, for the 5 x 3 grid with fixed-equilibrium x sides on which two
spilling builds once gave wrong results (the build now refuses spilling
kernels)."""
import itertools

import pytest

HALO, TX, PITCH, XPITCH = 3, 64, 71, 65
P, F, RF, O = 0, 1, 2, 3


def stage_slots(R):
    """Slots one lane's staging writes: its column in every staged row, and
    its halo value (a halo slot for lanes < 2 H R, else a pad slot)."""
    rows = R + 2 * HALO
    pad = rows * PITCH
    writes = {}
    for lane in range(64):
        ws = [r * PITCH + lane + HALO for r in range(rows)]
        if lane < 2 * HALO * R:
            hrow, c = lane // (2 * HALO), lane % (2 * HALO)
            hlx = c - HALO if c < HALO else c + 64 - HALO
            ws.append((hrow + HALO) * PITCH + hlx + HALO)
        else:
            ws.append(pad + (lane - 2 * HALO * R))
        writes[lane] = ws
    return writes, pad + max(1, 64 - 2 * HALO * R)


def x_pass_reads(R, neg):
    """Slots lane reads in the x pass (strip s = lane / R of row lane % R:
    the R + 5 samples of its R + 1 faces), and the flux-difference slots it
    writes."""
    out = {}
    for lane in range(64):
        r, s = lane % R, lane // R
        b = (r + HALO) * PITCH + s * R
        reads = [b + (R + 5 - k if neg else k) for k in range(R + 5)]
        writes = [r * XPITCH + s * R + m for m in range(R)]
        out[lane] = (reads, writes)
    return out


def y_pass_reads(R, neg):
    """Slots lane reads in the y pass (its column, the R + 5 rows of the
    strip's faces, and the centre value of each cell) and the flux-difference
    slots the update reads."""
    out = {}
    for lane in range(64):
        col = lane + HALO
        reads = [((R + 5 - k) if neg else k) * PITCH + col for k in range(R + 5)]
        reads += [(m + HALO) * PITCH + col for m in range(R)]
        dx = [m * XPITCH + lane for m in range(R)]
        out[lane] = (reads, dx)
    return out


@pytest.mark.parametrize("R", [2, 4, 8])
def test_staging_covers_every_slot_the_passes_read(R):
    writes, nslots = stage_slots(R)
    written = [s for ws in writes.values() for s in ws]
    assert len(written) == len(set(written)), "two lanes write one LDS slot"
    assert max(written) < nslots
    wset = set(written)
    for neg in (False, True):
        xp, yp = x_pass_reads(R, neg), y_pass_reads(R, neg)
        dx_written = set()
        for lane in range(64):
            reads, dxw = xp[lane]
            missing = [q for q in reads if q not in wset]
            assert not missing, (R, neg, "x pass", lane, missing[:4])
            dx_written.update(dxw)
        for lane in range(64):
            reads, dx = yp[lane]
            missing = [q for q in reads if q not in wset]
            assert not missing, (R, neg, "y pass", lane, missing[:4])
            assert all(q in dx_written for q in dx), (R, neg, "dx", lane)
        # the y pass reads only its own column: the next plane's staging,
        # which the kernels issue without a barrier after it, writes those
        # slots from the same lane (same address, kept in order)
        for lane in range(64):
            own = {r * PITCH + lane + HALO for r in range(R + 2 * HALO)}
            assert set(yp[lane][0]) <= own


def x_source(gx, nx, bc_lo, bc_hi):
    """(kind, column) of global column gx for a row in the domain, as
    x_source_g: 'norm' (a cell, or its periodic image), 'mirx', 'const'
    (fixed equilibrium), 'out' (outflow ghost array) or 'none' (unused)."""
    if 0 <= gx < nx:
        return "norm", gx
    lo = gx < 0
    m = -1 - gx if lo else gx - nx
    bc = bc_lo if lo else bc_hi
    if bc == P:
        return "norm", gx % nx
    if m >= HALO:
        return "none", 0
    if bc == RF:
        return "mirx", m if lo else nx - 1 - m
    return ("out" if bc == O else "const"), 0


def row_desc(gy, ny, bc_lo, bc_hi):
    if 0 <= gy < ny:
        return "norm", gy
    lo = gy < 0
    m = -1 - gy if lo else gy - ny
    bc = bc_lo if lo else bc_hi
    if bc == P:
        return "norm", gy % ny
    if m >= HALO:
        return "none", 0
    if bc == RF:
        return "miry", m if lo else ny - 1 - m
    return ("out" if bc == O else "const"), 0


GRIDS = [(67, 45, (P, P, P, P)), (67, 45, (P, P, RF, RF)), (130, 37, (RF, RF, F, F)),
         (70, 41, (F, F, P, P)), (69, 43, (RF, RF, RF, RF)), (9, 7, (RF, RF, RF, RF)),
         (5, 6, (P, P, RF, RF)), (3, 4, (RF, RF, P, P)), (2, 3, (P, P, P, P)),
         (5, 3, (F, F, RF, RF)), (1, 2, (P, P, P, P)), (600, 21, (P, P, RF, RF)),
         (1100, 9, (RF, RF, P, P)), (64, 30, (P, P, P, P)), (40, 17, (O, O, P, P))]


@pytest.mark.parametrize("R", [2, 4, 8])
@pytest.mark.parametrize("nx,ny,bc", GRIDS)
def test_boundary_tiles_stage_only_valid_sources(nx, ny, bc, R):
    """Every staged value of a boundary tile has a source: a cell of the
    domain (its periodic image, or its mirror across a reflecting wall), a
    fixed-equilibrium constant, an outflow ghost array entry, or an explicit
    zero. A value that a face of a cell inside the domain uses is never
    one of the zeros ('none'), so no cell's update reads an unset value."""
    tiles_x, tiles_y = -(-nx // TX), -(-ny // R)
    for ty, tx in itertools.product(range(tiles_y), range(tiles_x)):
        x0, y0 = tx * TX, ty * R
        for lane in range(64):
            gx = x0 + lane
            for r in range(R + 2 * HALO):
                gy = y0 - HALO + r
                rk, _ = row_desc(gy, ny, bc[2], bc[3])
                ck, _ = x_source(gx, nx, bc[0], bc[1])
                # the y faces of cell (gx, y0 + m), m < R, use rows
                # y0 + m - 3 .. y0 + m + 3 of column gx
                used = 0 <= gx < nx and any(0 <= y0 + m < ny and abs(gy - (y0 + m)) <= HALO
                                            for m in range(R))
                if used:
                    assert rk != "none", (nx, ny, bc, R, gx, gy)
                    assert ck == "norm"
                # a column beyond the domain inside the tile (lanes past nx),
                # in a centre row: the x faces of the domain's last cells use it
                xused = (not 0 <= gx < nx and 0 <= gy < ny and y0 <= gy < y0 + R
                         and any(0 <= gx2 < nx and abs(gx - gx2) <= HALO
                                 for gx2 in range(x0, min(x0 + TX, nx))))
                if xused:
                    assert ck != "none", (nx, ny, bc, R, gx, gy)
        # halo lanes: columns -3..-1 and 64..66 of the R centre rows
        for lane in range(2 * HALO * R):
            hrow, c = lane // (2 * HALO), lane % (2 * HALO)
            hlx = c - HALO if c < HALO else c + 64 - HALO
            gx, gy = x0 + hlx, y0 + hrow
            ck, _ = x_source(gx, nx, bc[0], bc[1]) if gy < ny else ("none", 0)
            # the x faces of cell (gx', gy), |gx - gx'| <= 3, gx' in the domain
            used = gy < ny and any(0 <= gx2 < nx and abs(gx - gx2) <= HALO
                                   for gx2 in range(x0, min(x0 + TX, nx)))
            if used and not (0 <= gx < nx):
                assert ck != "none", (nx, ny, bc, R, gx, gy)
