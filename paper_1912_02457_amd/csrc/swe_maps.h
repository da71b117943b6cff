// Index maps of the ghost frames, shared by the device code and the
// host-side bounds check (tests/host_check.cpp): the ghost cells of the
// boundary kinds, the corner depths around them, the frame cells a stage
// writes for the next one, and the nearest nested side of a relaxation-zone
// cell.  Pure integer arithmetic, no memory access.
//
// Ghost cells.  Wall ghosts mirror the state with the normal momentum and f
// negated (eq. tradWallBCx and f(-x) = -f(x) of eq. KxWallBCReq); periodic
// ghosts wrap; nested ghosts take the external state at the stage time and
// the f / north angle stored for them at init.  The mapping is split into a
// column part, fixed for a lane over a whole tile, and a row part, the same
// for every lane of a row.
#pragma once

#include "swe_device.h"

namespace swe {

__host__ __device__ inline int imin(int a, int b) { return a < b ? a : b; }
__host__ __device__ inline int imax(int a, int b) { return a > b ? a : b; }

struct ColMap {
    int ci;       // source column
    int cc0, cc1; // source corner columns of the cell's west and east corners
    float su, sf; // sign of hu and f (wall ghost)
    int nside;    // nested side 0 (W) / 1 (E) for a nested ghost column, else -1
    int nlayer;   // 0 for the ghost next to the domain, 1 for the outer one
};

struct RowMap {
    int cr;       // source row
    int crc;      // source corner row of the cell's north corners
    float sv, sf; // sign of hv and f (wall ghost)
    int nside;    // nested side 2 (S) / 3 (N) for a nested ghost row, else -1
    int nlayer;
};

// corner index c in [-2, n+2] of an axis with n cells
__host__ __device__ inline int map_corner(int c, int n, int lo, int hi)
{
    if (c < 0) return lo == BC_PERIODIC ? c + n : -c;
    if (c > n) return hi == BC_PERIODIC ? c - n : 2 * n - c;
    return c;
}

// i in [-2, nx+1]
__host__ __device__ inline ColMap col_map(const Dom &d, int i)
{
    const int nx = d.nx;
    ColMap m;
    m.ci = i; m.su = 1.f; m.sf = 1.f; m.nside = -1; m.nlayer = 0;
    if (i < 0) {
        if (d.bc[0] == BC_PERIODIC) m.ci = i + nx;
        else { m.ci = -1 - i; if (d.bc[0] == BC_WALL) { m.su = -1.f; m.sf = -1.f; } else { m.nside = 0; m.nlayer = -1 - i; } }
    } else if (i >= nx) {
        if (d.bc[1] == BC_PERIODIC) m.ci = i - nx;
        else { m.ci = 2 * nx - 1 - i; if (d.bc[1] == BC_WALL) { m.su = -1.f; m.sf = -1.f; } else { m.nside = 1; m.nlayer = i - nx; } }
    }
    m.cc0 = map_corner(i, nx, d.bc[0], d.bc[1]);
    m.cc1 = map_corner(i + 1, nx, d.bc[0], d.bc[1]);
    return m;
}

// r in [-2, ny+1]
__host__ __device__ inline RowMap row_map(const Dom &d, int r)
{
    const int ny = d.ny;
    RowMap m;
    m.cr = r; m.sv = 1.f; m.sf = 1.f; m.nside = -1; m.nlayer = 0;
    if (r < 0) {
        if (d.bc[2] == BC_PERIODIC) m.cr = r + ny;
        else { m.cr = -1 - r; if (d.bc[2] == BC_WALL) { m.sv = -1.f; m.sf = -1.f; } else { m.nside = 2; m.nlayer = -1 - r; } }
    } else if (r >= ny) {
        if (d.bc[3] == BC_PERIODIC) m.cr = r - ny;
        else { m.cr = 2 * ny - 1 - r; if (d.bc[3] == BC_WALL) { m.sv = -1.f; m.sf = -1.f; } else { m.nside = 3; m.nlayer = r - ny; } }
    }
    m.crc = map_corner(r + 1, ny, d.bc[2], d.bc[3]);
    return m;
}

// Source of frame cell (il, r) (il in [-2, nx+1], r in [-2, ny+1]): a nested
// ghost takes boundary-table entry idx (side >= 0, layer 0 or 1); any other
// cell copies framed element `off` of its plane, with the sign flips of a
// wall ghost in `flip` (bits 31, 30, 29: hu, hv, f).  cof0 / cof1 are the
// framed corner-plane elements of the source's north-west / north-east
// corners.  A ghost column only ever contributes rows inside [0, ny) to an
// output; its rows outside (diagonal ghosts) get some in-range value that is
// never used.
struct GhostSrc {
    int side, idx, layer;
    uint32_t off, flip, cof0, cof1;
};

__host__ __device__ inline GhostSrc ghost_src(const Dom &d, const ColMap &cm, int il, int r)
{
    const RowMap rm = row_map(d, r);  // the same for all lanes
    const bool yin = r >= 0 && r < d.ny;
    GhostSrc g;
    g.side = -1; g.idx = 0; g.layer = 0; g.off = 0u; g.flip = 0u;
    if (yin && cm.nside >= 0) {
        g.side = cm.nside; g.layer = cm.nlayer; g.idx = cm.nside == 0 ? r : d.ny + r;
    } else if (!yin && rm.nside >= 0) {
        const int ii = imin(imax(il, 0), d.nx - 1);
        g.side = rm.nside; g.layer = rm.nlayer; g.idx = rm.nside == 2 ? 2 * d.ny + ii : 2 * d.ny + d.nx + ii;
    }
    if (g.side < 0) {
        g.off = cell_off(d, rm.cr, cm.ci);
        g.flip = (cm.su < 0.f ? 0x80000000u : 0u) | (rm.sv < 0.f ? 0x40000000u : 0u) |
                 ((cm.sf * rm.sf) < 0.f ? 0x20000000u : 0u);
    }
    g.cof0 = corner_off(d, rm.crc, cm.cc0);
    g.cof1 = corner_off(d, rm.crc, cm.cc1);
    return g;
}

// Frame cells of a cell plane, k in [0, frame_cells(d)): the four frame rows
// (-2, -1, ny, ny+1) over columns -2 .. nx+1, then the four frame columns
// (-2, -1, nx, nx+1) over rows 0 .. ny-1.
__host__ __device__ inline int frame_cells(const Dom &d) { return 4 * (d.nx + 4) + 4 * d.ny; }
__host__ __device__ inline void frame_cell(const Dom &d, int k, int &x, int &y)
{
    const int w = d.nx + 4;
    if (k < 4 * w) {
        const int q = k / w;
        y = q < 2 ? q - 2 : d.ny + q - 2;
        x = k - q * w - 2;
    } else {
        k -= 4 * w;
        const int q = k / d.ny;
        x = q < 2 ? q - 2 : d.nx + q - 2;
        y = k - q * d.ny;
    }
}

// Frame corners of the corner plane, k in [0, frame_corners(d)): corner rows
// -2, -1, ny+1, ny+2 over corner columns -2 .. nx+2, then corner columns
// -2, -1, nx+1, nx+2 over corner rows 0 .. ny.  Corner (x, y) holds corner
// (map_corner(x), map_corner(y)).
__host__ __device__ inline int frame_corners(const Dom &d) { return 4 * (d.nx + 5) + 4 * (d.ny + 1); }
__host__ __device__ inline void frame_corner(const Dom &d, int k, int &x, int &y)
{
    const int w = d.nx + 5;
    if (k < 4 * w) {
        const int q = k / w;
        y = q < 2 ? q - 2 : d.ny + q - 1;
        x = k - q * w - 2;
    } else {
        k -= 4 * w;
        const int q = k / (d.ny + 1);
        x = q < 2 ? q - 2 : d.nx + q - 1;
        y = k - q * (d.ny + 1);
    }
}

// Ghost columns that receive a copy of cell column x: a = on the west side
// (x < 2), b = on the east side (x >= nx-2); kNoFrame where the side is
// nested (written from the boundary data instead) or x is not next to it.
// A wall ghost is the mirror image (its normal momentum negated), a
// periodic ghost the wrapped copy (periodic sides come in pairs).  The same
// along y for ghost rows.
constexpr int kNoFrame = -1000;
__host__ __device__ inline void frame_copy_cols(const Dom &d, int x, int &a, int &b)
{
    const int nx = d.nx;
    a = b = kNoFrame;
    if (x < 2) a = d.bc[0] == BC_WALL ? -1 - x : (d.bc[0] == BC_PERIODIC ? nx + x : kNoFrame);
    if (x >= nx - 2) b = d.bc[1] == BC_WALL ? 2 * nx - 1 - x : (d.bc[1] == BC_PERIODIC ? x - nx : kNoFrame);
}
__host__ __device__ inline void frame_copy_rows(const Dom &d, int y, int &a, int &b)
{
    const int ny = d.ny;
    a = b = kNoFrame;
    if (y < 2) a = d.bc[2] == BC_WALL ? -1 - y : (d.bc[2] == BC_PERIODIC ? ny + y : kNoFrame);
    if (y >= ny - 2) b = d.bc[3] == BC_WALL ? 2 * ny - 1 - y : (d.bc[3] == BC_PERIODIC ? y - ny : kNoFrame);
}

// Every frame cell that the stage writing output cell (x, y) fills for the
// stage that reads the state next, one call f(xx, yy, flip, idx) each: the
// copies above (sign bit 31 of flip: hu negated, bit 30: hv negated) and,
// from the cell next to a nested side, both ghost layers of that side
// (idx >= 0: the boundary-table entry; -1 for the copies).  Nested targets
// are written whether or not the cell is land.  With nx, ny >= 2 at most 6
// calls arise (nested on one side and a copy on the other, along both axes).
// The stage kernels write the same cells (copies from the rows they update,
// nested ghosts after their row loop); tests/host_check.cpp checks this list
// against the frame cells the outputs depend on and against the frame fill.
template <class F>
__host__ __device__ inline void for_frame_targets(const Dom &d, int x, int y, F &&f)
{
    const int nx = d.nx, ny = d.ny;
    if (x == 0 && d.bc[0] == BC_NESTED) { f(-1, y, 0u, y); f(-2, y, 0u, y); }
    else if (x == nx - 1 && d.bc[1] == BC_NESTED) { f(nx, y, 0u, ny + y); f(nx + 1, y, 0u, ny + y); }
    if (y == 0 && d.bc[2] == BC_NESTED) { f(x, -1, 0u, 2 * ny + x); f(x, -2, 0u, 2 * ny + x); }
    else if (y == ny - 1 && d.bc[3] == BC_NESTED) { f(x, ny, 0u, 2 * ny + nx + x); f(x, ny + 1, 0u, 2 * ny + nx + x); }
    int a, b;
    frame_copy_cols(d, x, a, b);
    if (a != kNoFrame) f(a, y, d.bc[0] == BC_WALL ? 0x80000000u : 0u, -1);
    if (b != kNoFrame) f(b, y, d.bc[1] == BC_WALL ? 0x80000000u : 0u, -1);
    frame_copy_rows(d, y, a, b);
    if (a != kNoFrame) f(x, a, d.bc[2] == BC_WALL ? 0x40000000u : 0u, -1);
    if (b != kNoFrame) f(x, b, d.bc[3] == BC_WALL ? 0x40000000u : 0u, -1);
}

// nearest nested side of cell (i, o) (ties W, E, S, N) and its distance in
// cells; best = -1 without nested sides
__host__ __device__ inline void frs_side(const Dom &d, int i, int o, int &best, int &dd)
{
    const int nx = d.nx, ny = d.ny;
    const int dist[4] = {i, nx - 1 - i, o, ny - 1 - o};
    best = -1;
    dd = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (d.bc[k] == BC_NESTED && (best < 0 || dist[k] < dd)) { best = k; dd = dist[k]; }
}

// boundary-table entries of cell (i, o) on the four sides (W, E, S, N), and
// the one of the nested side `best`
__host__ __device__ inline void frs_candidates(const Dom &d, int i, int o, int (&idxs)[4])
{
    idxs[0] = o;
    idxs[1] = d.ny + o;
    idxs[2] = 2 * d.ny + i;
    idxs[3] = 2 * d.ny + d.nx + i;
}

__host__ __device__ inline int frs_pick(const int (&idxs)[4], int best)
{
    return best == 0 ? idxs[0] : best == 1 ? idxs[1] : best == 2 ? idxs[2] : idxs[3];
}

}  // namespace swe
