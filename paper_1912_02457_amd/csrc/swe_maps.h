// Index maps of the stage kernels' loads, shared by the device code and the
// host-side bounds check (tests/host_check.cpp): the virtual ghost cells of
// the boundary kinds, the corner depths around them, and the nearest nested
// side of a relaxation-zone cell.  Pure integer arithmetic, no memory access.
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

// Source of a ghost-path load of row r at lane column il (il in [-2, nx+1]):
// a nested ghost reads boundary-table entry idx (side >= 0, layer 0 or 1);
// any other cell reads element `off` of the state planes, with the sign
// flips of a wall ghost in `flip` (bits 31, 30, 29: hu, hv, f).  cof0 / cof1
// are the corner-plane elements of the cell's north-west / north-east
// corners.  A lane in a ghost column only ever contributes rows inside
// [0, ny); its rows outside (diagonal ghosts) read some in-bounds value that
// is never used.
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
        g.off = (uint32_t)rm.cr * (uint32_t)d.pitch + (uint32_t)cm.ci;
        g.flip = (cm.su < 0.f ? 0x80000000u : 0u) | (rm.sv < 0.f ? 0x40000000u : 0u) |
                 ((cm.sf * rm.sf) < 0.f ? 0x20000000u : 0u);
    }
    const uint32_t cof = (uint32_t)rm.crc * (uint32_t)d.cpitch;
    g.cof0 = cof + (uint32_t)cm.cc0;
    g.cof1 = cof + (uint32_t)cm.cc1;
    return g;
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
