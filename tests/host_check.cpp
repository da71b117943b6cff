// Host-side checks of the index arithmetic and the allocator the library
// runs, built with AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_host_sanitized.py (no GPU needed):
//
//  1. every element a stage kernel reads or writes lies inside its framed
//     plane or table: for each tile of every tiling the tuner can pick (one
//     and two band heights, four tile orders) of domains from 2 x 2 up,
//     under every combination of boundary kinds, the row and corner loads,
//     the own-cell loads and stores, the frame writes of edge tiles
//     (swe_maps.h: for_frame_targets), the boundary-table entries of nested
//     ghosts and the relaxation-zone entries;
//  2. the frames: the cells the stage kernels write for the next stage are
//     exactly the frame cells an output depends on (the ghost columns next to
//     rows 0 .. ny-1 and the ghost rows next to columns 0 .. nx-1), each
//     written once, with the source and sign flips (or boundary entry) that
//     the library's frame fill takes for it (ghost_src); the fill's
//     enumerations of frame cells and frame corners cover each exactly once
//     and read only interior cells and corners;
//  3. at the largest domain the library accepts, the 32-bit element offsets
//     equal the exact ones (no wrap-around);
//  4. the serving loop's arena allocator (swe_arena.h) under random
//     allocate / release sequences: blocks are aligned, never overlap each
//     other or the free list, the free list stays coalesced, used + free
//     equals the size, and releasing everything leaves one free block.
#include "swe_arena.h"
#include "swe_device.h"
#include "swe_maps.h"

#include <cstdint>
#include <cstdio>
#include <map>
#include <random>
#include <set>
#include <utility>
#include <vector>

using namespace swe;

static long g_bad = 0;

#define CHECK(cond, ...)                                                   \
    do {                                                                   \
        if (!(cond)) {                                                     \
            if (g_bad < 20) { printf("FAIL %s: ", #cond); printf(__VA_ARGS__); printf("\n"); } \
            ++g_bad;                                                       \
        }                                                                  \
    } while (0)

static int pitch_of(int n) { return (n + 63) / 64 * 64; }

// the layout of swe_api.hip's make_layout
static Dom make_dom(int nx, int ny, const int bc[4], int frs_w)
{
    Dom d{};
    d.nx = nx; d.ny = ny;
    d.pitch = pitch_of(frame_cols(nx));
    d.cpitch = pitch_of(frame_cols(nx) + 1);
    d.P = 2 * nx + 2 * ny;
    for (int k = 0; k < 4; ++k) d.bc[k] = bc[k];
    d.frs_w = frs_w;
    return d;
}

static uint64_t plane_elems(const Dom &d) { return (uint64_t)frame_rows(d.ny) * d.pitch; }
static uint64_t corner_elems(const Dom &d) { return (uint64_t)(frame_rows(d.ny) + 1) * d.cpitch; }

// every access of one stage launch under tiling T (nb boundary snapshots)
static void check_tiling(const Dom &d, const Tiling &T, int nb)
{
    const int nx = d.nx, ny = d.ny;
    const uint64_t plane = plane_elems(d), cplane = corner_elems(d);
    const uint64_t P = (uint64_t)d.P;
    const uint64_t bnd_elems = (uint64_t)(nb > 0 ? nb : 1) * 3 * P;
    for (int b = 0; b < T.nblocks; ++b)
        for (int w = 0; w < kWavesPerBlock; ++w) {
            const int tile = block_tile(T, b, w);
            if (tile < 0) continue;
            int strip, y0, y1;
            tile_place(T, tile, ny, strip, y0, y1);
            const int x0 = strip * kStrip;
            const bool edge = x0 < kHalo || x0 + kStrip > nx - kHalo || y0 < kHalo || y1 > ny - kHalo;
            const int klast = y1 + 1;
            for (int lane = 0; lane < kWave; ++lane) {
                const int i = x0 - kHalo + lane;
                const bool out_lane = lane >= kHalo && lane < kWave - kHalo && i < nx;
                CHECK(i >= -kFrame && (uint64_t)(i + kFrame) < (uint64_t)d.pitch, "column %d of %dx%d", i, nx, ny);
                CHECK(corner_off(d, y0 - 2, i) + 1 < cplane, "first corner row, tile %d", tile);
                for (int k = y0 - 2; k <= klast; ++k) {
                    CHECK(k >= -kFrame && cell_off(d, k, i) < plane, "row %d col %d", k, i);
                    CHECK(corner_off(d, k + 1, i) + 1 < cplane, "corner row %d", k + 1);
                }
                for (int o = y0; o < y1; ++o) {
                    // own-cell loads (every lane) and stores (output lanes)
                    CHECK(cell_off(d, o, i) < plane, "own cell %d %d", o, i);
                    if (!out_lane) continue;
                    if (edge)
                        for_frame_targets(d, i, o, [&](int xx, int yy, uint32_t, int idx) {
                            CHECK(xx >= -kFrame && xx < nx + kFrame && yy >= -kFrame && yy < ny + kFrame,
                                  "frame target %d %d", xx, yy);
                            CHECK(cell_off(d, yy, xx) < plane, "frame target offset");
                            if (idx >= 0) {
                                CHECK(nb >= 1, "nested frame without boundary snapshots");
                                CHECK((uint64_t)idx < P, "boundary entry %d", idx);
                                for (int bk = 0; bk <= (nb > 1 ? nb - 2 : 0); ++bk) {
                                    const uint64_t last = (uint64_t)bk * 3 * P + (uint64_t)idx + 2 * P + (nb > 1 ? 3 * P : 0);
                                    CHECK(last < bnd_elems, "boundary snapshot element %llu", (unsigned long long)last);
                                }
                            }
                        });
                    else
                        for_frame_targets(d, i, o, [&](int, int, uint32_t, int) {
                            CHECK(false, "interior tile cell %d %d has frame targets", i, o);
                        });
                    // relaxation zone
                    if (d.frs_w > 0) {
                        int best, dd;
                        frs_side(d, i, o, best, dd);
                        if (best >= 0 && dd < d.frs_w) {
                            CHECK(dd >= 0 && dd < kMaxFrs, "zone distance %d", dd);
                            int idxs[4];
                            frs_candidates(d, i, o, idxs);
                            const int idx = frs_pick(idxs, best);
                            CHECK(idx >= 0 && (uint64_t)idx < P, "zone boundary entry %d", idx);
                        }
                    }
                }
            }
        }
}

// the frame cells written by the stages, against the frame cells an output
// depends on and against the library's frame fill (ghost_src)
static void check_frames(const Dom &d)
{
    const int nx = d.nx, ny = d.ny;
    std::map<std::pair<int, int>, int> seen;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x)
            for_frame_targets(d, x, y, [&](int xx, int yy, uint32_t flip, int idx) {
                ++seen[std::make_pair(xx, yy)];
                const GhostSrc g = ghost_src(d, col_map(d, xx), xx, yy);
                if (idx >= 0) {
                    CHECK(g.side >= 0 && g.idx == idx, "nested frame (%d, %d): fill entry %d, stage entry %d", xx, yy,
                          g.idx, idx);
                } else {
                    CHECK(g.side < 0 && g.off == cell_off(d, y, x), "frame (%d, %d): fill source differs from (%d, %d)",
                          xx, yy, x, y);
                    CHECK((g.flip & 0xC0000000u) == flip, "frame (%d, %d): sign flips %x vs %x", xx, yy, g.flip, flip);
                }
            });
    // the frame cells an output depends on: ghost columns beside rows 0 .. ny-1,
    // ghost rows beside columns 0 .. nx-1; each written exactly once
    size_t want = 0;
    auto times = [&](int x, int y) {
        const auto it = seen.find(std::make_pair(x, y));
        return it == seen.end() ? 0 : it->second;
    };
    for (int y = 0; y < ny; ++y)
        for (int xx : {-2, -1, nx, nx + 1}) {
            ++want;
            const int n = times(xx, y);
            CHECK(n == 1, "ghost column cell (%d, %d) written %d times (%dx%d, bc %d%d%d%d)", xx, y, n, nx, ny, d.bc[0],
                  d.bc[1], d.bc[2], d.bc[3]);
        }
    for (int x = 0; x < nx; ++x)
        for (int yy : {-2, -1, ny, ny + 1}) {
            ++want;
            const int n = times(x, yy);
            CHECK(n == 1, "ghost row cell (%d, %d) written %d times", x, yy, n);
        }
    CHECK(seen.size() == want, "%zu frame cells written, %zu expected", seen.size(), want);
    // the fill's enumerations: each frame cell / corner once, interior sources
    std::set<std::pair<int, int>> cells, corners;
    for (int k = 0; k < frame_cells(d); ++k) {
        int x, y;
        frame_cell(d, k, x, y);
        CHECK(x >= -2 && x < nx + 2 && y >= -2 && y < ny + 2 && !(x >= 0 && x < nx && y >= 0 && y < ny),
              "frame cell %d -> (%d, %d)", k, x, y);
        cells.insert(std::make_pair(x, y));
        const GhostSrc g = ghost_src(d, col_map(d, x), x, y);
        if (g.side < 0) {
            const RowMap rm = row_map(d, y);
            const ColMap cm = col_map(d, x);
            CHECK(rm.cr >= 0 && rm.cr < ny && cm.ci >= 0 && cm.ci < nx, "frame (%d, %d) source (%d, %d)", x, y, cm.ci, rm.cr);
        } else {
            CHECK(g.idx >= 0 && g.idx < d.P && g.layer >= 0 && g.layer < 2, "frame (%d, %d) entry %d", x, y, g.idx);
        }
    }
    CHECK((int)cells.size() == (nx + 4) * (ny + 4) - nx * ny, "frame cells enumerated %zu", cells.size());
    for (int k = 0; k < frame_corners(d); ++k) {
        int x, y;
        frame_corner(d, k, x, y);
        CHECK(x >= -2 && x <= nx + 2 && y >= -2 && y <= ny + 2 && !(x >= 0 && x <= nx && y >= 0 && y <= ny),
              "frame corner %d -> (%d, %d)", k, x, y);
        corners.insert(std::make_pair(x, y));
        const int cx = map_corner(x, nx, d.bc[0], d.bc[1]), cy = map_corner(y, ny, d.bc[2], d.bc[3]);
        CHECK(cx >= 0 && cx <= nx && cy >= 0 && cy <= ny, "corner (%d, %d) source (%d, %d)", x, y, cx, cy);
    }
    CHECK((int)corners.size() == (nx + 5) * (ny + 5) - (nx + 1) * (ny + 1), "frame corners enumerated %zu",
          corners.size());
}

static void check_maps()
{
    const int nxs[] = {2, 3, 5, 60, 61, 62, 63, 65, 121, 257};
    const int nys[] = {2, 3, 5, 7, 16, 33, 100};
    long cases = 0, frames = 0;
    for (int nx : nxs)
        for (int ny : nys)
            for (int bx = 0; bx < 3; ++bx)
                for (int byk = 0; byk < 3; ++byk)
                    for (int mixed = 0; mixed < 2; ++mixed) {
                        // periodic needs both sides of an axis; a wall/nested mix otherwise
                        int bc[4];
                        bc[0] = bx; bc[1] = bx == BC_PERIODIC ? BC_PERIODIC : (mixed ? (bx == BC_WALL ? BC_NESTED : BC_WALL) : bx);
                        bc[2] = byk; bc[3] = byk == BC_PERIODIC ? BC_PERIODIC : (mixed ? (byk == BC_WALL ? BC_NESTED : BC_WALL) : byk);
                        const bool nested = bc[0] == BC_NESTED || bc[1] == BC_NESTED || bc[2] == BC_NESTED || bc[3] == BC_NESTED;
                        const Dom d = make_dom(nx, ny, bc, nested ? 10 : 0);
                        check_frames(d);
                        ++frames;
                        for (int nb : {1, 3}) {
                            if (!nested && nb > 1) continue;
                            for (int by = 1; by <= 24; by += (by < 8 ? 1 : 5))
                                for (int tail : {0, 1, 3})
                                    for (int order = 0; order < 4; ++order) {
                                        Tiling T = make_tiling_tail(nx, ny, by, tail ? 1 + tail % 3 : 0, tail * 2);
                                        T.order = order;
                                        check_tiling(d, T, nested ? nb : 0);
                                        ++cases;
                                    }
                        }
                    }
    printf("maps: %ld tilings and %ld frame layouts checked\n", cases, frames);
}

// 32-bit element offsets at the largest domains the library accepts (the
// framed corner plane just below 4 GiB): equal to the exact 64-bit ones
static void check_offsets_largest()
{
    const int bc[4] = {BC_NESTED, BC_WALL, BC_PERIODIC, BC_PERIODIC};
    const int shapes[][2] = {{16384, 16384}, {32700, 32000}, {65500, 16000}, {2, 500000000}};
    for (auto &s : shapes) {
        const int nx = s[0], ny = s[1];
        if ((uint64_t)(frame_rows(ny) + 1) * pitch_of(frame_cols(nx) + 1) * 4 >= ((uint64_t)1 << 32)) continue;
        const Dom d = make_dom(nx, ny, bc, 10);
        const int cols[] = {-2, -1, 0, 1, nx / 2, nx - 1, nx, nx + 1, frame_cols(nx) - 3};
        const int rows[] = {-2, -1, 0, 1, ny / 2, ny - 2, ny - 1, ny, ny + 1};
        for (int c : cols)
            for (int r : rows) {
                const uint64_t exact = (uint64_t)(r + 2) * (uint64_t)d.pitch + (uint64_t)(c + 2);
                CHECK(exact == cell_off(d, r, c) && exact < plane_elems(d) && (exact << 2) < ((uint64_t)1 << 32),
                      "cell offset wraps at %dx%d (%d, %d)", nx, ny, c, r);
                const uint64_t ce = (uint64_t)(r + 3) * (uint64_t)d.cpitch + (uint64_t)(c + 3);
                CHECK(ce == corner_off(d, r + 1, c + 1) && ce < corner_elems(d) && (ce << 2) < ((uint64_t)1 << 32),
                      "corner offset wraps at %dx%d", nx, ny);
                const GhostSrc g = ghost_src(d, col_map(d, c), c, r);
                CHECK(g.cof1 < corner_elems(d), "ghost corner beyond the plane at %dx%d", nx, ny);
            }
    }
    printf("offsets: largest domains checked\n");
}

static void check_arena()
{
    std::mt19937_64 rng(12345);
    long ops = 0;
    for (int trial = 0; trial < 200; ++trial) {
        Arena a;
        const size_t size = (size_t)(1 + rng() % 4096) * kArenaAlign + (rng() % 3) * 17;
        a.reset(size / kArenaAlign * kArenaAlign);
        const size_t cap = a.size();
        std::vector<std::pair<size_t, size_t>> live;  // (offset, aligned bytes)
        for (int step = 0; step < 400; ++step, ++ops) {
            if (!live.empty() && (rng() % 3 == 0 || step > 350)) {
                const size_t k = rng() % live.size();
                a.release(live[k].first, live[k].second);
                live.erase(live.begin() + (long)k);
            } else {
                const size_t want = 1 + rng() % (cap / 4 + 1);
                size_t off = 0;
                if (a.alloc(want, &off)) {
                    const size_t bytes = arena_align_up(want);
                    CHECK(off % kArenaAlign == 0 && off + bytes <= cap, "block [%zu, %zu) of %zu", off, off + bytes, cap);
                    for (auto &b : live)
                        CHECK(off + bytes <= b.first || b.first + b.second <= off, "blocks overlap");
                    live.push_back({off, bytes});
                }
            }
            size_t used = 0, freeb = 0, prev_end = 0;
            bool first = true;
            for (auto &b : live) used += b.second;
            a.each_free([&](size_t o, size_t n) {
                CHECK(n > 0 && o % kArenaAlign == 0 && o + n <= cap, "free block [%zu, %zu)", o, o + n);
                if (!first) CHECK(o > prev_end, "free blocks not coalesced at %zu", o);
                for (auto &b : live) CHECK(o + n <= b.first || b.first + b.second <= o, "free block overlaps a live one");
                prev_end = o + n;
                first = false;
                freeb += n;
            });
            CHECK(used == a.used() && used + freeb == cap && a.peak() >= used, "accounting %zu + %zu != %zu", used,
                  freeb, cap);
        }
        for (auto &b : live) a.release(b.first, b.second);
        int nfree = 0;
        a.each_free([&](size_t o, size_t n) { CHECK(o == 0 && n == cap, "not one block after release"); ++nfree; });
        CHECK(a.used() == 0 && nfree == (cap ? 1 : 0), "arena not empty after releasing all");
    }
    printf("arena: %ld operations checked\n", ops);
}

int main()
{
    check_maps();
    check_offsets_largest();
    check_arena();
    printf("bad %ld\n", g_bad);
    return g_bad != 0;
}
