// Host-side checks of the index arithmetic and the allocator the library
// runs, built with AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_host_sanitized.py (no GPU needed):
//
//  1. every element a stage kernel reads or writes lies inside its plane or
//     table: for each tile of every tiling the tuner can pick (one and two
//     band heights, four tile orders) of domains from 2 x 2 up, under every
//     combination of boundary kinds, the state and corner offsets of the
//     plain path, the ghost sources (swe_maps.h: ghost_src, col_map,
//     row_map, map_corner -- the functions and composition the kernels
//     use), the own-cell loads and stores, the boundary-table and ghost
//     tables of nested sides, and the relaxation-zone entries;
//  2. at the largest domain the library accepts, the 32-bit element offsets
//     equal the exact ones (no wrap-around);
//  3. the serving loop's arena allocator (swe_arena.h) under random
//     allocate / release sequences: blocks are aligned, never overlap each
//     other or the free list, the free list stays coalesced, used + free
//     equals the size, and releasing everything leaves one free block.
#include "swe_arena.h"
#include "swe_device.h"
#include "swe_maps.h"

#include <cstdint>
#include <cstdio>
#include <random>
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

static Dom make_dom(int nx, int ny, const int bc[4], int frs_w)
{
    Dom d{};
    d.nx = nx; d.ny = ny;
    d.pitch = pitch_of(nx);
    d.cpitch = pitch_of(nx + 1);
    d.P = 2 * nx + 2 * ny;
    for (int k = 0; k < 4; ++k) d.bc[k] = bc[k];
    d.frs_w = frs_w;
    return d;
}

// every access of one stage launch under tiling T (nb boundary snapshots)
static void check_tiling(const Dom &d, const Tiling &T, int nb)
{
    const int nx = d.nx, ny = d.ny;
    const uint64_t plane = (uint64_t)ny * d.pitch, cplane = (uint64_t)(ny + 1) * d.cpitch;
    const uint64_t P = (uint64_t)d.P;
    const uint64_t bnd_elems = (uint64_t)(nb > 0 ? nb : 1) * 3 * P;
    for (int b = 0; b < T.nblocks; ++b)
        for (int w = 0; w < kWavesPerBlock; ++w) {
            const int tile = block_tile(T, b, w);
            if (tile < 0) continue;
            int strip, y0, y1;
            tile_place(T, tile, ny, strip, y0, y1);
            const int x0 = strip * kStrip;
            const bool ghost = !(x0 >= kHalo && x0 + kStrip + kHalo <= nx && y0 >= kHalo && y1 + kHalo <= ny);
            const int klast = y1 + 1;
            for (int lane = 0; lane < kWave; ++lane) {
                const int i = x0 - kHalo + lane;
                const bool out_lane = lane >= kHalo && lane < kWave - kHalo && i < nx;
                if (!ghost) {
                    CHECK(i >= 0 && i < nx, "plain tile column %d of %dx%d", i, nx, ny);
                    const uint64_t c0 = (uint64_t)(y0 - 2) * d.cpitch + (uint64_t)i;
                    CHECK(y0 - 2 >= 0 && c0 + 1 < cplane, "first corner row, tile %d", tile);
                    for (int k = y0 - 2; k <= klast; ++k) {
                        CHECK(k >= 0 && (uint64_t)k * d.pitch + (uint64_t)i < plane, "row %d col %d", k, i);
                        CHECK((uint64_t)(k + 1) * d.cpitch + (uint64_t)i + 1 < cplane, "corner row %d", k + 1);
                    }
                } else {
                    const int il = imin(i, nx + 1);
                    const ColMap cm = col_map(d, il);
                    CHECK(cm.cc0 >= 0 && cm.cc0 <= nx && cm.cc1 >= 0 && cm.cc1 <= nx, "corner cols %d %d", cm.cc0,
                          cm.cc1);
                    const int c0r = map_corner(y0 - 2, ny, d.bc[2], d.bc[3]);
                    CHECK(c0r >= 0 && c0r <= ny, "first corner row %d", c0r);
                    for (int k = y0 - 2; k <= klast; ++k) {
                        const GhostSrc g = ghost_src(d, cm, il, k);
                        if (g.side >= 0) {
                            CHECK(nb >= 1, "nested ghost without boundary snapshots");
                            CHECK(g.idx >= 0 && (uint64_t)g.idx < P && g.layer >= 0 && g.layer < 2,
                                  "boundary entry %d layer %d", g.idx, g.layer);
                            for (int bk = 0; bk <= (nb > 1 ? nb - 2 : 0); ++bk) {
                                const uint64_t a = (uint64_t)bk * 3 * P + (uint64_t)g.idx;
                                const uint64_t last = a + 2 * P + (nb > 1 ? 3 * P : 0);
                                CHECK(last < bnd_elems, "boundary snapshot element %llu", (unsigned long long)last);
                            }
                            CHECK((uint64_t)g.layer * P + (uint64_t)g.idx < 2 * P, "ghost-table entry");
                        } else {
                            CHECK(g.off < plane, "ghost source %u of %llu (row %d col %d)", g.off,
                                  (unsigned long long)plane, k, il);
                        }
                        CHECK(g.cof0 < cplane && g.cof1 < cplane, "ghost corners %u %u", g.cof0, g.cof1);
                    }
                }
                if (!out_lane) continue;
                for (int o = y0; o < y1; ++o) {
                    // own-cell loads and stores of the update
                    CHECK(i >= 0 && (uint64_t)o * d.pitch + (uint64_t)i < plane, "own cell %d %d", o, i);
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

static void check_maps()
{
    const int nxs[] = {2, 3, 5, 60, 61, 62, 63, 65, 121, 257};
    const int nys[] = {2, 3, 5, 7, 16, 33, 100};
    long cases = 0;
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
    printf("maps: %ld tilings checked\n", cases);
}

// 32-bit element offsets at the largest domain the library accepts (its
// corner plane just below 4 GiB): equal to the exact 64-bit ones
static void check_offsets_largest()
{
    const int bc[4] = {BC_NESTED, BC_WALL, BC_PERIODIC, BC_PERIODIC};
    // nx, ny with (ny + 1) * pitch(nx + 1) * 4 < 2^32
    const int shapes[][2] = {{16384, 16384}, {32767, 32000}, {65535, 16000}, {2, 500000000}};
    for (auto &s : shapes) {
        const int nx = s[0], ny = s[1];
        if ((uint64_t)(ny + 1) * pitch_of(nx + 1) * 4 >= ((uint64_t)1 << 32)) continue;
        const Dom d = make_dom(nx, ny, bc, 10);
        const int cols[] = {-2, -1, 0, 1, nx / 2, nx - 1, nx, nx + 1};
        const int rows[] = {-2, -1, 0, 1, ny / 2, ny - 2, ny - 1, ny, ny + 1};
        for (int c : cols)
            for (int r : rows) {
                const ColMap cm = col_map(d, c);
                const RowMap rm = row_map(d, r);
                const GhostSrc g = ghost_src(d, cm, c, r);
                if (g.side < 0) {
                    const uint64_t exact = (uint64_t)rm.cr * (uint64_t)d.pitch + (uint64_t)cm.ci;
                    CHECK(exact == g.off && exact < ((uint64_t)1 << 30), "offset wraps at %dx%d (%d, %d)", nx, ny, c, r);
                }
                const uint64_t ce = (uint64_t)rm.crc * (uint64_t)d.cpitch + (uint64_t)cm.cc1;
                CHECK(ce == g.cof1 && ce < ((uint64_t)1 << 30), "corner offset wraps at %dx%d", nx, ny);
            }
        // the plain path's row offset at the last row and column
        const uint64_t last = (uint64_t)(ny - 1) * d.pitch + (uint64_t)(nx - 1);
        CHECK((uint32_t)((uint32_t)(ny - 1) * (uint32_t)d.pitch + (uint32_t)(nx - 1)) == last, "row offset wraps");
        CHECK((last << 2) < ((uint64_t)1 << 32), "byte offset of a plane element beyond 4 GiB");
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
