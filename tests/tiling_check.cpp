// Host-side check of the stage kernels' wave-to-tile map (block_tile,
// tile_place) for one and two band heights, every tile order, and ragged,
// tiny and large domains: every (strip, row) of the domain is covered by
// exactly one wave, every tile index is produced once, and every tile's rows
// lie inside the domain.  Built and run by tests/test_tiling_map.py.
#include "swe_device.h"

#include <cstdio>
#include <vector>

using namespace swe;

static long check(int nx, int ny, const Tiling &T0, int order)
{
    Tiling T = T0;
    T.order = order;
    long bad = 0;
    std::vector<unsigned char> cover((size_t)T.nstrips * ny, 0);
    std::vector<unsigned char> seen(T.ntiles, 0);
    for (int b = 0; b < T.nblocks; ++b)
        for (int w = 0; w < kWavesPerBlock; ++w) {
            const int t = block_tile(T, b, w);
            if (t < 0) continue;
            if (t >= T.ntiles) { ++bad; continue; }
            seen[t]++;
            int s, y0, y1;
            tile_place(T, t, ny, s, y0, y1);
            if (s < 0 || s >= T.nstrips || y0 < 0 || y0 >= y1 || y1 > ny) { ++bad; continue; }
            for (int y = y0; y < y1; ++y) cover[(size_t)s * ny + y]++;
        }
    for (unsigned char v : seen) bad += v != 1;
    for (unsigned char v : cover) bad += v != 1;
    if (T.nrb1 < T.nrb && !(T.by2 > 0 && T.by2 < T.by)) ++bad;
    if (bad) printf("FAIL nx %d ny %d by %d by2 %d nrb1 %d nrb %d order %d: %ld\n", nx, ny, T.by, T.by2, T.nrb1,
                    T.nrb, order, bad);
    return bad;
}

int main()
{
    long cases = 0, bad = 0;
    const int nxs[] = {2, 5, 60, 61, 119, 1000, 2600};
    const int nys[] = {2, 3, 16, 17, 97, 301, 900};
    const int tails[] = {0, 1, 2, 5, 17, 64, 150, 899};
    for (int nx : nxs)
        for (int ny : nys)
            for (int by = 1; by <= 70; by += (by < 16 ? 1 : 7))
                for (int by2 = 0; by2 <= 5; ++by2)
                    for (int tail : tails)
                        for (int order = 0; order < 4; ++order) {
                            bad += check(nx, ny, make_tiling_tail(nx, ny, by, by2, tail), order);
                            ++cases;
                        }
    // the largest domain the build addresses, with the tilings the tuner picks there
    const int big[][3] = {{48, 3, 500}, {24, 2, 300}, {64, 4, 772}, {5, 0, 0}};
    for (auto &q : big)
        for (int order = 0; order < 4; order += 1) {
            bad += check(16384, 16384, make_tiling_tail(16384, 16384, q[0], q[1], q[2]), order);
            ++cases;
        }
    printf("cases %ld bad %ld\n", cases, bad);
    return bad != 0;
}
