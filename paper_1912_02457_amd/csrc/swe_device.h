// Device-side data structures of the gfx950 shallow-water stage kernels.
//
// One domain lives in a caller-provided device workspace:
//   state Q^n (eta, hu, hv) and Q* as float32 planes, the corner depths, the
//   Coriolis plane f in which NaN marks a land cell (the static mask costs no
//   extra bytes, as in the section "Moving wet-dry boundary and land mask"),
//   small forcing tables and a control block holding the time, the CFL
//   accumulators and the error flag.
//
// Every plane carries a frame of kHalo ghost cells on each side, so that the
// stage kernels read ghost cells like any other (no per-lane boundary logic
// in the row loop): cell (i, r), -2 <= i < nx + 2 (and the padding columns
// up to the last strip's reach), -2 <= r < ny + 2, is element
// (r + 2) * pitch + (i + 2); corner (i, r), -2 <= i, r <= n + 2, is element
// (r + 2) * cpitch + (i + 2) of the corner plane.  The frames of the static
// planes (f, north angle, corner depths) are filled at init; those of Q^n
// and Q* by the stage that writes the state, for the stage that reads it.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace swe {

enum { BC_WALL = 0, BC_PERIODIC = 1, BC_NESTED = 2 };
enum { FR_NONE = 0, FR_LINEAR = 1, FR_QUADRATIC = 2, FR_MANNING = 3 };

constexpr int kWave = 64;                  // wavefront width on CDNA
constexpr int kHalo = 2;                   // stencil reach: slope of the neighbour's face value
constexpr int kStrip = kWave - 2 * kHalo;  // output columns per wave
constexpr int kWavesPerBlock = 4;
constexpr int kMaxFrs = 32;

// The CFL maximum is accumulated with atomicMax into kCflSlots words, each on
// its own 128-byte line and picked by tile index, so that thousands of
// wavefronts do not serialise on one address; readers take the max of the
// slots (one per lane of a wavefront).
constexpr int kCflSlots = 64;
constexpr int kCflStride = 32;  // uint32 words between slots (128 B)

// Control block; the time and the CFL accumulator are double-buffered by
// step parity so that both stage kernels of a step read the same values
// while the next step's slots are being produced.
struct Ctrl {
    double t[2];         // time at the start of the step of each parity
    uint32_t flags;      // bit 0: non-finite state produced; bit 1: water depth below -kappa
    float dt_last;       // dt of the last step taken
    int64_t steps;       // steps taken (no-op steps past t_end excluded)
    double t_end;        // > 0: clamp steps to end exactly at t_end, skip steps after it
    double mass, energy; // results of the diagnostics reduction
    // dt update policy (Dom::dt_interval > 0): dt held since the last update
    // and the time of the next update, per parity like t
    double dt_hold[2], t_upd[2];
    double pad[5];
    // max over non-land cells of max((|u|+c)/dx, (|v|+c)/dy) as float bits, per parity
    uint32_t wslot[2][kCflSlots][kCflStride];
};

// host-side text of the error flags
inline const char *flag_message(uint32_t flags)
{
    if ((flags & 3u) == 3u) return "non-finite state and water depth below -kappa";
    return (flags & 2u) ? "water depth below -kappa (positivity lost)" : "non-finite state";
}

// host-side maximum over the slots of one parity
inline float ctrl_wmax(const Ctrl &c, int parity)
{
    uint32_t m = 0;
    for (int k = 0; k < kCflSlots; ++k) m = c.wslot[parity][k][0] > m ? c.wslot[parity][k][0] : m;
    float f;
    __builtin_memcpy(&f, &m, sizeof(f));
    return f;
}

// host-side: the dt the next step of this parity takes (t_end clamp aside)
inline double ctrl_next_dt(const Ctrl &c, int parity, float courant_q, double dt_interval)
{
    if (dt_interval > 0.0 && c.dt_hold[parity] > 0.0 && c.t[parity] < c.t_upd[parity]) return c.dt_hold[parity];
    float wm = ctrl_wmax(c, parity);
    return wm > 0 ? (double)(courant_q / wm) : INFINITY;
}

// Everything a stage kernel needs, passed by value.
struct Dom {
    int nx, ny, pitch, cpitch, P;  // P = 2 ny + 2 nx perimeter cells; pitches of the framed planes
    int bc[4];                     // W, E, S, N
    float dx, dy, rdx, rdy, kx, ky; // kx = dx / (2 g)
    float g, theta, kappa, inv2kappa, kappa_sq, courant_q; // courant_q = C / 4
    float theta2;                  // 2 theta (the limiter works on twice the slopes)
    float grdx2, grdy2;            // g / (2 dx), g / (2 dy): the bathymetry source's factors
    int friction;
    float fric_c;                  // r, r, or g n^2 (Manning)
    double inv_rho_w;
    double dt_interval;            // > 0: dt re-evaluated only once this much time has passed
    double g64, kappa64, dx64, dy64;  // float64 copies for the diagnostics reductions
    int frs_w;
    float *eta, *hu, *hv;          // Q^n, updated in place by stage 2 (all planes: frame origin)
    float *eta1, *hu1, *hv1;       // Q*
    // compensated state (swe_params.compensated_state): the rounding error of
    // each stored value of Q^n and Q*, kept as the upper 16 bits of its
    // float32 value (bfloat16, framed like the state), so that value + error carries
    // the state to about 2^-10 of a float32 ulp; NULL when off
    uint16_t *eta_lo, *hu_lo, *hv_lo, *eta1_lo, *hu1_lo, *hv1_lo;
    const float *Hc, *f, *north;
    const float *fghost, *nghost;  // [2 layers][P] f and north angle of nested ghost cells
    const float *frs_alpha;        // [kMaxFrs] 1 - tanh(d / d0)
    int nb;                        // boundary snapshots
    const double *bnd_t;
    const float *bnd;              // [nb][3][P]
    int nw;                        // wind snapshots
    const double *wind_t;
    const float *wind;             // [nw][2]
    int w10n, w10nx, w10ny;        // wind at 10 m on its own grid: snapshots, samples (0 = none)
    float w10sx, w10sy;            // samples per cell along x and y
    float w10q;                    // rho_air / rho_w (wind at 10 m) or 1 / rho_w (stress field)
    int w10_kind;                  // 0: wind at 10 m, stress of Large and Pond per cell; 1: stress field
    const double *w10_t;
    const float *w10;              // [w10n][w10ny][w10nx][2] m/s
    Ctrl *ctrl;
    double *partials;              // diagnostics partial sums
};

// frame layout (see the top of this file)
constexpr int kFrame = kHalo;
__host__ __device__ inline uint32_t cell_off(const Dom &d, int r, int i)
{
    return (uint32_t)(r + kFrame) * (uint32_t)d.pitch + (uint32_t)(i + kFrame);
}
__host__ __device__ inline uint32_t corner_off(const Dom &d, int r, int i)
{
    return (uint32_t)(r + kFrame) * (uint32_t)d.cpitch + (uint32_t)(i + kFrame);
}
// columns a plane must hold: the lanes of the last 60-column strip reach
// column 60 * nstrips + 1; corners one further
__host__ __device__ inline int frame_cols(int nx) { return (nx + kStrip - 1) / kStrip * kStrip + 2 * kFrame; }
__host__ __device__ inline int frame_rows(int ny) { return ny + 2 * kFrame; }

struct Tiling {
    int by;       // rows per wave of the head bands
    int order;    // bit 0: row-block-major tile numbering; bit 1: no XCD grouping
    int nstrips;  // ceil(nx / kStrip)
    int nrb;      // row bands in all
    int ntiles;   // nstrips * nrb
    int nblocks;  // blocks of the launch
    int by2;      // rows per wave of the tail bands (== by: one band height)
    int nrb1;     // head bands, by rows each; bands nrb1 .. nrb-1 have by2 rows
    int ntiles1;  // nstrips * nrb1: tiles 0 .. ntiles1-1 lie in the head
    int nblk1;    // blocks 0 .. nblk1-1 hold the head tiles, the rest the tail
};

// Rows per wave for a domain.  A wave's work is proportional to its rows plus
// the ~4 halo rows it also loads and reconstructs; the kernel time is about
// the total work spread over the resident wave slots plus one wave's worth of
// tail (measured on config-2, 1024^2 and 4096^2 domains: this picks 8, 5-7 and
// 16-24 rows, the measured optima).
inline int pick_rows_per_wave(int nx, int ny, int cus, int waves_per_simd)
{
    const double slots = (double)cus * 4 * waves_per_simd;
    const long nstrips = (nx + kStrip - 1) / kStrip;
    int best = 8;
    double best_cost = 1e300;
    for (int by = 2; by <= 256; by += (by < 16 ? 1 : (by < 64 ? 4 : 16))) {
        long waves = nstrips * ((ny + by - 1) / by);
        double cost = (double)waves * (by + 4) / slots + (by + 4);
        if (cost < best_cost - 1e-9) { best_cost = cost; best = by; }
    }
    return best;
}

// One band height for the whole domain.
inline Tiling make_tiling(int nx, int ny, int by)
{
    Tiling t;
    t.by = by;
    t.order = 0;
    t.nstrips = (nx + kStrip - 1) / kStrip;
    t.nrb = (ny + by - 1) / by;
    t.ntiles = t.nstrips * t.nrb;
    t.nblocks = (t.ntiles + kWavesPerBlock - 1) / kWavesPerBlock;
    t.by2 = by;
    t.nrb1 = t.nrb;
    t.ntiles1 = t.ntiles;
    t.nblk1 = t.nblocks;
    return t;
}

// Two band heights: the first rows in bands of `by` rows (the head), the last
// rows -- at least tail_rows of them -- in bands of by2 < by rows (the tail).
// The head's tiles are launched first, so the waves that finish the launch
// are the short tail waves: the drain at the end of a launch shrinks while
// most rows keep the lower halo overhead of tall bands.  Falls back to one
// band height when the arguments leave no head or no tail.
inline Tiling make_tiling_tail(int nx, int ny, int by, int by2, int tail_rows)
{
    Tiling t = make_tiling(nx, ny, by);
    if (by2 <= 0 || by2 >= by || tail_rows <= 0 || tail_rows >= ny) return t;
    const int nrb1 = (ny - tail_rows) / by;
    if (nrb1 <= 0) return t;
    const int ytail = nrb1 * by;
    t.by2 = by2;
    t.nrb1 = nrb1;
    t.nrb = nrb1 + (ny - ytail + by2 - 1) / by2;
    t.ntiles1 = t.nstrips * nrb1;
    t.ntiles = t.nstrips * t.nrb;
    t.nblk1 = (t.ntiles1 + kWavesPerBlock - 1) / kWavesPerBlock;
    t.nblocks = t.nblk1 + (t.ntiles - t.ntiles1 + kWavesPerBlock - 1) / kWavesPerBlock;
    return t;
}

// Blocks are dispatched round-robin over the 8 XCDs.  Unless order bit 1 is
// set, block b of a range of n blocks is renumbered so that each XCD gets a
// contiguous run of the range (neighbouring tiles share halo rows in that
// XCD's L2).  A bijection of [0, n).
__host__ __device__ inline int xcd_group(int b, int n, int order)
{
    if (order & 2) return b;
    const int q8 = n >> 3, r8 = n & 7, x8 = b & 7;
    return x8 * q8 + (x8 < r8 ? x8 : r8) + (b >> 3);
}

// Tile of wave `wid` of block b, or -1 for a wave without one.  Head blocks
// come first and carry only head tiles; each part is grouped per XCD on its own.
__host__ __device__ inline int block_tile(const Tiling &T, int b, int wid)
{
    if (b < T.nblk1) {
        const int t = xcd_group(b, T.nblk1, T.order) * kWavesPerBlock + wid;
        return t < T.ntiles1 ? t : -1;
    }
    const int t = T.ntiles1 + xcd_group(b - T.nblk1, T.nblocks - T.nblk1, T.order) * kWavesPerBlock + wid;
    return t < T.ntiles ? t : -1;
}

// Strip and rows [y0, y1) of a tile (0 <= tile < T.ntiles).  Within the head
// and within the tail, tiles are numbered strip-major (order bit 0 clear) or
// row-band-major, with the strips in the order 0, last, 1, 2, ...
__host__ __device__ inline void tile_place(const Tiling &T, int tile, int ny, int &strip, int &y0, int &y1)
{
    int t = tile, nb = T.nrb1, by = T.by, base = 0;
    if (tile >= T.ntiles1) {
        t = tile - T.ntiles1;
        nb = T.nrb - T.nrb1;
        by = T.by2;
        base = T.nrb1 * T.by;
    }
    int rb;
    if (T.order & 1) { rb = t / T.nstrips; strip = t - rb * T.nstrips; }
    else { strip = t / nb; rb = t - strip * nb; }
    // the two edge strips (ghost columns, relaxation zones: the slowest
    // tiles) come first, so that they are not left for the end of a launch
    strip = strip == 0 ? 0 : (strip == 1 ? T.nstrips - 1 : strip - 1);
    y0 = base + rb * by;
    y1 = y0 + by < ny ? y0 + by : ny;
}

// ---- ensemble: many domains in one launch per stage ------------------------
constexpr int kEnsParts = 8;  // queue partitions (blocks b with b % 8 == k drain part k)

struct EnsMember {
    Dom d;
    Tiling T;
    int pflip;  // this member's step parity = ensemble parity ^ pflip
    int pad[3];
};

struct EnsItem {
    int member;
    int tile;
};

struct EnsCtrl {
    uint32_t head[2][2][kEnsParts][32];  // [stage][parity][part], one 128-byte line each
    uint32_t part_begin[kEnsParts];
    uint32_t part_len[kEnsParts];
};

}  // namespace swe
