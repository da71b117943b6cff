// Preprocessing of the input fields on the device, before a domain is
// created: bathymetry at the cell intersections from cell values (section
// "Bathymetry"), erosion of the land mask (same section), and factor-two
// refinement and coarsening of cell fields, land mask and corner depths
// (section "Refinement and coarsening of grid").  Device pointers in and out,
// asynchronous on the caller's stream, no device memory of the library's own.
#include <cmath>
#include <algorithm>
#include <cstdint>
#include <mutex>
#include <string>

#include "swe_host.h"

namespace {

using swe::set_error;

// ---------------------------------------------------------------------------
// Bathymetry reconstruction, one launch per round.
//   round 0 (INIT): corners = the average over the water cells meeting there
//     of each cell's limited plane evaluated at the corner (eqs. recon_1-3)
//     applied to the cell values themselves;
//   round k >= 1: misfit dH = Hm - (mean of the cell's corners) on water
//     cells, its corner estimate by the same three equations added to the
//     corners, then H <- (1 - w) H + (w/4) (sum of the 4 neighbours) with a
//     neighbour outside the domain replaced by the corner itself.
// Corners that touch no water cell hold the mean of the four cell values
// around them (edge cells repeated).
//
// Work decomposition: one wave per (strip, row segment).  Lane l holds
// corner column I = 58 s - 3 + l and cell column i = I (the cell to the
// upper right of the corner); an output corner reads columns I-3 .. I+3, so
// lanes 3..60 store and the six others are halo.  The wave walks up the
// rows with a register pipeline: the step that loads corner row a and cell
// row a-1 computes the misfit of cell row a-1, the slopes and corner
// contributions of cell row a-2, the corrected corners of row a-2 and the
// smoothed output row a-3.  Neighbouring columns come through DPP lane
// shifts; the next row's loads are issued before the current row is used.
constexpr int RSTRIP = 58;

constexpr int kDppShl1 = 0x130;  // wave_shl:1 -- value of lane + 1
constexpr int kDppShr1 = 0x138;  // wave_shr:1 -- value of lane - 1
__device__ __forceinline__ int lane_right(int v) { return __builtin_amdgcn_update_dpp(0, v, kDppShl1, 0xF, 0xF, false); }
__device__ __forceinline__ int lane_left(int v) { return __builtin_amdgcn_update_dpp(0, v, kDppShr1, 0xF, 0xF, false); }
__device__ __forceinline__ float lane_right(float v) { return __int_as_float(lane_right(__float_as_int(v))); }
__device__ __forceinline__ float lane_left(float v) { return __int_as_float(lane_left(__float_as_int(v))); }

// Element access through a 32-bit byte offset from a uniform base pointer
// (the scalar-base + vector-offset addressing form; no 64-bit address
// arithmetic per lane).  Every plane stays below 4 GiB.
__device__ __forceinline__ float ldf(const float *__restrict__ base, uint32_t i)
{
    return *reinterpret_cast<const float *>(reinterpret_cast<const char *>(base) + (i << 2));
}
__device__ __forceinline__ int ldb(const uint8_t *__restrict__ base, uint32_t i)
{
    return *reinterpret_cast<const uint8_t *>(reinterpret_cast<const char *>(base) + i);
}
__device__ __forceinline__ void stf(float *__restrict__ base, uint32_t i, float v)
{
    *reinterpret_cast<float *>(reinterpret_cast<char *>(base) + (i << 2)) = v;
}

__device__ __forceinline__ float minmod2(float a, float b)
{
    const float mn = fminf(a, b), mx = fmaxf(a, b);
    return ((a > 0.0f) & (b > 0.0f)) ? mn : (((a < 0.0f) & (b < 0.0f)) ? mx : 0.0f);
}

// Blocks go to the 8 XCDs round-robin; give each XCD a contiguous run of
// blocks so that neighbouring strips and segments share lines in one L2.
__device__ __forceinline__ int xcd_block(int b, int n)
{
    int q = n >> 3, r = n & 7, x = b & 7, k = b >> 3;
    return x * q + min(x, r) + k;
}

template <bool INIT, int R>
__global__ __launch_bounds__(256) void recon_round_kernel(int nx, int ny, int nsx, int nitems,
                                                          const float *__restrict__ Hm,
                                                          const uint8_t *__restrict__ land,
                                                          const float *__restrict__ Hin, float w,
                                                          float *__restrict__ Hout)
{
    constexpr int NS = R + 6;  // steps: three warm-up rows below, three above
    const int lane = threadIdx.x & 63;
    // the wave's index is the same in all its lanes: read it as a scalar, so
    // that the row offsets below are scalar too and every load and store is
    // a scalar row base plus the lane's column
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int item = xcd_block(blockIdx.x, gridDim.x) * 4 + wv;
    if (item >= nitems) return;  // whole waves leave together
    const int J0 = (item / nsx) * R, I = (item % nsx) * RSTRIP - 3 + lane;
    const uint32_t Ic = (uint32_t)min(max(I, 0), nx), ic = (uint32_t)min(max(I, 0), nx - 1);
    const bool col_in = I >= 0 && I < nx;
    const bool store = lane >= 3 && lane < 3 + RSTRIP && I <= nx;
    const uint32_t nxc = (uint32_t)nx + 1;
    const float wq = 0.25f * w, wp = 1.0f - w;
    const int a0 = J0 - 3;

    // every load of the segment first (clamped rows: always valid
    // addresses), so the wave waits for memory once, not once per row
    float Hb[NS], Mb[NS];
    int Lb[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        const uint32_t rc = (uint32_t)min(max(a0 + k, 0), ny), rm = (uint32_t)min(max(a0 + k - 1, 0), ny - 1);
        Hb[k] = INIT ? 0.f : ldf(Hin, rc * nxc + Ic);
        Mb[k] = ldf(Hm, rm * (uint32_t)nx + ic);
        Lb[k] = 0;
    }
    if (land) {
#pragma unroll
        for (int k = 0; k < NS; ++k)
            Lb[k] = ldb(land, (uint32_t)min(max(a0 + k - 1, 0), ny - 1) * (uint32_t)nx + ic);
    }

    // pipeline registers; names give the row relative to the newest corner row a
    float H1 = 0.f, H1r = 0.f, H2 = 0.f;       // corners a-1 (and its right neighbour), a-2
    float D2 = 0.f, D3 = 0.f;                  // misfit of cell rows a-2, a-3
    int W2 = 0, W3 = 0, W4 = 0, W3l = 0, W4l = 0;  // water flags (l: of the cell to the left)
    float UR3 = 0.f, UL3 = 0.f;                // cell row a-3: estimates at its upper corners
    float P3 = 0.f, P4 = 0.f;                  // corrected corners of rows a-3, a-4
    float M1 = 0.f, M2 = 0.f, M3 = 0.f;        // clamped cell values, rows a-2, a-3, a-4
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        const int a = a0 + k;
        const float Ha = Hb[k], Mc = Mb[k];

        // misfit of cell row a-1
        const int W1 = ((a - 1 >= 0) & (a - 1 < ny) & col_in & (Lb[k] == 0)) ? 1 : 0;
        const float Har = lane_right(Ha);
        const float D1 = W1 ? (INIT ? Mc : Mc - 0.25f * (H1 + H1r + Ha + Har)) : 0.f;

        // slopes and corner estimates of cell row a-2
        const float Dl = lane_left(D2), Dr = lane_right(D2);
        const int W2l = lane_left(W2), W2r = lane_right(W2);
        const float sx = minmod2(W2l ? D2 - Dl : 0.f, W2r ? Dr - D2 : 0.f);
        const float sy = minmod2(W3 ? D2 - D3 : 0.f, W1 ? D1 - D2 : 0.f);
        const float UR2 = D2 + 0.5f * sx + 0.5f * sy, UL2 = D2 - 0.5f * sx + 0.5f * sy;
        const float DR2 = D2 + 0.5f * sx - 0.5f * sy, DL2 = D2 - 0.5f * sx - 0.5f * sy;

        // corrected corner row a-2: cells (a-3, I-1), (a-3, I), (a-2, I-1), (a-2, I)
        const float UR3l = lane_left(UR3), DR2l = lane_left(DR2);
        // absent cells add +0, which leaves the running sum unchanged;
        // dividing by 1, 2 or 4 is exact, by 3 within one rounding
        const float acc = (((W3l ? UR3l : 0.f) + (W3 ? UL3 : 0.f)) + (W2l ? DR2l : 0.f)) + (W2 ? DL2 : 0.f);
        const int cnt = W3l + W3 + W2l + W2;
        const float est = acc * (cnt == 4 ? 0.25f : cnt == 3 ? 1.0f / 3.0f : cnt == 2 ? 0.5f : 1.0f);
        const float P2 = INIT ? est : H2 + est;

        // output row Y = a-3 (the first six steps only fill the pipeline)
        const int Y = a - 3;
        if (k >= 6) {
            const float P3l = lane_left(P3), P3r = lane_right(P3);
            const float M2l = lane_left(M2), M3l = lane_left(M3);
            const bool keep = (W4l | W4 | W3l | W3) != 0;
            const float fill = 0.25f * (M3l + M3 + M2l + M2);
            const float sm = (I > 0 ? P3l : P3) + (I < nx ? P3r : P3) + (Y > 0 ? P4 : P3) + (Y < ny ? P2 : P3);
            const float out = keep ? (INIT ? P3 : wp * P3 + wq * sm) : fill;
            if (store & (Y <= ny)) stf(Hout, (uint32_t)Y * nxc + (uint32_t)I, out);
        }

        H2 = H1; H1 = Ha; H1r = Har;
        D3 = D2; D2 = D1;
        W4 = W3; W3 = W2; W2 = W1; W4l = W3l; W3l = W2l;
        UR3 = UR2; UL3 = UL2;
        P4 = P3; P3 = P2;
        M3 = M2; M2 = M1; M1 = Mc;
    }
}

template <bool INIT>
hipError_t launch_recon_round(int R, unsigned blocks, hipStream_t s, int nx, int ny, int nsx, int items,
                              const float *Hm, const uint8_t *land, const float *Hin, float w, float *Hout)
{
    if (R == 16)
        hipLaunchKernelGGL((recon_round_kernel<INIT, 16>), dim3(blocks), dim3(256), 0, s, nx, ny, nsx, items, Hm,
                           land, Hin, w, Hout);
    else
        hipLaunchKernelGGL((recon_round_kernel<INIT, 8>), dim3(blocks), dim3(256), 0, s, nx, ny, nsx, items, Hm,
                           land, Hin, w, Hout);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Land erosion: a land cell with a water 4-neighbour (outside = land) turns
// into water of the given depth, its surface the largest surface among those
// water neighbours, its momenta 0.  Output mask holds 0/1.
__global__ __launch_bounds__(256) void erode_kernel(int nx, int ny, const uint8_t *__restrict__ land,
                                                    const float *__restrict__ Hm, const float *__restrict__ eta,
                                                    const float *__restrict__ hu, const float *__restrict__ hv,
                                                    float depth, uint8_t *__restrict__ land_o,
                                                    float *__restrict__ Hm_o, float *__restrict__ eta_o,
                                                    float *__restrict__ hu_o, float *__restrict__ hv_o)
{
    int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= nx) return;
    for (int j = blockIdx.y; j < ny; j += gridDim.y) {
        size_t k = (size_t)j * nx + i;
        bool L = land[k] != 0;
        bool eroded = false;
        float e = -INFINITY;
        if (L) {
            if (i > 0 && land[k - 1] == 0) { eroded = true; if (eta) e = fmaxf(e, eta[k - 1]); }
            if (i + 1 < nx && land[k + 1] == 0) { eroded = true; if (eta) e = fmaxf(e, eta[k + 1]); }
            if (j > 0 && land[k - nx] == 0) { eroded = true; if (eta) e = fmaxf(e, eta[k - nx]); }
            if (j + 1 < ny && land[k + nx] == 0) { eroded = true; if (eta) e = fmaxf(e, eta[k + nx]); }
        }
        land_o[k] = (L && !eroded) ? 1 : 0;
        Hm_o[k] = eroded ? depth : Hm[k];
        if (eta) eta_o[k] = eroded ? e : eta[k];
        if (hu) hu_o[k] = eroded ? 0.0f : hu[k];
        if (hv) hv_o[k] = eroded ? 0.0f : hv[k];
    }
}

// ---------------------------------------------------------------------------
// Factor-two refinement of cell fields: generalized-minmod slopes per cell
// (a difference toward land or the outside is 0), evaluated at the four
// sub-cell centres.  n_fields planes; rows of all planes are strided over
// gridDim.y.  The land mask is inherited by the children (plane 0 writes it).
__device__ __forceinline__ float minmod3(float a, float b, float c)
{
    if (a > 0.0f && b > 0.0f && c > 0.0f) return fminf(a, fminf(b, c));
    if (a < 0.0f && b < 0.0f && c < 0.0f) return fmaxf(a, fmaxf(b, c));
    return 0.0f;
}

__global__ __launch_bounds__(256) void refine_cells_kernel(int nx, int ny, int nf, const float *__restrict__ in,
                                                           const uint8_t *__restrict__ land, float theta,
                                                           float *__restrict__ out, uint8_t *__restrict__ land_o)
{
    int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= nx) return;
    const size_t plane = (size_t)nx * ny, oplane = 4 * plane;
    for (long row = blockIdx.y; row < (long)nf * ny; row += gridDim.y) {
        int f = (int)(row / ny), j = (int)(row - (long)f * ny);
        const float *v = in + f * plane;
        size_t k = (size_t)j * nx + i;
        auto wet = [&](size_t q) { return land == nullptr || land[q] == 0; };
        float c = v[k], sx = 0.0f, sy = 0.0f;
        bool L = !wet(k);
        if (!L) {
            float dl = (i > 0 && wet(k - 1)) ? c - v[k - 1] : 0.0f;
            float dr = (i + 1 < nx && wet(k + 1)) ? v[k + 1] - c : 0.0f;
            float ds = (j > 0 && wet(k - nx)) ? c - v[k - nx] : 0.0f;
            float dn = (j + 1 < ny && wet(k + nx)) ? v[k + nx] - c : 0.0f;
            sx = minmod3(theta * dl, 0.5f * (dl + dr), theta * dr);
            sy = minmod3(theta * ds, 0.5f * (ds + dn), theta * dn);
        }
        float *o = out + f * oplane + (size_t)(2 * j) * (2 * nx) + 2 * i;
        float2 lo = make_float2(c + -0.25f * sx + -0.25f * sy, c + 0.25f * sx + -0.25f * sy);
        float2 hi = make_float2(c + -0.25f * sx + 0.25f * sy, c + 0.25f * sx + 0.25f * sy);
        *reinterpret_cast<float2 *>(o) = lo;
        *reinterpret_cast<float2 *>(o + 2 * nx) = hi;
        if (f == 0 && land_o) {
            uint8_t b = L ? 1 : 0;
            uint8_t *lo8 = land_o + (size_t)(2 * j) * (2 * nx) + 2 * i;
            lo8[0] = b; lo8[1] = b; lo8[2 * nx] = b; lo8[2 * nx + 1] = b;
        }
    }
}

// Corner depths at the refined intersections: the bilinear surface of each
// coarse cell at its corners, edge midpoints and centre.
__global__ __launch_bounds__(256) void refine_corners_kernel(int nx, int ny, const float *__restrict__ Hc,
                                                             float *__restrict__ out)
{
    const int NX = 2 * nx + 1, NY = 2 * ny + 1;
    int I = blockIdx.x * 256 + threadIdx.x;
    if (I >= NX) return;
    for (int J = blockIdx.y; J < NY; J += gridDim.y) {
        int j = J >> 1, i = I >> 1;
        const float *a = Hc + (size_t)j * (nx + 1) + i;
        float v;
        if (!(J & 1) && !(I & 1)) v = a[0];
        else if (!(J & 1)) v = 0.5f * (a[0] + a[1]);
        else if (!(I & 1)) v = 0.5f * (a[0] + a[nx + 1]);
        else v = 0.25f * ((a[0] + a[1]) + (a[nx + 1] + a[nx + 2]));
        out[(size_t)J * NX + I] = v;
    }
}

// Factor-two coarsening: the average of the water children (all four when
// none is water); a coarse cell is land when all four children are.
__global__ __launch_bounds__(256) void coarsen_cells_kernel(int nx, int ny, int nf, const float *__restrict__ in,
                                                            const uint8_t *__restrict__ land,
                                                            float *__restrict__ out, uint8_t *__restrict__ land_o)
{
    const int cx = nx / 2, cy = ny / 2;
    int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= cx) return;
    const size_t plane = (size_t)nx * ny, oplane = (size_t)cx * cy;
    for (long row = blockIdx.y; row < (long)nf * cy; row += gridDim.y) {
        int f = (int)(row / cy), j = (int)(row - (long)f * cy);
        size_t k0 = (size_t)(2 * j) * nx + 2 * i, k1 = k0 + nx;
        const float *v = in + f * plane;
        float2 a = *reinterpret_cast<const float2 *>(v + k0);
        float2 b = *reinterpret_cast<const float2 *>(v + k1);
        bool w0 = true, w1 = true, w2 = true, w3 = true;
        if (land) { w0 = land[k0] == 0; w1 = land[k0 + 1] == 0; w2 = land[k1] == 0; w3 = land[k1 + 1] == 0; }
        bool any = w0 | w1 | w2 | w3;
        if (!any) w0 = w1 = w2 = w3 = true;
        float s = 0.0f;
        int n = 0;
        if (w0) { s += a.x; n++; }
        if (w1) { s += a.y; n++; }
        if (w2) { s += b.x; n++; }
        if (w3) { s += b.y; n++; }
        out[f * oplane + (size_t)j * cx + i] = s / (float)n;
        if (f == 0 && land_o) land_o[(size_t)j * cx + i] = any ? 0 : 1;
    }
}

__global__ __launch_bounds__(256) void coarsen_corners_kernel(int nx, int ny, const float *__restrict__ Hc,
                                                              float *__restrict__ out)
{
    const int CX = nx / 2 + 1, CY = ny / 2 + 1;
    int I = blockIdx.x * 256 + threadIdx.x;
    if (I >= CX) return;
    for (int J = blockIdx.y; J < CY; J += gridDim.y)
        out[(size_t)J * CX + I] = Hc[(size_t)(2 * J) * (nx + 1) + 2 * I];
}

// ---------------------------------------------------------------------------
constexpr int64_t kPlaneLimit = (int64_t)1 << 32;  // bytes of any one plane

bool plane_ok(int64_t rows, int64_t cols, int64_t elem) { return rows * cols * elem < kPlaneLimit; }

int hip_error(hipError_t e, const char *what)
{
    return set_error(SWE_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

dim3 row_grid(int64_t cols, int64_t rows)
{
    return dim3((unsigned)((cols + 255) / 256), (unsigned)std::min<int64_t>(rows, 32768));
}

}  // namespace

extern "C" int swe_reconstruct_bathymetry(int32_t nx, int32_t ny, const float *Hm, const uint8_t *land,
                                          int32_t iters, float smooth, float *Hc, float *scratch,
                                          void *hip_stream)
{
    if (nx < 1 || ny < 1) return set_error(SWE_E_ARG, "nx and ny must be >= 1");
    if (!plane_ok(ny + 1, nx + 1, 4)) return set_error(SWE_E_ARG, "corner plane must stay below 4 GiB");
    if (!Hm || !Hc) return set_error(SWE_E_ARG, "Hm and Hc must be device pointers");
    if (iters < 0 || iters > 100000) return set_error(SWE_E_ARG, "iters must be in [0, 100000]");
    if (iters > 0 && !scratch) return set_error(SWE_E_ARG, "scratch is required when iters > 0");
    if (!(smooth >= 0.0f && smooth <= 1.0f)) return set_error(SWE_E_ARG, "smooth must be in [0, 1]");
    hipStream_t s = (hipStream_t)hip_stream;
    // rows per segment: 16 when that still gives about four waves per SIMD,
    // else 8 (more waves, more warm-up rows)
    const int nsx = (nx + 1 + RSTRIP - 1) / RSTRIP;
    const int R = (int64_t)nsx * ((ny + 1 + 15) / 16) >= 4096 ? 16 : 8;
    const int nsy = (ny + 1 + R - 1) / R;
    const int64_t items = (int64_t)nsx * nsy;
    if (items > INT32_MAX / 2) return set_error(SWE_E_ARG, "domain too large");
    const unsigned blocks = (unsigned)((items + 3) / 4);
    // round k writes Hc when iters - k is even, so the last round ends in Hc
    float *buf[2] = {Hc, scratch};
    float *cur = buf[iters & 1];
    hipError_t e = launch_recon_round<true>(R, blocks, s, nx, ny, nsx, (int)items, Hm, land, nullptr, smooth, cur);
    if (e != hipSuccess) return hip_error(e, "recon_round_kernel<init>");
    for (int k = 1; k <= iters; ++k) {
        float *nxt = buf[(iters - k) & 1];
        e = launch_recon_round<false>(R, blocks, s, nx, ny, nsx, (int)items, Hm, land, cur, smooth, nxt);
        if (e != hipSuccess) return hip_error(e, "recon_round_kernel");
        cur = nxt;
    }
    return SWE_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free reconstruction: the corner plane the rounds ping-pong
// through lives in a device array of the library's own instead of caller
// memory.  Each GPU the library runs on holds its own copy of the array
// until the process ends; in host code the array's name is only a stand-in,
// so its device address is looked up once per device (hipGetSymbolAddress,
// with that device current) and only that address is handed to kernels.
// Every round overwrites every corner of the plane it writes, so nothing in
// the array has to start at zero.
// ---------------------------------------------------------------------------
namespace {

constexpr int64_t kStaticScratchFloats = (int64_t)4 << 20;  // 16 MiB: up to 4,194,304 corners
static __device__ __align__(256) float scratch[kStaticScratchFloats];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float *g_scratch_ptr[kMaxDevices] = {};

// device address of this device's copy of `scratch`
int static_scratch(float **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_error(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return set_error(SWE_E_ARG, "device index beyond the static scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_error(e, "hipGetSymbolAddress(scratch)");
        if (!p) return set_error(SWE_E_HIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = static_cast<float *>(p);
    }
    *out = g_scratch_ptr[dev];
    return SWE_OK;
}

}  // namespace

extern "C" int swe_reconstruct_bathymetry_noalloc(int32_t nx, int32_t ny, const float *Hm, const uint8_t *land,
                                                  int32_t iters, float smooth, float *Hc, void *hip_stream)
{
    if (nx < 1 || ny < 1) return set_error(SWE_E_ARG, "nx and ny must be >= 1");
    if ((int64_t)(nx + 1) * (int64_t)(ny + 1) > kStaticScratchFloats)
        return set_error(SWE_E_ARG, "corner plane larger than the static scratch ((nx+1)(ny+1) <= 4194304)");
    float *scr = nullptr;
    if (iters > 0) {
        const int rc = static_scratch(&scr);
        if (rc != SWE_OK) return rc;
    }
    return swe_reconstruct_bathymetry(nx, ny, Hm, land, iters, smooth, Hc, scr, hip_stream);
}

extern "C" int swe_erode_land(int32_t nx, int32_t ny, const uint8_t *land, const float *Hm, const float *eta,
                              const float *hu, const float *hv, float land_depth, uint8_t *land_out,
                              float *Hm_out, float *eta_out, float *hu_out, float *hv_out, void *hip_stream)
{
    if (nx < 1 || ny < 1) return set_error(SWE_E_ARG, "nx and ny must be >= 1");
    if (!plane_ok(ny, nx, 4)) return set_error(SWE_E_ARG, "cell plane must stay below 4 GiB");
    if (!land || !Hm || !land_out || !Hm_out) return set_error(SWE_E_ARG, "land, Hm and their outputs are required");
    if ((eta == nullptr) != (eta_out == nullptr) || (hu == nullptr) != (hu_out == nullptr) ||
        (hv == nullptr) != (hv_out == nullptr))
        return set_error(SWE_E_ARG, "eta, hu and hv need an output exactly when given");
    if (!std::isfinite(land_depth)) return set_error(SWE_E_ARG, "land_depth must be finite");
    hipLaunchKernelGGL(erode_kernel, row_grid(nx, ny), dim3(256), 0, (hipStream_t)hip_stream, nx, ny, land, Hm, eta,
                       hu, hv, land_depth, land_out, Hm_out, eta_out, hu_out, hv_out);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SWE_OK : hip_error(e, "erode_kernel");
}

extern "C" int swe_refine2(int32_t nx, int32_t ny, int32_t n_fields, const float *fields, const uint8_t *land,
                           float theta, float *fields_out, uint8_t *land_out, const float *Hc, float *Hc_out,
                           void *hip_stream)
{
    if (nx < 1 || ny < 1 || n_fields < 0) return set_error(SWE_E_ARG, "nx, ny >= 1 and n_fields >= 0 required");
    if (!plane_ok(2 * (int64_t)ny + 1, 2 * (int64_t)nx + 1, 4))
        return set_error(SWE_E_ARG, "refined corner plane must stay below 4 GiB");
    if (n_fields > 0 && (!fields || !fields_out)) return set_error(SWE_E_ARG, "fields and fields_out are required");
    if (land_out && (!land || n_fields == 0)) return set_error(SWE_E_ARG, "land_out needs land and at least one field");
    if ((Hc == nullptr) != (Hc_out == nullptr)) return set_error(SWE_E_ARG, "Hc and Hc_out go together");
    if (!(theta >= 1.0f && theta <= 2.0f)) return set_error(SWE_E_ARG, "theta must be in [1, 2]");
    hipStream_t s = (hipStream_t)hip_stream;
    if (n_fields > 0) {
        hipLaunchKernelGGL(refine_cells_kernel, row_grid(nx, (int64_t)n_fields * ny), dim3(256), 0, s, nx, ny,
                           n_fields, fields, land, theta, fields_out, land_out);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_error(e, "refine_cells_kernel");
    }
    if (Hc) {
        hipLaunchKernelGGL(refine_corners_kernel, row_grid(2 * (int64_t)nx + 1, 2 * (int64_t)ny + 1), dim3(256), 0, s,
                           nx, ny, Hc, Hc_out);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_error(e, "refine_corners_kernel");
    }
    return SWE_OK;
}

extern "C" int swe_coarsen2(int32_t nx, int32_t ny, int32_t n_fields, const float *fields, const uint8_t *land,
                            float *fields_out, uint8_t *land_out, const float *Hc, float *Hc_out, void *hip_stream)
{
    if (nx < 2 || ny < 2 || (nx & 1) || (ny & 1) || n_fields < 0)
        return set_error(SWE_E_ARG, "nx and ny must be even and >= 2, n_fields >= 0");
    if (!plane_ok(ny + 1, nx + 1, 4)) return set_error(SWE_E_ARG, "corner plane must stay below 4 GiB");
    if (n_fields > 0 && (!fields || !fields_out)) return set_error(SWE_E_ARG, "fields and fields_out are required");
    if (land_out && (!land || n_fields == 0)) return set_error(SWE_E_ARG, "land_out needs land and at least one field");
    if ((Hc == nullptr) != (Hc_out == nullptr)) return set_error(SWE_E_ARG, "Hc and Hc_out go together");
    hipStream_t s = (hipStream_t)hip_stream;
    if (n_fields > 0) {
        hipLaunchKernelGGL(coarsen_cells_kernel, row_grid(nx / 2, (int64_t)n_fields * (ny / 2)), dim3(256), 0, s, nx,
                           ny, n_fields, fields, land, fields_out, land_out);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_error(e, "coarsen_cells_kernel");
    }
    if (Hc) {
        hipLaunchKernelGGL(coarsen_corners_kernel, row_grid(nx / 2 + 1, ny / 2 + 1), dim3(256), 0, s, nx, ny, Hc,
                           Hc_out);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_error(e, "coarsen_corners_kernel");
    }
    return SWE_OK;
}
