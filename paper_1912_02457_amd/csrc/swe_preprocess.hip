// Preprocessing of the input fields on the device, before a domain is
// created: bathymetry at the cell intersections from cell values (section
// "Bathymetry"), erosion of the land mask (same section), and factor-two
// refinement and coarsening of cell fields, land mask and corner depths
// (section "Refinement and coarsening of grid").  Device pointers in and out,
// asynchronous on the caller's stream, no device memory of the library's own.
#include <cmath>
#include <cstdint>
#include <string>

#include "swe_host.h"

namespace {

using swe::set_error;

// ---------------------------------------------------------------------------
// Bathymetry reconstruction.  One launch per round; each 256-thread block
// produces a 64 x 16 tile of corners from an LDS window of the previous
// round's corners (3-corner halo), the cell values and the water flags.
//   round 0 (INIT): corners = the average over the water cells meeting there
//     of each cell's limited plane evaluated at the corner (eqs. recon_1-3)
//     applied to the cell values themselves;
//   round k >= 1: misfit dH = Hm - (mean of the cell's corners) on water
//     cells, its corner estimate by the same three equations added to the
//     corners, then H <- (1 - w) H + (w/4) (sum of the 4 neighbours) with a
//     neighbour outside the domain replaced by the corner itself.
// Corners that touch no water cell hold the mean of the four cell values
// around them (edge cells repeated).
constexpr int RTX = 64, RTY = 16, RTHREADS = 256;
constexpr int WCR = RTY + 6, WCC = RTX + 6;  // corner window
constexpr int WMR = RTY + 5, WMC = RTX + 5;  // cell window

__device__ __forceinline__ float minmod2(float a, float b)
{
    if (a > 0.0f && b > 0.0f) return fminf(a, b);
    if (a < 0.0f && b < 0.0f) return fmaxf(a, b);
    return 0.0f;
}

// Blocks go to the 8 XCDs round-robin; give each XCD a contiguous run of
// tiles so that neighbouring tiles share halo lines in the same L2.
__device__ __forceinline__ int xcd_tile(int b, int n)
{
    int q = n >> 3, r = n & 7, x = b & 7, k = b >> 3;
    return x * q + min(x, r) + k;
}

template <bool INIT>
__global__ __launch_bounds__(RTHREADS) void recon_round_kernel(int nx, int ny, int nbx, const float *__restrict__ Hm,
                                                               const uint8_t *__restrict__ land,
                                                               const float *__restrict__ Hin, float w,
                                                               float *__restrict__ Hout)
{
    __shared__ float sH[WCR][WCC];  // corners in, then corrected corners
    __shared__ float sM[WMR][WMC];  // cell values
    __shared__ float sD[WMR][WMC];  // misfit (or cell values in round 0)
    __shared__ float sSx[WMR][WMC], sSy[WMR][WMC];
    __shared__ uint8_t sW[WMR][WMC];  // water cell inside the domain

    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int J0 = (t / nbx) * RTY, I0 = (t % nbx) * RTX;
    const int nxc = nx + 1;
    const int tid = threadIdx.x;

    if (!INIT) {
        for (int idx = tid; idx < WCR * WCC; idx += RTHREADS) {
            int r = idx / WCC, c = idx - r * WCC;
            int J = J0 - 3 + r, I = I0 - 3 + c;
            bool in = J >= 0 && J <= ny && I >= 0 && I <= nx;
            sH[r][c] = in ? Hin[(uint32_t)J * (uint32_t)nxc + (uint32_t)I] : 0.0f;
        }
    }
    for (int idx = tid; idx < WMR * WMC; idx += RTHREADS) {
        int r = idx / WMC, c = idx - r * WMC;
        int j = J0 - 3 + r, i = I0 - 3 + c;
        bool in = j >= 0 && j < ny && i >= 0 && i < nx;
        uint32_t k = in ? (uint32_t)j * (uint32_t)nx + (uint32_t)i : 0u;
        sM[r][c] = in ? Hm[k] : 0.0f;
        sW[r][c] = in && (land == nullptr || land[k] == 0);
    }
    __syncthreads();

    for (int idx = tid; idx < WMR * WMC; idx += RTHREADS) {
        int r = idx / WMC, c = idx - r * WMC;
        float d = 0.0f;
        if (sW[r][c]) {
            // a water cell lies inside the domain, so its four corners do too
            d = INIT ? sM[r][c]
                     : sM[r][c] - 0.25f * (sH[r][c] + sH[r][c + 1] + sH[r + 1][c] + sH[r + 1][c + 1]);
        }
        sD[r][c] = d;
    }
    __syncthreads();

    // limited slopes (cell units); a difference toward a non-water cell is 0
    for (int idx = tid; idx < WMR * WMC; idx += RTHREADS) {
        int r = idx / WMC, c = idx - r * WMC;
        float sx = 0.0f, sy = 0.0f;
        if (r >= 1 && r < WMR - 1 && c >= 1 && c < WMC - 1 && sW[r][c]) {
            float v = sD[r][c];
            float dl = sW[r][c - 1] ? v - sD[r][c - 1] : 0.0f;
            float dr = sW[r][c + 1] ? sD[r][c + 1] - v : 0.0f;
            float ds = sW[r - 1][c] ? v - sD[r - 1][c] : 0.0f;
            float dn = sW[r + 1][c] ? sD[r + 1][c] - v : 0.0f;
            sx = minmod2(dl, dr);
            sy = minmod2(ds, dn);
        }
        sSx[r][c] = sx;
        sSy[r][c] = sy;
    }
    __syncthreads();

    // corner estimates: the planes of the (up to four) water cells at a
    // corner, evaluated there and averaged (cells taken in row-major order)
    for (int idx = tid; idx < (RTY + 2) * (RTX + 2); idx += RTHREADS) {
        int r = 2 + idx / (RTX + 2), c = 2 + idx % (RTX + 2);
        float acc = 0.0f;
        int cnt = 0;
        if (sW[r - 1][c - 1]) { acc += sD[r - 1][c - 1] + 0.5f * sSx[r - 1][c - 1] + 0.5f * sSy[r - 1][c - 1]; cnt++; }
        if (sW[r - 1][c]) { acc += sD[r - 1][c] - 0.5f * sSx[r - 1][c] + 0.5f * sSy[r - 1][c]; cnt++; }
        if (sW[r][c - 1]) { acc += sD[r][c - 1] + 0.5f * sSx[r][c - 1] - 0.5f * sSy[r][c - 1]; cnt++; }
        if (sW[r][c]) { acc += sD[r][c] - 0.5f * sSx[r][c] - 0.5f * sSy[r][c]; cnt++; }
        float est = cnt ? acc / (float)cnt : 0.0f;
        sH[r][c] = INIT ? est : sH[r][c] + est;
    }
    __syncthreads();

    for (int idx = tid; idx < RTY * RTX; idx += RTHREADS) {
        int r = 3 + idx / RTX, c = 3 + idx % RTX;
        int J = J0 - 3 + r, I = I0 - 3 + c;
        if (J > ny || I > nx) continue;
        bool keep = sW[r - 1][c - 1] | sW[r - 1][c] | sW[r][c - 1] | sW[r][c];
        float out;
        if (keep) {
            float p = sH[r][c];
            if (INIT) {
                out = p;
            } else {
                float s = sH[r][I > 0 ? c - 1 : c] + sH[r][I < nx ? c + 1 : c] + sH[J > 0 ? r - 1 : r][c] +
                          sH[J < ny ? r + 1 : r][c];
                out = (1.0f - w) * p + 0.25f * w * s;
            }
        } else {
            // cells (J-1, I-1), (J-1, I), (J, I-1), (J, I), clamped to the domain
            int rs = J > 0 ? r - 1 : r, rn = J < ny ? r : r - 1;
            int cw = I > 0 ? c - 1 : c, ce = I < nx ? c : c - 1;
            out = 0.25f * (sM[rs][cw] + sM[rs][ce] + sM[rn][cw] + sM[rn][ce]);
        }
        Hout[(uint32_t)J * (uint32_t)nxc + (uint32_t)I] = out;
    }
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
    int nbx = (nx + 1 + RTX - 1) / RTX, nby = (ny + 1 + RTY - 1) / RTY;
    int64_t tiles = (int64_t)nbx * nby;
    if (tiles > INT32_MAX) return set_error(SWE_E_ARG, "domain too large");
    // round k writes Hc when iters - k is even, so the last round ends in Hc
    float *buf[2] = {Hc, scratch};
    float *cur = buf[iters & 1];
    hipLaunchKernelGGL(recon_round_kernel<true>, dim3((unsigned)tiles), dim3(RTHREADS), 0, s, nx, ny, nbx, Hm,
                       land, (const float *)nullptr, smooth, cur);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, "recon_round_kernel<init>");
    for (int k = 1; k <= iters; ++k) {
        float *nxt = buf[(iters - k) & 1];
        hipLaunchKernelGGL(recon_round_kernel<false>, dim3((unsigned)tiles), dim3(RTHREADS), 0, s, nx, ny, nbx,
                           Hm, land, (const float *)cur, smooth, nxt);
        e = hipGetLastError();
        if (e != hipSuccess) return hip_error(e, "recon_round_kernel");
        cur = nxt;
    }
    return SWE_OK;
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
