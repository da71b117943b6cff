// Host side of the C ABI declared in include/swe.h: parameter validation,
// workspace layout, uploads, launches, HIP-graph replay of step chunks and
// kernel timing.  No exception crosses the ABI.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "swe_host.h"

using namespace swe;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(SWE_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr)                                   \
    do {                                                \
        hipError_t e_ = (expr);                         \
        if (e_ != hipSuccess) return hip_fail(e_, #expr); \
    } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
int pitch_of(int n) { return (int)align_up((size_t)n, 64); }

Layout make_layout(const swe_params &p, int max_wind, int max_bnd)
{
    Layout L;
    // framed planes (swe_device.h): cells -2 .. nx+1 (and the last strip's
    // reach) by -2 .. ny+1, corners one row and column more
    const int fc = frame_cols(p.nx);
    size_t plane = (size_t)frame_rows(p.ny) * pitch_of(fc) * sizeof(float);
    size_t cplane = (size_t)(frame_rows(p.ny) + 1) * pitch_of(fc + 1) * sizeof(float);
    size_t P = 2 * (size_t)p.ny + 2 * (size_t)p.nx;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes, kAlign); return o; };
    L.eta = take(plane); L.hu = take(plane); L.hv = take(plane);
    L.eta1 = take(plane); L.hu1 = take(plane); L.hv1 = take(plane);
    const size_t lo = p.compensated_state ? plane / 2 : 0;  // 16-bit rounding errors
    L.eta_lo = take(lo); L.hu_lo = take(lo); L.hv_lo = take(lo);
    L.eta1_lo = take(lo); L.hu1_lo = take(lo); L.hv1_lo = take(lo);
    L.Hc = take(cplane);
    L.f = take(plane);
    L.north = p.north_projection ? take(plane) : take(0);
    L.fghost = take(2 * P * sizeof(float));
    L.nghost = take(2 * P * sizeof(float));
    L.alpha = take(kMaxFrs * sizeof(float));
    L.bnd_t = take((size_t)max_bnd * sizeof(double));
    L.bnd = take((size_t)max_bnd * 3 * P * sizeof(float));
    L.wind_t = take((size_t)max_wind * sizeof(double));
    L.wind = take((size_t)max_wind * 2 * sizeof(float));
    L.ctrl = take(sizeof(Ctrl));
    L.partials = take(2 * (size_t)p.ny * sizeof(double));
    L.total = off;
    return L;
}

int validate(const swe_params *p)
{
    if (!p) return fail(SWE_E_ARG, "params is NULL");
    if (p->nx < 2 || p->ny < 2) return fail(SWE_E_ARG, "nx and ny must be >= 2");
    // the kernels address a plane with 32-bit byte offsets: the framed
    // corner-depth plane, the largest, must stay below 4 GiB (about 1.07e9
    // cells)
    if (p->nx > (1 << 29) || p->ny > (1 << 29) ||
        (int64_t)(frame_rows(p->ny) + 1) * (int64_t)(((int64_t)frame_cols(p->nx) + 1 + 63) / 64 * 64) * 4 >=
            ((int64_t)1 << 32))
        return fail(SWE_E_ARG, "domain too large: one plane must stay below 4 GiB");
    if (!(std::isfinite(p->dx) && p->dx > 0 && std::isfinite(p->dy) && p->dy > 0))
        return fail(SWE_E_ARG, "dx and dy must be finite and > 0");
    if (!(std::isfinite(p->g) && p->g > 0)) return fail(SWE_E_ARG, "g must be > 0");
    if (!(p->courant > 0 && p->courant <= 1)) return fail(SWE_E_ARG, "courant must be in (0, 1]");
    if (!(p->theta >= 1 && p->theta <= 2)) return fail(SWE_E_ARG, "theta must be in [1, 2]");
    if (!(std::isfinite(p->kappa) && p->kappa > 0)) return fail(SWE_E_ARG, "kappa must be > 0");
    for (int k = 0; k < 4; ++k)
        if (p->bc[k] < SWE_BC_WALL || p->bc[k] > SWE_BC_NESTED) return fail(SWE_E_ARG, "unknown boundary kind");
    if ((p->bc[0] == SWE_BC_PERIODIC) != (p->bc[1] == SWE_BC_PERIODIC) ||
        (p->bc[2] == SWE_BC_PERIODIC) != (p->bc[3] == SWE_BC_PERIODIC))
        return fail(SWE_E_ARG, "periodic boundaries must be set on both sides of an axis");
    if (p->friction < SWE_FRICTION_NONE || p->friction > SWE_FRICTION_MANNING)
        return fail(SWE_E_ARG, "unknown friction law");
    if (!(std::isfinite(p->friction_coeff) && p->friction_coeff >= 0))
        return fail(SWE_E_ARG, "friction_coeff must be >= 0");
    if (!(std::isfinite(p->rho_w) && p->rho_w > 0)) return fail(SWE_E_ARG, "rho_w must be > 0");
    if (p->frs_width < 1 || p->frs_width > kMaxFrs) return fail(SWE_E_ARG, "frs_width must be in [1, 32]");
    if (!(std::isfinite(p->frs_d0) && p->frs_d0 > 0)) return fail(SWE_E_ARG, "frs_d0 must be > 0");
    if (p->north_projection != 0 && p->north_projection != 1) return fail(SWE_E_ARG, "north_projection must be 0 or 1");
    if (p->compensated_state != 0 && p->compensated_state != 1)
        return fail(SWE_E_ARG, "compensated_state must be 0 or 1");
    return SWE_OK;
}

bool all_finite(const float *a, size_t n)
{
    uint32_t bad = 0;  // branch-free so that the loop vectorises
    for (size_t k = 0; k < n; ++k) {
        uint32_t b;
        std::memcpy(&b, a + k, sizeof b);
        bad |= (uint32_t)((b & 0x7f800000u) == 0x7f800000u);
    }
    return bad == 0;
}

bool any_nested(const swe_params &p)
{
    for (int k = 0; k < 4; ++k)
        if (p.bc[k] == SWE_BC_NESTED) return true;
    return false;
}

}  // namespace

int swe::set_error(int code, const std::string &msg) { return fail(code, msg); }

namespace {

// Host-to-device uploads go through one process-wide pinned staging buffer
// (at most 64 MiB, larger arrays go in row chunks): a copy from pageable
// memory straight into a pitched device plane would be split by the runtime
// into row-sized transfers.  The buffer is held for the whole upload
// sequence of one call.
constexpr size_t kStageCap = (size_t)64 << 20;
std::mutex g_stage_mu;
char *g_stage = nullptr;
size_t g_stage_bytes = 0;

class Uploader {
public:
    Uploader(hipStream_t s, size_t hint) : lk_(g_stage_mu), s_(s) { hint_ = std::min(hint, kStageCap); }
    ~Uploader()
    {
        if (pending_) (void)hipStreamSynchronize(s_);
    }
    // w x h floats (rows of w) into device rows of dpitch floats at dst
    hipError_t plane(void *dst, int dpitch, const float *src, int w, int h)
    {
        const size_t rowb = (size_t)w * sizeof(float);
        hipError_t e;
        if ((e = ensure(std::max(rowb, hint_))) != hipSuccess) return e;
        for (int r0 = 0; r0 < h;) {
            size_t room = g_stage_bytes - used_;
            if (room < rowb) {
                if ((e = flush()) != hipSuccess) return e;
                room = g_stage_bytes;
            }
            const int rows = (int)std::min<size_t>((size_t)(h - r0), room / rowb);
            char *stg = g_stage + used_;
            std::memcpy(stg, src + (size_t)r0 * w, (size_t)rows * rowb);
            e = hipMemcpy2DAsync((char *)dst + (size_t)r0 * dpitch * sizeof(float), (size_t)dpitch * sizeof(float),
                                 stg, rowb, rowb, (size_t)rows, hipMemcpyHostToDevice, s_);
            if (e != hipSuccess) return e;
            pending_ = true;
            used_ += ((size_t)rows * rowb + 255) / 256 * 256;
            r0 += rows;
        }
        return hipSuccess;
    }
    hipError_t flush()
    {
        hipError_t e = pending_ ? hipStreamSynchronize(s_) : hipSuccess;
        pending_ = false;
        used_ = 0;
        return e;
    }

private:
    hipError_t ensure(size_t need)
    {
        if (g_stage_bytes >= need) return hipSuccess;
        if (pending_) {
            hipError_t e = flush();
            if (e != hipSuccess) return e;
        }
        if (g_stage) (void)hipHostFree(g_stage);
        g_stage = nullptr;
        g_stage_bytes = 0;
        hipError_t e = hipHostMalloc((void **)&g_stage, need, hipHostMallocDefault);
        if (e == hipSuccess) g_stage_bytes = need;
        return e;
    }
    std::unique_lock<std::mutex> lk_;
    hipStream_t s_;
    size_t hint_ = 0, used_ = 0;
    bool pending_ = false;
};

// f of the two ghost layers of nested sides: the mirrored interior cell
// (layer 0 <- the outermost interior cell, layer 1 <- the next one), with the
// real f even where that cell is land.
void build_ghost_table(const swe_params &p, const float *field, std::vector<float> &out)
{
    const int nx = p.nx, ny = p.ny, P = 2 * nx + 2 * ny;
    out.assign(2 * (size_t)P, 0.f);
    for (int layer = 0; layer < 2; ++layer) {
        float *o = out.data() + (size_t)layer * P;
        for (int j = 0; j < ny; ++j) {
            o[j] = field ? field[(size_t)j * nx + layer] : 0.f;
            o[ny + j] = field ? field[(size_t)j * nx + (nx - 1 - layer)] : 0.f;
        }
        for (int i = 0; i < nx; ++i) {
            o[2 * ny + i] = field ? field[(size_t)layer * nx + i] : 0.f;
            o[2 * ny + nx + i] = field ? field[(size_t)(ny - 1 - layer) * nx + i] : 0.f;
        }
    }
}

int reset_time_and_cfl(swe_domain *d, double t)
{
    d->parity = 0;
    HIP_TRY(launch_ctrl_reset(d->dom.ctrl, t, 0, d->stream));
    HIP_TRY(launch_cfl(d->dom, 0, d->stream));
    return SWE_OK;
}

// A new Q^n (init, set_state): its frame for the time of the current
// parity, then Q* (frames included) as a copy of it.
int copy_state_to_star(swe_domain *d)
{
    HIP_TRY(launch_frame_state(d->dom, d->parity, d->stream));
    size_t plane = (size_t)frame_rows(d->p.ny) * d->dom.pitch * sizeof(float);
    HIP_TRY(hipMemcpyAsync(d->dom.eta1, d->dom.eta, plane, hipMemcpyDeviceToDevice, d->stream));
    HIP_TRY(hipMemcpyAsync(d->dom.hu1, d->dom.hu, plane, hipMemcpyDeviceToDevice, d->stream));
    HIP_TRY(hipMemcpyAsync(d->dom.hv1, d->dom.hv, plane, hipMemcpyDeviceToDevice, d->stream));
    // a state handed in as float32 values carries no rounding error yet
    uint16_t *lo[6] = {d->dom.eta_lo, d->dom.hu_lo, d->dom.hv_lo, d->dom.eta1_lo, d->dom.hu1_lo, d->dom.hv1_lo};
    for (uint16_t *q : lo)
        if (q) HIP_TRY(hipMemsetAsync(q, 0, plane / 2, d->stream));
    return SWE_OK;
}

int check_ready(swe_domain *d)
{
    if (!d) return fail(SWE_E_ARG, "domain is NULL");
    if (d->ensemble) return fail(SWE_E_STATE, "domain belongs to an ensemble: step the ensemble");
    if (any_nested(d->p) && !d->has_bnd) return fail(SWE_E_STATE, "nested boundary without boundary data");
    return SWE_OK;
}

int launch_step(swe_domain *d, int parity, double dt_fixed, hipStream_t s, bool timed)
{
    bool proj = d->p.north_projection != 0;
    if (timed) {
        while (d->ev_pool.size() < d->ev_used + 4) {
            hipEvent_t ev;
            HIP_TRY(hipEventCreate(&ev));
            d->ev_pool.push_back(ev);
        }
        hipEvent_t *pe = &d->ev_pool[d->ev_used];
        HIP_TRY(launch_stage(1, proj, d->dom, d->T[0], parity, dt_fixed, s, pe[0], pe[1]));
        HIP_TRY(launch_stage(2, proj, d->dom, d->T[1], parity, dt_fixed, s, pe[2], pe[3]));
        d->ev_used += 4;
        d->timed_steps += 1;
        return SWE_OK;
    }
    HIP_TRY(launch_stage(1, proj, d->dom, d->T[0], parity, dt_fixed, s, nullptr, nullptr));
    HIP_TRY(launch_stage(2, proj, d->dom, d->T[1], parity, dt_fixed, s, nullptr, nullptr));
    return SWE_OK;
}

constexpr int kGraphChunk = 16;

int get_graph(swe_domain *d, int steps, int parity, hipGraphExec_t *out)
{
    auto key = std::make_pair(steps, parity);
    auto it = d->graphs.find(key);
    if (it != d->graphs.end()) { *out = it->second; return SWE_OK; }
    if (!d->capture_stream) HIP_TRY(hipStreamCreateWithFlags(&d->capture_stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(d->capture_stream, hipStreamCaptureModeThreadLocal));
    int rc = SWE_OK;
    for (int k = 0; k < steps && rc == SWE_OK; ++k) rc = launch_step(d, (parity + k) & 1, 0.0, d->capture_stream, false);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(d->capture_stream, &g);
    if (rc != SWE_OK) { if (g) (void)hipGraphDestroy(g); return rc; }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (e != hipSuccess) { (void)hipGraphDestroy(g); return hip_fail(e, "hipGraphInstantiate"); }
    d->graph_objs.push_back(g);
    d->graphs[key] = ex;
    *out = ex;
    return SWE_OK;
}

// Captured step graphs embed the tiling: dropped when it changes.
void drop_graphs(swe_domain *d)
{
    for (auto &kv : d->graphs) (void)hipGraphExecDestroy(kv.second);
    for (auto g : d->graph_objs) (void)hipGraphDestroy(g);
    d->graphs.clear();
    d->graph_objs.clear();
}

int read_ctrl(swe_domain *d, Ctrl *c)
{
    if (!d->pinned_ctrl) HIP_TRY(hipHostMalloc((void **)&d->pinned_ctrl, sizeof(Ctrl), hipHostMallocDefault));
    HIP_TRY(hipMemcpyAsync(d->pinned_ctrl, d->dom.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, d->stream));
    HIP_TRY(hipStreamSynchronize(d->stream));
    std::memcpy(c, d->pinned_ctrl, sizeof(Ctrl));
    return SWE_OK;
}

// Pinned host planes for state copies: three (eta, hu, hv), and three more
// for their rounding errors when the state is compensated.
int ensure_pinned_state(swe_domain *d)
{
    if (d->pinned_state) return SWE_OK;
    const size_t n = (size_t)(d->p.compensated_state ? 6 : 3) * d->p.nx * d->p.ny;
    HIP_TRY(hipHostMalloc((void **)&d->pinned_state, n * sizeof(float), hipHostMallocDefault));
    return SWE_OK;
}

// True for memory the device cannot address directly (plain pageable host
// memory): such destinations are filled through the pinned staging planes.
bool is_pageable(const void *p)
{
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return true;
    }
    return a.type == hipMemoryTypeUnregistered;
}

}  // namespace

extern "C" {

const char *swe_last_error(void) { return g_last_error.c_str(); }

int swe_workspace_bytes(const swe_params *p, int32_t max_wind_times, int32_t max_bnd_times, size_t *bytes)
{
    int rc = validate(p);
    if (rc) return rc;
    if (!bytes || max_wind_times < 1 || max_bnd_times < 0) return fail(SWE_E_ARG, "bad workspace query");
    *bytes = make_layout(*p, max_wind_times, max_bnd_times).total;
    return SWE_OK;
}

int swe_init_domain(const swe_params *p, void *dev_workspace, size_t bytes, void *hip_stream,
                    int32_t max_wind_times, int32_t max_bnd_times, const float *Hc, const uint8_t *land,
                    const float *f, const float *theta, const float *eta, const float *hu, const float *hv,
                    swe_domain **out)
{
    int rc = validate(p);
    if (rc) return rc;
    if (!out || !Hc || !f || !eta || !hu || !hv || !dev_workspace) return fail(SWE_E_ARG, "NULL array");
    if (max_wind_times < 1 || max_bnd_times < 0) return fail(SWE_E_ARG, "bad forcing bounds");
    if (any_nested(*p) && max_bnd_times < 1) return fail(SWE_E_ARG, "nested sides need max_bnd_times >= 1");
    if (((uintptr_t)dev_workspace) % kAlign) return fail(SWE_E_ARG, "workspace must be 256-byte aligned");
    *out = nullptr;
    const int nx = p->nx, ny = p->ny;
    const size_t nc = (size_t)nx * ny, nk = (size_t)(nx + 1) * (ny + 1);
    if (!all_finite(Hc, nk) || !all_finite(f, nc) || !all_finite(eta, nc) || !all_finite(hu, nc) ||
        !all_finite(hv, nc) || (theta && !all_finite(theta, nc)))
        return fail(SWE_E_ARG, "non-finite input");
    if (p->bc[0] == SWE_BC_PERIODIC)
        for (int j = 0; j <= ny; ++j)
            if (Hc[(size_t)j * (nx + 1)] != Hc[(size_t)j * (nx + 1) + nx])
                return fail(SWE_E_ARG, "periodic x: corner depths at x=0 and x=nx differ");
    if (p->bc[2] == SWE_BC_PERIODIC)
        for (int i = 0; i <= nx; ++i)
            if (Hc[i] != Hc[(size_t)ny * (nx + 1) + i])
                return fail(SWE_E_ARG, "periodic y: corner depths at y=0 and y=ny differ");
    Layout L = make_layout(*p, max_wind_times, max_bnd_times);
    if (bytes < L.total) return fail(SWE_E_NOMEM, "workspace too small");

    swe_domain *d = new (std::nothrow) swe_domain();
    if (!d) return fail(SWE_E_NOMEM, "host allocation failed");
    d->p = *p;
    d->stream = (hipStream_t)hip_stream;
    d->ws = (char *)dev_workspace;
    d->L = L;
    d->max_wind = max_wind_times;
    d->max_bnd = max_bnd_times;
    d->has_bnd = false;

    Dom &D = d->dom;
    D.nx = nx; D.ny = ny;
    D.pitch = pitch_of(frame_cols(nx));
    D.cpitch = pitch_of(frame_cols(nx) + 1);
    D.P = 2 * nx + 2 * ny;
    for (int k = 0; k < 4; ++k) D.bc[k] = p->bc[k];
    D.dx = (float)p->dx; D.dy = (float)p->dy;
    D.rdx = (float)(1.0 / p->dx); D.rdy = (float)(1.0 / p->dy);
    D.kx = (float)(p->dx / (2.0 * p->g)); D.ky = (float)(p->dy / (2.0 * p->g));
    D.g = (float)p->g; D.theta = (float)p->theta; D.kappa = (float)p->kappa;
    D.theta2 = (float)(2.0 * p->theta);
    D.grdx2 = (float)(0.5 * p->g / p->dx); D.grdy2 = (float)(0.5 * p->g / p->dy);
    D.inv2kappa = (float)(1.0 / (2.0 * p->kappa)); D.kappa_sq = (float)(p->kappa * p->kappa);
    D.courant_q = (float)(0.25 * p->courant);
    D.friction = p->friction;
    D.fric_c = p->friction == SWE_FRICTION_MANNING ? (float)(p->g * p->friction_coeff * p->friction_coeff)
                                                    : (float)p->friction_coeff;
    D.inv_rho_w = 1.0 / p->rho_w;
    D.g64 = p->g; D.kappa64 = p->kappa; D.dx64 = p->dx; D.dy64 = p->dy;
    D.frs_w = any_nested(*p) ? p->frs_width : 0;
    char *w = d->ws;
    D.eta = (float *)(w + L.eta); D.hu = (float *)(w + L.hu); D.hv = (float *)(w + L.hv);
    D.eta1 = (float *)(w + L.eta1); D.hu1 = (float *)(w + L.hu1); D.hv1 = (float *)(w + L.hv1);
    if (p->compensated_state) {
        D.eta_lo = (uint16_t *)(w + L.eta_lo); D.hu_lo = (uint16_t *)(w + L.hu_lo); D.hv_lo = (uint16_t *)(w + L.hv_lo);
        D.eta1_lo = (uint16_t *)(w + L.eta1_lo); D.hu1_lo = (uint16_t *)(w + L.hu1_lo);
        D.hv1_lo = (uint16_t *)(w + L.hv1_lo);
    }
    D.Hc = (const float *)(w + L.Hc);
    D.f = (const float *)(w + L.f);
    D.north = p->north_projection ? (const float *)(w + L.north) : nullptr;
    D.fghost = (const float *)(w + L.fghost);
    D.nghost = (const float *)(w + L.nghost);
    D.frs_alpha = (const float *)(w + L.alpha);
    D.nb = 0; D.bnd_t = (const double *)(w + L.bnd_t); D.bnd = (const float *)(w + L.bnd);
    D.nw = 0; D.wind_t = (const double *)(w + L.wind_t); D.wind = (const float *)(w + L.wind);
    D.ctrl = (Ctrl *)(w + L.ctrl);
    D.partials = (double *)(w + L.partials);
    {
        int dev = 0, cus = 256;
        if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        d->cus = cus > 0 ? cus : 256;
    }
    for (int st = 0; st < 2; ++st) {
        d->wps[st] = stage_waves_per_simd(st + 1, p->north_projection != 0, p->compensated_state != 0);
        d->T[st] = make_tiling(nx, ny, pick_rows_per_wave(nx, ny, d->cus, d->wps[st]));
    }

    hipStream_t s = d->stream;
    int r = SWE_OK;
    // f with land encoded as NaN
    std::vector<float> fl(f, f + nc);
    if (land)
        for (size_t k = 0; k < nc; ++k)
            if (land[k]) fl[k] = std::nanf("");
    std::vector<float> fg, ng, alpha(kMaxFrs, 0.f);
    build_ghost_table(*p, f, fg);
    build_ghost_table(*p, theta, ng);
    for (int k = 0; k < kMaxFrs; ++k) alpha[k] = (float)(1.0 - std::tanh((double)k / p->frs_d0));
    static const Ctrl c0{};
    hipError_t e;
    {
        Uploader up(s, (5 + (p->north_projection ? 1 : 0)) * (nk + 64 * (size_t)(ny + 1)) * sizeof(float));
        std::vector<float> th0;
        if (p->north_projection && !theta) th0.assign(nc, 0.f);
        // the planes start at zero (frames and padding columns included);
        // the interior cells and corners are uploaded at their frame origin
        auto org = [&](size_t off) { return w + off + (2 * (size_t)D.pitch + 2) * sizeof(float); };
        char *corg = w + L.Hc + (2 * (size_t)D.cpitch + 2) * sizeof(float);
        if ((e = hipMemsetAsync(w + L.eta, 0, L.fghost - L.eta, s)) ||
            (e = up.plane(org(L.eta), D.pitch, eta, nx, ny)) || (e = up.plane(org(L.hu), D.pitch, hu, nx, ny)) ||
            (e = up.plane(org(L.hv), D.pitch, hv, nx, ny)) || (e = up.plane(corg, D.cpitch, Hc, nx + 1, ny + 1)) ||
            (e = up.plane(org(L.f), D.pitch, fl.data(), nx, ny)) ||
            (p->north_projection && (e = up.plane(org(L.north), D.pitch, theta ? theta : th0.data(), nx, ny))) ||
            (e = up.flush())) {
            delete d;
            return hip_fail(e, "upload");
        }
    }
    if ((e = hipMemcpyAsync(w + L.fghost, fg.data(), fg.size() * sizeof(float), hipMemcpyHostToDevice, s)) ||
        (e = hipMemcpyAsync(w + L.nghost, ng.data(), ng.size() * sizeof(float), hipMemcpyHostToDevice, s)) ||
        (e = hipMemcpyAsync(w + L.alpha, alpha.data(), alpha.size() * sizeof(float), hipMemcpyHostToDevice, s)) ||
        (e = hipMemcpyAsync(w + L.ctrl, &c0, sizeof(Ctrl), hipMemcpyHostToDevice, s))) {
        delete d;
        return hip_fail(e, "upload");
    }
    // uniform zero wind until set
    double wt0 = 0.0;
    float w0[2] = {0.f, 0.f};
    if ((e = hipMemcpyAsync(w + L.wind_t, &wt0, sizeof(double), hipMemcpyHostToDevice, s)) ||
        (e = hipMemcpyAsync(w + L.wind, w0, sizeof(w0), hipMemcpyHostToDevice, s))) {
        delete d;
        return hip_fail(e, "upload");
    }
    D.nw = 1;
    if ((e = launch_frame_static(D, s)) != hipSuccess) { delete d; return hip_fail(e, "frames"); }
    if ((r = reset_time_and_cfl(d, 0.0)) || (r = copy_state_to_star(d))) { delete d; return r; }
    if ((e = hipStreamSynchronize(s)) != hipSuccess) { delete d; return hip_fail(e, "init sync"); }
    *out = d;
    return SWE_OK;
}

int swe_set_forcing(swe_domain *d, int32_t kind, int32_t n_times, const double *times, const float *data)
{
    if (!d || !times || !data || n_times < 1) return fail(SWE_E_ARG, "bad forcing arguments");
    if (d->ensemble) return fail(SWE_E_STATE, "domain belongs to an ensemble");
    for (int k = 0; k < n_times; ++k) {
        if (!std::isfinite(times[k])) return fail(SWE_E_ARG, "non-finite forcing time");
        if (k > 0 && !(times[k] > times[k - 1])) return fail(SWE_E_ARG, "forcing times must increase");
    }
    char *w = d->ws;
    hipStream_t s = d->stream;
    if (kind == SWE_FORCING_WIND_STRESS) {
        if (n_times > d->max_wind) return fail(SWE_E_ARG, "more wind snapshots than the workspace holds");
        if (!all_finite(data, 2 * (size_t)n_times)) return fail(SWE_E_ARG, "non-finite wind data");
        HIP_TRY(hipMemcpyAsync(w + d->L.wind_t, times, n_times * sizeof(double), hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(w + d->L.wind, data, 2 * (size_t)n_times * sizeof(float), hipMemcpyHostToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));
        d->dom.nw = n_times;
    } else if (kind == SWE_FORCING_BOUNDARY) {
        size_t n = (size_t)n_times * 3 * d->dom.P;
        if (n_times > d->max_bnd) return fail(SWE_E_ARG, "more boundary snapshots than the workspace holds");
        if (!all_finite(data, n)) return fail(SWE_E_ARG, "non-finite boundary data");
        HIP_TRY(hipMemcpyAsync(w + d->L.bnd_t, times, n_times * sizeof(double), hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(w + d->L.bnd, data, n * sizeof(float), hipMemcpyHostToDevice, s));
        d->dom.nb = n_times;
        d->has_bnd = true;
        // the nested ghosts of Q^n from the new boundary data
        HIP_TRY(launch_frame_state(d->dom, d->parity, s));
        HIP_TRY(hipStreamSynchronize(s));
    } else {
        return fail(SWE_E_ARG, "unknown forcing kind");
    }
    // kernel arguments changed: captured graphs are stale
    drop_graphs(d);
    return SWE_OK;
}

int swe_set_boundary_field(swe_domain *d, int32_t n_times, int32_t n_x, int32_t n_y, const double *times,
                           const float *data)
{
    if (!d || !times || !data || n_times < 1) return fail(SWE_E_ARG, "bad boundary-field arguments");
    if (n_x < 1 || n_y < 1 || n_x > (1 << 28) || n_y > (1 << 28)) return fail(SWE_E_ARG, "bad sample counts");
    if (n_times > d->max_bnd) return fail(SWE_E_ARG, "more boundary snapshots than the workspace holds");
    const int nx = d->p.nx, ny = d->p.ny, P = 2 * nx + 2 * ny, Q = 2 * n_y + 2 * n_x;
    if (!all_finite(data, (size_t)n_times * 3 * Q)) return fail(SWE_E_ARG, "non-finite boundary data");
    // one side's samples sit at the centres of n equal parts of the side; a
    // boundary cell takes the linear interpolation at its centre, clamped to
    // the end samples (what a texture fetch with linear filtering returns)
    auto side = [](const float *src, int n, float *dst, int m) {
        for (int j = 0; j < m; ++j) {
            double g = ((double)j + 0.5) * n / m - 0.5;
            g = std::min(std::max(g, 0.0), (double)(n - 1));
            int k0 = (int)g, k1 = std::min(k0 + 1, n - 1);
            double w = g - k0;
            dst[j] = (float)((1.0 - w) * src[k0] + w * src[k1]);
        }
    };
    std::vector<float> cells((size_t)n_times * 3 * P);
    for (int t = 0; t < n_times; ++t)
        for (int f = 0; f < 3; ++f) {
            const float *a = data + ((size_t)t * 3 + f) * Q;
            float *o = cells.data() + ((size_t)t * 3 + f) * P;
            side(a, n_y, o, ny);                        // West, by row
            side(a + n_y, n_y, o + ny, ny);             // East
            side(a + 2 * n_y, n_x, o + 2 * ny, nx);     // South, by column
            side(a + 2 * n_y + n_x, n_x, o + 2 * ny + nx, nx);  // North
        }
    return swe_set_forcing(d, SWE_FORCING_BOUNDARY, n_times, times, cells.data());
}

int swe_wind_field_bytes(int32_t n_times, int32_t nx_w, int32_t ny_w, size_t *bytes)
{
    if (!bytes || n_times < 1 || nx_w < 1 || ny_w < 1 || (int64_t)nx_w * ny_w > ((int64_t)1 << 26))
        return fail(SWE_E_ARG, "bad wind-field size");
    *bytes = align_up((size_t)n_times * sizeof(double), kAlign) + (size_t)n_times * nx_w * ny_w * 2 * sizeof(float);
    return SWE_OK;
}

namespace {

// Gridded wind (kind 0, with rho_air) or gridded stress (kind 1).
int set_field(swe_domain *d, int kind, int32_t n_times, int32_t nx_w, int32_t ny_w, const double *times,
              const float *w10, double rho_air, void *dev_buffer, size_t bytes)
{
    if (!d) return fail(SWE_E_ARG, "domain is NULL");
    if (d->ensemble) return fail(SWE_E_STATE, "domain belongs to an ensemble");
    if (n_times == 0) {
        d->dom.w10n = 0;
        drop_graphs(d);  // the graphs hold the domain block by value
        return SWE_OK;
    }
    size_t need = 0;
    int rc = swe_wind_field_bytes(n_times, nx_w, ny_w, &need);
    if (rc) return rc;
    if (!times || !w10 || !dev_buffer) return fail(SWE_E_ARG, "NULL argument");
    if (((uintptr_t)dev_buffer) % kAlign) return fail(SWE_E_ARG, "wind buffer must be 256-byte aligned");
    if (bytes < need) return fail(SWE_E_NOMEM, "wind buffer too small");
    if (!(std::isfinite(rho_air) && rho_air > 0)) return fail(SWE_E_ARG, "rho_air must be > 0");
    for (int k = 0; k < n_times; ++k) {
        if (!std::isfinite(times[k])) return fail(SWE_E_ARG, "non-finite wind time");
        if (k > 0 && !(times[k] > times[k - 1])) return fail(SWE_E_ARG, "wind times must increase");
    }
    const size_t nv = (size_t)n_times * nx_w * ny_w * 2;
    if (!all_finite(w10, nv)) return fail(SWE_E_ARG, "non-finite wind");
    char *b = (char *)dev_buffer;
    const size_t toff = align_up((size_t)n_times * sizeof(double), kAlign);
    HIP_TRY(hipMemcpyAsync(b, times, (size_t)n_times * sizeof(double), hipMemcpyHostToDevice, d->stream));
    {
        Uploader up(d->stream, nv * sizeof(float));
        hipError_t e;
        // rows of one sample line (nx_w (u, v) pairs), contiguous on the device
        if ((e = up.plane(b + toff, 2 * nx_w, w10, 2 * nx_w, n_times * ny_w)) || (e = up.flush()))
            return hip_fail(e, "wind upload");
    }
    Dom &D = d->dom;
    D.w10_t = (const double *)b;
    D.w10 = (const float *)(b + toff);
    D.w10nx = nx_w;
    D.w10ny = ny_w;
    D.w10sx = (float)((double)nx_w / d->p.nx);
    D.w10sy = (float)((double)ny_w / d->p.ny);
    D.w10q = (float)((kind == 0 ? rho_air : 1.0) / d->p.rho_w);
    D.w10_kind = kind;
    D.w10n = n_times;
    drop_graphs(d);  // the graphs hold the domain block by value
    return SWE_OK;
}

}  // namespace

int swe_set_wind_field(swe_domain *d, int32_t n_times, int32_t nx_w, int32_t ny_w, const double *times,
                       const float *w10, double rho_air, void *dev_buffer, size_t bytes)
{
    return set_field(d, 0, n_times, nx_w, ny_w, times, w10, rho_air, dev_buffer, bytes);
}

int swe_set_stress_field(swe_domain *d, int32_t n_times, int32_t nx_w, int32_t ny_w, const double *times,
                         const float *tau, void *dev_buffer, size_t bytes)
{
    return set_field(d, 1, n_times, nx_w, ny_w, times, tau, 1.0, dev_buffer, bytes);
}

int swe_step(swe_domain *d, int32_t n_steps)
{
    int rc = check_ready(d);
    if (rc) return rc;
    if (n_steps < 0) return fail(SWE_E_ARG, "n_steps < 0");
    int left = n_steps;
    if (!d->timing) {
        // whole chunks, then the remainder, each through a graph captured on
        // its first use and kept per (steps, parity): at most 2 x 16 graphs
        while (left > 0) {
            const int n = left >= kGraphChunk ? kGraphChunk : left;
            hipGraphExec_t g;
            if ((rc = get_graph(d, n, d->parity, &g))) return rc;
            HIP_TRY(hipGraphLaunch(g, d->stream));
            d->parity = (d->parity + n) & 1;
            left -= n;
        }
    }
    for (; left > 0; --left) {
        if ((rc = launch_step(d, d->parity, 0.0, d->stream, d->timing))) return rc;
        d->parity ^= 1;
    }
    return SWE_OK;
}

int swe_step_dt(swe_domain *d, int32_t n_steps, const double *dts)
{
    int rc = check_ready(d);
    if (rc) return rc;
    if (n_steps < 0 || (n_steps > 0 && !dts)) return fail(SWE_E_ARG, "bad dt sequence");
    for (int k = 0; k < n_steps; ++k)
        if (!(std::isfinite(dts[k]) && dts[k] > 0)) return fail(SWE_E_ARG, "dt must be finite and > 0");
    for (int k = 0; k < n_steps; ++k) {
        if ((rc = launch_step(d, d->parity, dts[k], d->stream, d->timing))) return rc;
        d->parity ^= 1;
    }
    return SWE_OK;
}

int swe_run_until(swe_domain *d, double t_end, int64_t *steps_taken)
{
    int rc = check_ready(d);
    if (rc) return rc;
    if (!std::isfinite(t_end)) return fail(SWE_E_ARG, "t_end must be finite");
    Ctrl c;
    if ((rc = read_ctrl(d, &c))) return rc;
    int64_t s0 = c.steps;
    double t = c.t[d->parity];
    if (t_end > t) {
        HIP_TRY(launch_set_t_end(d->dom.ctrl, t_end, d->stream));
        // estimate the remaining steps from the current dt, then check
        const int chunk_max = 4096;
        while (true) {
            if ((rc = read_ctrl(d, &c))) break;
            t = c.t[d->parity];
            if (c.flags) break;
            if (t >= t_end) break;
            double dt = ctrl_next_dt(c, d->parity, d->dom.courant_q, d->dom.dt_interval);
            if (!std::isfinite(dt)) dt = 1.0;
            double est = (t_end - t) / dt;
            int n = (int)std::min<double>(chunk_max, std::max<double>(kGraphChunk, std::ceil(est * 1.05) + 1));
            if ((rc = swe_step(d, n))) break;
        }
        HIP_TRY(launch_set_t_end(d->dom.ctrl, 0.0, d->stream));
        if (rc) return rc;
    }
    if ((rc = read_ctrl(d, &c))) return rc;
    if (steps_taken) *steps_taken = c.steps - s0;
    if (c.flags) return fail(SWE_E_UNSTABLE, flag_message(c.flags));
    return SWE_OK;
}

int swe_read_state(swe_domain *d, float *eta, float *hu, float *hv, double *t, double *dt_next)
{
    if (!d) return fail(SWE_E_ARG, "domain is NULL");
    const int nx = d->p.nx, ny = d->p.ny;
    float *dst[3] = {eta, hu, hv};
    const size_t org = 2 * (size_t)d->dom.pitch + 2;  // cell (0, 0) of a framed plane
    float *src[3] = {d->dom.eta + org, d->dom.hu + org, d->dom.hv + org};
    const size_t plane = (size_t)nx * ny;
    bool staged[3] = {false, false, false};
    for (int k = 0; k < 3; ++k) {
        if (!dst[k]) continue;
        float *to = dst[k];
        if (is_pageable(dst[k])) {
            int rc0 = ensure_pinned_state(d);
            if (rc0) return rc0;
            to = d->pinned_state + k * plane;
            staged[k] = true;
        }
        HIP_TRY(hipMemcpy2DAsync(to, (size_t)nx * sizeof(float), src[k], (size_t)d->dom.pitch * sizeof(float),
                                 (size_t)nx * sizeof(float), (size_t)ny, hipMemcpyDefault, d->stream));
    }
    Ctrl c;
    int rc = read_ctrl(d, &c);  // also waits for the copies above
    if (rc) return rc;
    for (int k = 0; k < 3; ++k)
        if (staged[k]) std::memcpy(dst[k], d->pinned_state + k * plane, plane * sizeof(float));
    if (t) *t = c.t[d->parity];
    if (dt_next) *dt_next = ctrl_next_dt(c, d->parity, d->dom.courant_q, d->dom.dt_interval);
    if (c.flags) return fail(SWE_E_UNSTABLE, flag_message(c.flags));
    return SWE_OK;
}

int swe_set_dt_policy(swe_domain *d, double interval)
{
    if (!d) return fail(SWE_E_ARG, "domain is NULL");
    if (!(std::isfinite(interval) && interval >= 0.0)) return fail(SWE_E_ARG, "interval must be finite and >= 0");
    if (d->ensemble) return fail(SWE_E_STATE, "domain belongs to an ensemble");
    d->dom.dt_interval = interval;
    drop_graphs(d);  // the graphs hold the domain block by value
    HIP_TRY(launch_policy_reset(d->dom.ctrl, d->parity, d->stream));
    HIP_TRY(hipStreamSynchronize(d->stream));
    return SWE_OK;
}

int swe_set_state(swe_domain *d, const float *eta, const float *hu, const float *hv, double t)
{
    if (!d || !eta || !hu || !hv) return fail(SWE_E_ARG, "NULL argument");
    if (d->ensemble) return fail(SWE_E_STATE, "domain belongs to an ensemble");
    const int nx = d->p.nx, ny = d->p.ny;
    size_t nc = (size_t)nx * ny;
    if (!std::isfinite(t) || !all_finite(eta, nc) || !all_finite(hu, nc) || !all_finite(hv, nc))
        return fail(SWE_E_ARG, "non-finite state");
    int rc;
    {
        Uploader up(d->stream, 3 * nc * sizeof(float));
        hipError_t e;
        const size_t org = 2 * (size_t)d->dom.pitch + 2;
        if ((e = up.plane(d->dom.eta + org, d->dom.pitch, eta, nx, ny)) ||
            (e = up.plane(d->dom.hu + org, d->dom.pitch, hu, nx, ny)) ||
            (e = up.plane(d->dom.hv + org, d->dom.pitch, hv, nx, ny)) || (e = up.flush()))
            return hip_fail(e, "upload");
    }
    if ((rc = reset_time_and_cfl(d, t)) ||
        (rc = copy_state_to_star(d)))
        return rc;
    HIP_TRY(hipStreamSynchronize(d->stream));
    return SWE_OK;
}

int swe_diagnostics(swe_domain *d, double *mass, double *energy)
{
    if (!d) return fail(SWE_E_ARG, "domain is NULL");
    HIP_TRY(launch_diagnostics(d->dom, d->stream));
    Ctrl c;
    int rc = read_ctrl(d, &c);
    if (rc) return rc;
    if (mass) *mass = c.mass;
    if (energy) *energy = c.energy;
    return SWE_OK;
}

int swe_status(swe_domain *d)
{
    if (!d) return fail(SWE_E_ARG, "domain is NULL");
    Ctrl c;
    int rc = read_ctrl(d, &c);
    if (rc) return rc;
    return c.flags ? fail(SWE_E_UNSTABLE, flag_message(c.flags)) : SWE_OK;
}

int swe_set_tiling(swe_domain *d, int32_t rows_per_wave, int32_t order)
{
    if (!d) return fail(SWE_E_ARG, "domain is NULL");
    if (d->ensemble) return fail(SWE_E_STATE, "domain belongs to an ensemble");
    if (rows_per_wave < 0 || rows_per_wave > 4096) return fail(SWE_E_ARG, "rows_per_wave out of range");
    if (order < -1 || order > 3) return fail(SWE_E_ARG, "order must be -1 (default) or 0..3");
    for (int st = 0; st < 2; ++st) {
        int by = rows_per_wave ? rows_per_wave : pick_rows_per_wave(d->p.nx, d->p.ny, d->cus, d->wps[st]);
        d->T[st] = make_tiling(d->p.nx, d->p.ny, by);
        if (order >= 0) d->T[st].order = order;
    }
    drop_graphs(d);
    return SWE_OK;
}

int swe_set_stage_tiling(swe_domain *d, int32_t stage, int32_t rows_per_wave, int32_t tail_rows_per_wave,
                         int32_t tail_rows, int32_t order)
{
    if (!d) return fail(SWE_E_ARG, "domain is NULL");
    if (d->ensemble) return fail(SWE_E_STATE, "domain belongs to an ensemble");
    if (stage != 1 && stage != 2) return fail(SWE_E_ARG, "stage must be 1 or 2");
    if (rows_per_wave < 1 || rows_per_wave > 4096) return fail(SWE_E_ARG, "rows_per_wave must be in [1, 4096]");
    if (tail_rows_per_wave < 0 || tail_rows_per_wave > 4096 || tail_rows < 0)
        return fail(SWE_E_ARG, "tail_rows_per_wave must be in [0, 4096] and tail_rows >= 0");
    if (order < -1 || order > 3) return fail(SWE_E_ARG, "order must be -1 (default) or 0..3");
    Tiling &T = d->T[stage - 1];
    const int o = order >= 0 ? order : T.order;
    T = make_tiling_tail(d->p.nx, d->p.ny, rows_per_wave, tail_rows_per_wave, tail_rows);
    T.order = o;
    drop_graphs(d);
    return SWE_OK;
}

int swe_get_stage_tiling(swe_domain *d, int32_t stage, int32_t *rows_per_wave, int32_t *tail_rows_per_wave,
                         int32_t *tail_rows, int32_t *order, int32_t *waves)
{
    if (!d) return fail(SWE_E_ARG, "domain is NULL");
    if (stage != 1 && stage != 2) return fail(SWE_E_ARG, "stage must be 1 or 2");
    const Tiling &T = d->T[stage - 1];
    const bool two = T.nrb1 < T.nrb;
    if (rows_per_wave) *rows_per_wave = T.by;
    if (tail_rows_per_wave) *tail_rows_per_wave = two ? T.by2 : 0;
    if (tail_rows) *tail_rows = two ? d->p.ny - T.nrb1 * T.by : 0;
    if (order) *order = T.order;
    if (waves) *waves = T.ntiles;
    return SWE_OK;
}

// Median-based time of one stage kernel under tiling T (one warm-up and
// eight event-timed launches, the middle two summed, so that a disturbed
// launch does not decide).  Each launch follows one of the other stage
// kernel (untimed, under its tiling `other`), as in a step: what that kernel
// leaves in the caches, and the state it writes, are what the timed one
// starts from.
struct StageTimer {
    static constexpr int kReps = 8;
    hipEvent_t ev[2 * kReps] = {};
    int made = 0;
    ~StageTimer() { for (int k = 0; k < made; ++k) (void)hipEventDestroy(ev[k]); }
    hipError_t init()
    {
        for (; made < 2 * kReps; ++made) {
            hipError_t e = hipEventCreate(&ev[made]);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    hipError_t time(swe_domain *d, int stage, const Tiling &T, const Tiling &other, float *out)
    {
        const bool proj = d->p.north_projection != 0;
        const int ostage = 3 - stage;
        hipError_t he = launch_stage(ostage, proj, d->dom, other, d->parity, 0.0, d->stream, nullptr, nullptr);
        if (he == hipSuccess) he = launch_stage(stage, proj, d->dom, T, d->parity, 0.0, d->stream, nullptr, nullptr);
        for (int k = 0; k < kReps && he == hipSuccess; ++k) {
            he = launch_stage(ostage, proj, d->dom, other, d->parity, 0.0, d->stream, nullptr, nullptr);
            if (he == hipSuccess)
                he = launch_stage(stage, proj, d->dom, T, d->parity, 0.0, d->stream, ev[2 * k], ev[2 * k + 1]);
        }
        if (he != hipSuccess || (he = hipStreamSynchronize(d->stream)) != hipSuccess) return he;
        float ms[kReps];
        for (int k = 0; k < kReps && he == hipSuccess; ++k) {
            ms[k] = 0.f;
            he = hipEventElapsedTime(&ms[k], ev[2 * k], ev[2 * k + 1]);
        }
        if (he != hipSuccess) return he;
        std::sort(ms, ms + kReps);
        *out = ms[kReps / 2 - 1] + ms[kReps / 2];
        return hipSuccess;
    }
};

// Band heights the sweep tries.
constexpr int kTileHeights[] = {2, 3, 4, 5, 6, 7, 8, 10, 12, 14, 16, 20, 24, 32, 48, 64};
constexpr int kNumTileHeights = sizeof(kTileHeights) / sizeof(kTileHeights[0]);

// The tail tilings the sweep tries with head bands of `by` rows: tails of
// 1..4-row bands holding about a quarter, a half, one or two rounds of the
// stage kernel's resident wave slots; duplicates dropped.
void tail_candidates(const swe_domain *d, int stage, int by, std::vector<Tiling> &out)
{
    const int nx = d->p.nx, ny = d->p.ny;
    const double slots = (double)d->cus * 4 * d->wps[stage - 1];
    const int nstrips = (nx + kStrip - 1) / kStrip;
    const size_t first = out.size();
    for (int by2 = 1; by2 <= 4 && by2 < by; ++by2) {
        for (double rounds : {0.25, 0.5, 1.0, 2.0}) {
            const int bands = (int)std::lround(rounds * slots / nstrips);
            const int tail = std::max(1, bands) * by2;
            if (tail + by > ny) continue;
            const Tiling T = make_tiling_tail(nx, ny, by, by2, tail);
            if (T.nrb1 == T.nrb) continue;
            bool dup = false;
            for (size_t k = first; k < out.size(); ++k) dup |= out[k].by2 == T.by2 && out[k].nrb1 == T.nrb1;
            if (!dup) out.push_back(T);
        }
    }
}

// Time one stage kernel over candidate tilings and return the fastest: first
// one band height for the whole domain (2 .. 64 rows), then the tails of
// tail_candidates around the best height and the next two taller ones, then
// the other tile numberings of the winner.  A candidate replaces the
// incumbent only when it is more than 1 % faster.  Last, the three fastest
// candidates seen are timed again, twice each, and the best of those
// measurements wins (one timing of eight launches can be off by a few per
// cent).
int sweep_stage(swe_domain *d, int stage, const Tiling &other, Tiling *best_T)
{
    const int nx = d->p.nx, ny = d->p.ny;
    StageTimer tm;
    hipError_t he = tm.init();
    Tiling best = d->T[stage - 1];
    float best_ms = INFINITY;
    int best_k = -1;
    std::vector<std::pair<float, Tiling>> seen;
    auto time_one = [&](const Tiling &T, float *ms) {
        hipError_t e = tm.time(d, stage, T, other, ms);
        if (e == hipSuccess) seen.push_back({*ms, T});
        return e;
    };
    for (int k = 0; k < kNumTileHeights && he == hipSuccess; ++k) {
        if (kTileHeights[k] > ny && k != 0) break;
        const Tiling T = make_tiling(nx, ny, kTileHeights[k]);
        float ms = 0.f;
        if ((he = time_one(T, &ms)) != hipSuccess) break;
        if (ms < best_ms * 0.99f) { best_ms = ms; best = T; best_k = k; }
    }
    std::vector<Tiling> tails;
    for (int k = best_k; k >= 0 && k < best_k + 3 && k < kNumTileHeights; ++k)
        tail_candidates(d, stage, kTileHeights[k], tails);
    for (size_t k = 0; k < tails.size() && he == hipSuccess; ++k) {
        float ms = 0.f;
        if ((he = time_one(tails[k], &ms)) != hipSuccess) break;
        if (ms < best_ms * 0.99f) { best_ms = ms; best = tails[k]; }
    }
    // the tile numbering of the winner: row-band-major keeps the rows that
    // the resident waves touch close together (fewer pages in flight on
    // large domains); without per-XCD grouping as a control
    const Tiling won = best;
    for (int order = 1; order <= 3 && he == hipSuccess; ++order) {
        Tiling T = won;
        T.order = order;
        float ms = 0.f;
        if ((he = time_one(T, &ms)) != hipSuccess) break;
        if (ms < best_ms * 0.99f) { best_ms = ms; best = T; }
    }
    // confirmation round over the three fastest candidates
    if (he == hipSuccess && seen.size() > 1) {
        std::stable_sort(seen.begin(), seen.end(),
                         [](const std::pair<float, Tiling> &a, const std::pair<float, Tiling> &b) { return a.first < b.first; });
        float conf_best = INFINITY;
        for (size_t k = 0; k < seen.size() && k < 3 && he == hipSuccess; ++k)
            for (int rep = 0; rep < 2 && he == hipSuccess; ++rep) {
                float ms = 0.f;
                if ((he = tm.time(d, stage, seen[k].second, other, &ms)) != hipSuccess) break;
                if (ms < conf_best) { conf_best = ms; best = seen[k].second; }
            }
    }
    if (he != hipSuccess) return hip_fail(he, "tiling sweep");
    *best_T = best;
    return SWE_OK;
}

// Brings the device's clocks up before tilings are compared: stage-1
// launches at the current tiling until about 25 ms of device time (at most
// 2000 launches) have passed.
hipError_t settle_clocks(swe_domain *d)
{
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t he = hipEventCreate(&a);
    if (he == hipSuccess) he = hipEventCreate(&b);
    const bool proj = d->p.north_projection != 0;
    float total = 0.f;
    for (int launches = 0; he == hipSuccess && total < 25.f && launches < 2000;) {
        he = hipEventRecord(a, d->stream);
        for (int k = 0; k < 20 && he == hipSuccess; ++k, ++launches)
            he = launch_stage(1, proj, d->dom, d->T[0], d->parity, 0.0, d->stream, nullptr, nullptr);
        if (he == hipSuccess) he = hipEventRecord(b, d->stream);
        if (he == hipSuccess) he = hipEventSynchronize(b);
        float ms = 0.f;
        if (he == hipSuccess) he = hipEventElapsedTime(&ms, a, b);
        total += ms;
    }
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    return he;
}

int swe_list_tilings(swe_domain *d, int32_t stage, int32_t *out, int32_t max_tilings, int32_t *n_tilings)
{
    if (!d) return fail(SWE_E_ARG, "domain is NULL");
    if (stage != 1 && stage != 2) return fail(SWE_E_ARG, "stage must be 1 or 2");
    if (max_tilings < 0 || (max_tilings > 0 && !out)) return fail(SWE_E_ARG, "bad output array");
    std::vector<Tiling> all;
    for (int k = 0; k < kNumTileHeights; ++k) {
        if (kTileHeights[k] > d->p.ny && k != 0) break;
        all.push_back(make_tiling(d->p.nx, d->p.ny, kTileHeights[k]));
    }
    const size_t uniform = all.size();
    for (size_t k = 0; k < uniform; ++k) tail_candidates(d, stage, all[k].by, all);
    for (size_t k = 0; k < all.size() && (int)k < max_tilings; ++k) {
        const bool two = all[k].nrb1 < all[k].nrb;
        out[3 * k] = all[k].by;
        out[3 * k + 1] = two ? all[k].by2 : 0;
        out[3 * k + 2] = two ? d->p.ny - all[k].nrb1 * all[k].by : 0;
    }
    if (n_tilings) *n_tilings = (int32_t)all.size();
    return SWE_OK;
}

int swe_autotune_tiling(swe_domain *d, int32_t *rows_per_wave)
{
    int rc = check_ready(d);
    if (rc) return rc;
    // Stage 1 writes only Q*, which every step overwrites; stage 2 writes
    // Q^{n+1} over Q^n.  Q^n (with its rounding errors when compensated) and
    // the control block (time, step count, CFL slots) are saved first and put
    // back afterwards, so the sweep leaves the simulation where it was.
    Ctrl saved;
    if ((rc = read_ctrl(d, &saved))) return rc;
    const int nx = d->p.nx, ny = d->p.ny;
    const size_t plane = (size_t)nx * ny;
    if ((rc = ensure_pinned_state(d))) return rc;
    // the three value planes (float32) and the three rounding-error planes
    // (16 bits), from cell (0, 0) of each framed plane; the state frame is
    // rebuilt afterwards
    const size_t org = 2 * (size_t)d->dom.pitch + 2;
    void *q[6] = {d->dom.eta + org, d->dom.hu + org, d->dom.hv + org, d->dom.eta_lo ? d->dom.eta_lo + org : nullptr,
                  d->dom.hu_lo ? d->dom.hu_lo + org : nullptr, d->dom.hv_lo ? d->dom.hv_lo + org : nullptr};
    const int nq = d->p.compensated_state ? 6 : 3;
    auto esz = [](int k) { return k < 3 ? sizeof(float) : sizeof(uint16_t); };
    for (int k = 0; k < nq; ++k)
        HIP_TRY(hipMemcpy2DAsync(d->pinned_state + k * plane, nx * esz(k), q[k], d->dom.pitch * esz(k), nx * esz(k),
                                 ny, hipMemcpyDeviceToHost, d->stream));
    Tiling T1 = d->T[0], T2 = d->T[1];
    hipError_t se = settle_clocks(d);
    // stage 1 between launches of the stage-2 kernel's current tiling, then
    // stage 2 between launches of the stage-1 tiling just found
    rc = se != hipSuccess ? hip_fail(se, "settle_clocks") : sweep_stage(d, 1, T2, &T1);
    if (!rc) rc = sweep_stage(d, 2, T1, &T2);
    // the state and control block go back even when the sweep failed
    for (int k = 0; k < nq; ++k)
        HIP_TRY(hipMemcpy2DAsync(q[k], d->dom.pitch * esz(k), d->pinned_state + k * plane, nx * esz(k), nx * esz(k),
                                 ny, hipMemcpyHostToDevice, d->stream));
    HIP_TRY(hipMemcpyAsync(d->dom.ctrl, &saved, sizeof(Ctrl), hipMemcpyHostToDevice, d->stream));
    HIP_TRY(launch_frame_state(d->dom, d->parity, d->stream));
    HIP_TRY(hipStreamSynchronize(d->stream));
    if (rc) return rc;
    d->T[0] = T1;
    d->T[1] = T2;
    drop_graphs(d);
    if (rows_per_wave) *rows_per_wave = T1.by;
    return SWE_OK;
}

int swe_get_tiling(swe_domain *d, int32_t stage, int32_t *rows_per_wave, int32_t *order, int32_t *waves)
{
    if (!d) return fail(SWE_E_ARG, "domain is NULL");
    if (stage != 1 && stage != 2) return fail(SWE_E_ARG, "stage must be 1 or 2");
    const Tiling &T = d->T[stage - 1];
    if (rows_per_wave) *rows_per_wave = T.by;
    if (order) *order = T.order;
    if (waves) *waves = T.ntiles;
    return SWE_OK;
}

int swe_enable_timing(swe_domain *d, int32_t on)
{
    if (!d) return fail(SWE_E_ARG, "domain is NULL");
    d->timing = on != 0;
    return SWE_OK;
}

int swe_stage_times(swe_domain *d, double *ms_stage1, double *ms_stage2, int64_t *launches, int32_t reset)
{
    if (!d) return fail(SWE_E_ARG, "domain is NULL");
    HIP_TRY(hipStreamSynchronize(d->stream));
    double a = 0, b = 0;
    for (size_t k = 0; k + 3 < d->ev_used; k += 4) {
        float x = 0, y = 0;
        HIP_TRY(hipEventElapsedTime(&x, d->ev_pool[k], d->ev_pool[k + 1]));
        HIP_TRY(hipEventElapsedTime(&y, d->ev_pool[k + 2], d->ev_pool[k + 3]));
        a += x;
        b += y;
    }
    int64_t n = d->timed_steps;
    if (ms_stage1) *ms_stage1 = n ? a / n : 0.0;
    if (ms_stage2) *ms_stage2 = n ? b / n : 0.0;
    if (launches) *launches = n;
    if (reset) {
        d->ev_used = 0;
        d->timed_steps = 0;
    }
    return SWE_OK;
}

void swe_destroy(swe_domain *d)
{
    if (!d) return;
    (void)hipStreamSynchronize(d->stream);  // NULL: the null stream
    if (d->ensemble) ensemble_forget(d->ensemble, d);
    for (auto &kv : d->graphs) (void)hipGraphExecDestroy(kv.second);
    for (auto g : d->graph_objs) (void)hipGraphDestroy(g);
    for (auto e : d->ev_pool) (void)hipEventDestroy(e);
    if (d->capture_stream) (void)hipStreamDestroy(d->capture_stream);
    if (d->pinned_ctrl) (void)hipHostFree(d->pinned_ctrl);
    if (d->pinned_state) (void)hipHostFree(d->pinned_state);
    delete d;
}

}  // extern "C"
