// Host side of the batched ensemble (include/swe.h): member table, device
// work queue, persistent stage launches, HIP-graph replay, timing.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "swe_host.h"

using namespace swe;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

#define EHIP(expr)                                                                           \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess) return set_error(SWE_E_HIP, std::string(#expr ": ") + hipGetErrorString(e_)); \
    } while (0)

constexpr int kEnsGraphChunk = 16;
constexpr int kDefaultRows = 16;
// One item per atomic: the items of a member differ little in cost, and
// taking several at once leaves the last waves of a launch with uneven
// loads (measured on 128 served-size domains: 2.8e10 cell-updates/s with 1,
// 2.0e10 with 4).
constexpr int kDefaultChunk = 1;

struct EnsLayout {
    size_t mem, items, ctrl, total;
};

int64_t count_items(swe_domain *const *m, int n, int by)
{
    int64_t t = 0;
    for (int k = 0; k < n; ++k) t += make_tiling(m[k]->p.nx, m[k]->p.ny, by).ntiles;
    return t;
}

EnsLayout ens_layout(int n, int64_t items)
{
    EnsLayout L;
    size_t off = 0;
    auto take = [&](size_t b) { size_t o = off; off = align_up(off + b, kAlign); return o; };
    L.mem = take(sizeof(EnsMember) * (size_t)n);
    L.items = take(sizeof(EnsItem) * (size_t)items);
    L.ctrl = take(sizeof(EnsCtrl));
    L.total = off;
    return L;
}

}  // namespace

size_t swe::ensemble_bytes_for_shapes(const std::vector<std::pair<int, int>> &shapes, int rows_per_wave)
{
    int by = rows_per_wave ? rows_per_wave : kDefaultRows;
    int64_t t = 0;
    for (auto &sh : shapes) t += make_tiling(sh.first, sh.second, by).ntiles;
    return ens_layout((int)shapes.size(), t).total;
}

struct swe_ensemble {
    std::vector<swe_domain *> members;
    hipStream_t stream = nullptr;
    hipStream_t capture_stream = nullptr;
    char *ws = nullptr;
    EnsLayout L{};
    EnsMember *d_mem = nullptr;
    EnsItem *d_items = nullptr;
    EnsCtrl *d_ctrl = nullptr;
    int64_t nitems = 0;
    int by = kDefaultRows;
    int chunk = kDefaultChunk;
    int nblocks = 0;
    int parity = 0;
    bool proj = false;
    bool w10 = false;  // some member has a gridded wind field
    bool comp = false; // members keep a compensated state
    std::map<std::pair<int, int>, hipGraphExec_t> graphs;
    std::vector<hipGraph_t> graph_objs;
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    int64_t timed_steps = 0;
    bool broken = false;  // a member was destroyed first
    bool use_graphs = true;
};

void swe::ensemble_forget(swe_ensemble *e, swe_domain *d)
{
    for (auto &m : e->members)
        if (m == d) m = nullptr;
    e->broken = true;
}

namespace {

int launch_ens_step(swe_ensemble *e, int parity, hipStream_t s, bool timed)
{
    if (timed) {
        while (e->ev_pool.size() < e->ev_used + 4) {
            hipEvent_t ev;
            EHIP(hipEventCreate(&ev));
            e->ev_pool.push_back(ev);
        }
        hipEvent_t *pe = &e->ev_pool[e->ev_used];
        EHIP(launch_ensemble(1, e->proj, e->w10, e->comp, e->d_mem, e->d_items, e->d_ctrl, parity, e->chunk, e->nblocks, s, pe[0], pe[1]));
        EHIP(launch_ensemble(2, e->proj, e->w10, e->comp, e->d_mem, e->d_items, e->d_ctrl, parity, e->chunk, e->nblocks, s, pe[2], pe[3]));
        e->ev_used += 4;
        e->timed_steps += 1;
        return SWE_OK;
    }
    EHIP(launch_ensemble(1, e->proj, e->w10, e->comp, e->d_mem, e->d_items, e->d_ctrl, parity, e->chunk, e->nblocks, s, nullptr, nullptr));
    EHIP(launch_ensemble(2, e->proj, e->w10, e->comp, e->d_mem, e->d_items, e->d_ctrl, parity, e->chunk, e->nblocks, s, nullptr, nullptr));
    return SWE_OK;
}

int ens_graph(swe_ensemble *e, int steps, int parity, hipGraphExec_t *out)
{
    auto key = std::make_pair(steps, parity);
    auto it = e->graphs.find(key);
    if (it != e->graphs.end()) { *out = it->second; return SWE_OK; }
    if (!e->capture_stream) EHIP(hipStreamCreateWithFlags(&e->capture_stream, hipStreamNonBlocking));
    EHIP(hipStreamBeginCapture(e->capture_stream, hipStreamCaptureModeThreadLocal));
    int rc = SWE_OK;
    for (int k = 0; k < steps && rc == SWE_OK; ++k) rc = launch_ens_step(e, (parity + k) & 1, e->capture_stream, false);
    hipGraph_t g = nullptr;
    hipError_t he = hipStreamEndCapture(e->capture_stream, &g);
    if (rc != SWE_OK) { if (g) (void)hipGraphDestroy(g); return rc; }
    if (he != hipSuccess) return set_error(SWE_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(he));
    hipGraphExec_t ex = nullptr;
    he = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (he != hipSuccess) { (void)hipGraphDestroy(g); return set_error(SWE_E_HIP, "hipGraphInstantiate failed"); }
    e->graph_objs.push_back(g);
    e->graphs[key] = ex;
    *out = ex;
    return SWE_OK;
}

int check_members(swe_domain *const *m, int n)
{
    if (!m || n < 1) return set_error(SWE_E_ARG, "an ensemble needs at least one member");
    for (int k = 0; k < n; ++k) {
        if (!m[k]) return set_error(SWE_E_ARG, "NULL member");
        if (m[k]->ensemble) return set_error(SWE_E_STATE, "member already belongs to an ensemble");
        for (int j = 0; j < k; ++j)
            if (m[j] == m[k]) return set_error(SWE_E_ARG, "member listed twice");
        if (m[k]->p.north_projection != m[0]->p.north_projection)
            return set_error(SWE_E_ARG, "members must share north_projection");
        if (m[k]->p.compensated_state != m[0]->p.compensated_state)
            return set_error(SWE_E_ARG, "members must share compensated_state");
        bool nested = false;
        for (int s = 0; s < 4; ++s) nested |= m[k]->p.bc[s] == SWE_BC_NESTED;
        if (nested && !m[k]->has_bnd) return set_error(SWE_E_STATE, "nested member without boundary data");
    }
    return SWE_OK;
}

}  // namespace

extern "C" {

int swe_ensemble_workspace_bytes(swe_domain *const *members, int32_t n, int32_t rows_per_wave, size_t *bytes)
{
    if (!bytes || rows_per_wave < 0 || rows_per_wave > 4096) return set_error(SWE_E_ARG, "bad arguments");
    if (!members || n < 1) return set_error(SWE_E_ARG, "an ensemble needs at least one member");
    for (int k = 0; k < n; ++k)
        if (!members[k]) return set_error(SWE_E_ARG, "NULL member");
    int by = rows_per_wave ? rows_per_wave : kDefaultRows;
    *bytes = ens_layout(n, count_items(members, n, by)).total;
    return SWE_OK;
}

int swe_ensemble_create(swe_domain *const *members, int32_t n, void *dev_workspace, size_t bytes, void *hip_stream,
                        int32_t rows_per_wave, int32_t chunk, swe_ensemble **out)
{
    int rc = check_members(members, n);
    if (rc) return rc;
    if (!out || !dev_workspace || rows_per_wave < 0 || rows_per_wave > 4096 || chunk < 0 || chunk > 1024)
        return set_error(SWE_E_ARG, "bad arguments");
    if (((uintptr_t)dev_workspace) % kAlign) return set_error(SWE_E_ARG, "workspace must be 256-byte aligned");
    int by = rows_per_wave ? rows_per_wave : kDefaultRows;
    int64_t nitems = count_items(members, n, by);
    if (nitems > (int64_t)1 << 31) return set_error(SWE_E_ARG, "too many work items");
    EnsLayout L = ens_layout(n, nitems);
    if (bytes < L.total) return set_error(SWE_E_NOMEM, "ensemble workspace too small");

    swe_ensemble *e = new (std::nothrow) swe_ensemble();
    if (!e) return set_error(SWE_E_NOMEM, "host allocation failed");
    e->members.assign(members, members + n);
    e->stream = (hipStream_t)hip_stream;
    e->ws = (char *)dev_workspace;
    e->L = L;
    e->d_mem = (EnsMember *)(e->ws + L.mem);
    e->d_items = (EnsItem *)(e->ws + L.items);
    e->d_ctrl = (EnsCtrl *)(e->ws + L.ctrl);
    e->nitems = nitems;
    e->by = by;
    e->chunk = chunk ? chunk : kDefaultChunk;
    e->proj = members[0]->p.north_projection != 0;
    e->comp = members[0]->p.compensated_state != 0;
    for (int k = 0; k < n; ++k) e->w10 |= members[k]->dom.w10n > 0;
    int w1 = ensemble_waves_per_simd(1, e->proj, e->comp), w2 = ensemble_waves_per_simd(2, e->proj, e->comp);
    e->nblocks = members[0]->cus * std::min(w1, w2);  // one wave per SIMD per block
    e->nblocks = (e->nblocks + kEnsParts - 1) / kEnsParts * kEnsParts;

    // member table
    std::vector<EnsMember> hm(n);
    for (int k = 0; k < n; ++k) {
        std::memset(&hm[k], 0, sizeof(EnsMember));
        hm[k].d = members[k]->dom;
        hm[k].T = make_tiling(members[k]->p.nx, members[k]->p.ny, by);
        hm[k].pflip = members[k]->parity;
    }
    // work queue: members by size, largest first; item j -> partition j % 8
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return (int64_t)members[a]->p.nx * members[a]->p.ny > (int64_t)members[b]->p.nx * members[b]->p.ny;
    });
    std::vector<std::vector<EnsItem>> parts(kEnsParts);
    int64_t j = 0;
    for (int k : order)
        for (int t = 0; t < hm[k].T.ntiles; ++t, ++j) parts[j % kEnsParts].push_back(EnsItem{k, t});
    std::vector<EnsItem> items;
    items.reserve((size_t)nitems);
    EnsCtrl hc;
    std::memset(&hc, 0, sizeof(hc));
    for (int p = 0; p < kEnsParts; ++p) {
        hc.part_begin[p] = (uint32_t)items.size();
        hc.part_len[p] = (uint32_t)parts[p].size();
        items.insert(items.end(), parts[p].begin(), parts[p].end());
    }
    hipStream_t s = e->stream;
    // member streams: everything is ordered on the ensemble stream from now on
    for (auto *m : e->members) {
        if (m->stream != s) EHIP(hipStreamSynchronize(m->stream));
    }
    hipError_t he;
    if ((he = hipMemcpyAsync(e->d_mem, hm.data(), sizeof(EnsMember) * (size_t)n, hipMemcpyHostToDevice, s)) ||
        (he = hipMemcpyAsync(e->d_items, items.data(), sizeof(EnsItem) * items.size(), hipMemcpyHostToDevice, s)) ||
        (he = hipMemcpyAsync(e->d_ctrl, &hc, sizeof(hc), hipMemcpyHostToDevice, s)) ||
        (he = hipStreamSynchronize(s))) {
        delete e;
        return set_error(SWE_E_HIP, std::string("ensemble upload: ") + hipGetErrorString(he));
    }
    for (auto *m : e->members) {
        m->ensemble = e;
        m->own_stream = m->stream;
        m->stream = s;
    }
    *out = e;
    return SWE_OK;
}

int swe_ensemble_step(swe_ensemble *e, int32_t n_steps)
{
    if (!e || n_steps < 0) return set_error(SWE_E_ARG, "bad arguments");
    if (e->broken) return set_error(SWE_E_STATE, "a member was destroyed before its ensemble");
    int left = n_steps, rc;
    if (!e->timing && e->use_graphs) {
        // whole chunks, then the remainder, each through a graph captured on
        // its first use and kept per (steps, parity)
        while (left > 0) {
            const int n = left >= kEnsGraphChunk ? kEnsGraphChunk : left;
            hipGraphExec_t g;
            if ((rc = ens_graph(e, n, e->parity, &g))) return rc;
            EHIP(hipGraphLaunch(g, e->stream));
            e->parity = (e->parity + n) & 1;
            left -= n;
        }
    }
    for (; left > 0; --left) {
        if ((rc = launch_ens_step(e, e->parity, e->stream, e->timing))) return rc;
        e->parity ^= 1;
    }
    if (n_steps & 1)
        for (auto *m : e->members) m->parity ^= 1;  // swe_read_state reads the member's current slot
    return SWE_OK;
}

int swe_ensemble_info(swe_ensemble *e, int32_t *rows_per_wave, int32_t *chunk, int64_t *items, int32_t *blocks)
{
    if (!e) return set_error(SWE_E_ARG, "ensemble is NULL");
    if (rows_per_wave) *rows_per_wave = e->by;
    if (chunk) *chunk = e->chunk;
    if (items) *items = e->nitems;
    if (blocks) *blocks = e->nblocks;
    return SWE_OK;
}

int swe_ensemble_use_graphs(swe_ensemble *e, int32_t on)
{
    if (!e) return set_error(SWE_E_ARG, "ensemble is NULL");
    e->use_graphs = on != 0;
    return SWE_OK;
}

int swe_ensemble_enable_timing(swe_ensemble *e, int32_t on)
{
    if (!e) return set_error(SWE_E_ARG, "ensemble is NULL");
    e->timing = on != 0;
    return SWE_OK;
}

int swe_ensemble_stage_times(swe_ensemble *e, double *ms1, double *ms2, int64_t *launches, int32_t reset)
{
    if (!e) return set_error(SWE_E_ARG, "ensemble is NULL");
    EHIP(hipStreamSynchronize(e->stream));
    double a = 0, b = 0;
    for (size_t k = 0; k + 3 < e->ev_used; k += 4) {
        float x = 0, y = 0;
        EHIP(hipEventElapsedTime(&x, e->ev_pool[k], e->ev_pool[k + 1]));
        EHIP(hipEventElapsedTime(&y, e->ev_pool[k + 2], e->ev_pool[k + 3]));
        a += x;
        b += y;
    }
    int64_t n = e->timed_steps;
    if (ms1) *ms1 = n ? a / n : 0.0;
    if (ms2) *ms2 = n ? b / n : 0.0;
    if (launches) *launches = n;
    if (reset) {
        e->ev_used = 0;
        e->timed_steps = 0;
    }
    return SWE_OK;
}

void swe_ensemble_destroy(swe_ensemble *e)
{
    if (!e) return;
    (void)hipStreamSynchronize(e->stream);  // NULL: the null stream
    for (auto &kv : e->graphs) (void)hipGraphExecDestroy(kv.second);
    for (auto g : e->graph_objs) (void)hipGraphDestroy(g);
    for (auto ev : e->ev_pool) (void)hipEventDestroy(ev);
    if (e->capture_stream) (void)hipStreamDestroy(e->capture_stream);
    for (auto *m : e->members) {
        if (!m) continue;
        m->stream = m->own_stream;
        m->ensemble = nullptr;
    }
    delete e;
}

}  // extern "C"
