// Serving loop (include/swe.h): continuous batching of forecast requests
// over one device arena.  Host-side only: the time stepping is the batched
// ensemble launch; this file holds the admission queue, the arena
// allocator, the tick sequence and the completion records.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>

#include "swe_arena.h"
#include "swe_host.h"

using namespace swe;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

#define SHIP(expr)                                                                                       \
    do {                                                                                                 \
        hipError_t e_ = (expr);                                                                          \
        if (e_ != hipSuccess) return set_error(SWE_E_HIP, std::string(#expr ": ") + hipGetErrorString(e_)); \
    } while (0)

// The leading fields of the device control block that a tick reads back for
// every active request (time, flags, step count).
struct CtrlHead {
    double t[2];
    uint32_t flags;
    float dt_last;
    int64_t steps;
    double t_end;
    double mass, energy;
    double pad0;
};
static_assert(offsetof(CtrlHead, t) == offsetof(Ctrl, t), "control block layout");
static_assert(offsetof(CtrlHead, flags) == offsetof(Ctrl, flags), "control block layout");
static_assert(offsetof(CtrlHead, steps) == offsetof(Ctrl, steps), "control block layout");
static_assert(sizeof(CtrlHead) <= sizeof(Ctrl), "control block layout");

struct Pending {
    swe_request r{};  // pointers below re-aimed at the owned copies
    std::vector<float> Hc, f, theta, eta, hu, hv, wind_tau, bnd;
    std::vector<uint8_t> land;
    std::vector<double> wind_t, bnd_t;
    size_t bytes = 0;
    int max_wind = 1;
};

struct Active {
    std::unique_ptr<Pending> req;
    swe_domain *dom = nullptr;
    size_t off = 0, bytes = 0;
    int64_t steps_seen = 0;
};

}  // namespace

struct swe_server {
    char *arena_base = nullptr;
    Arena arena;
    hipStream_t stream = nullptr, upload = nullptr;
    int max_active = 1, steps_per_tick = 1, rows = 0, chunk = 0;
    std::mutex qlock;  // guards pending and submitted (swe_server_submit may run beside a tick)
    std::deque<std::unique_ptr<Pending>> pending;
    std::vector<Active> active;
    std::deque<swe_completion> done;
    swe_ensemble *ens = nullptr;
    size_t ens_off = 0, ens_bytes = 0;          // queue block of the current ensemble
    size_t ens_new_off = 0, ens_new_bytes = 0;  // grown block, swapped in at the next rebuild
    bool dirty = false;  // the active set changed since the ensemble was built
    CtrlHead *heads = nullptr;  // pinned, one per active slot
    int64_t submitted = 0, admitted = 0, completed = 0, ticks = 0, cell_steps = 0;
    double t_rebuild = 0, t_launch = 0, t_admit = 0, t_wait = 0, t_retire = 0;
};

namespace {

void drop_ensemble(swe_server *s)
{
    if (s->ens) {
        swe_ensemble_destroy(s->ens);
        s->ens = nullptr;
    }
}

// Copies a request's host inputs so the caller may free them on return.
int copy_request(const swe_request *r, Pending *q)
{
    const swe_params &p = r->params;
    size_t nc = (size_t)p.nx * p.ny, nk = (size_t)(p.nx + 1) * (p.ny + 1);
    q->r = *r;
    q->Hc.assign(r->Hc, r->Hc + nk);
    q->f.assign(r->f, r->f + nc);
    if (r->theta) q->theta.assign(r->theta, r->theta + nc);
    if (r->land) q->land.assign(r->land, r->land + nc);
    q->eta.assign(r->eta, r->eta + nc);
    q->hu.assign(r->hu, r->hu + nc);
    q->hv.assign(r->hv, r->hv + nc);
    if (r->n_wind > 0) {
        q->wind_t.assign(r->wind_t, r->wind_t + r->n_wind);
        q->wind_tau.assign(r->wind_tau, r->wind_tau + 2 * (size_t)r->n_wind);
    }
    if (r->n_bnd > 0) {
        size_t per = 3 * (2 * (size_t)p.nx + 2 * (size_t)p.ny);
        q->bnd_t.assign(r->bnd_t, r->bnd_t + r->n_bnd);
        q->bnd.assign(r->bnd, r->bnd + per * r->n_bnd);
    }
    q->r.Hc = q->Hc.data();
    q->r.f = q->f.data();
    q->r.theta = r->theta ? q->theta.data() : nullptr;
    q->r.land = r->land ? q->land.data() : nullptr;
    q->r.eta = q->eta.data();
    q->r.hu = q->hu.data();
    q->r.hv = q->hv.data();
    q->r.wind_t = r->n_wind > 0 ? q->wind_t.data() : nullptr;
    q->r.wind_tau = r->n_wind > 0 ? q->wind_tau.data() : nullptr;
    q->r.bnd_t = r->n_bnd > 0 ? q->bnd_t.data() : nullptr;
    q->r.bnd = r->n_bnd > 0 ? q->bnd.data() : nullptr;
    return SWE_OK;
}

// Uploads a waiting request into its arena block on the upload stream.
int start_request(swe_server *s, Pending *q, size_t off, swe_domain **out)
{
    const swe_request &r = q->r;
    swe_domain *d = nullptr;
    int rc = swe_init_domain(&r.params, s->arena_base + off, q->bytes, s->upload, q->max_wind, r.n_bnd, r.Hc, r.land,
                             r.f, r.theta, r.eta, r.hu, r.hv, &d);
    if (rc) return rc;
    if (r.n_wind > 0 && (rc = swe_set_forcing(d, SWE_FORCING_WIND_STRESS, r.n_wind, r.wind_t, r.wind_tau))) {
        swe_destroy(d);
        return rc;
    }
    if (r.n_bnd > 0 && (rc = swe_set_forcing(d, SWE_FORCING_BOUNDARY, r.n_bnd, r.bnd_t, r.bnd))) {
        swe_destroy(d);
        return rc;
    }
    // the run-to-time rule: steps clamp to the horizon and stop there
    hipError_t he = launch_set_t_end(d->dom.ctrl, r.horizon, s->upload);
    if (he == hipSuccess) he = hipStreamSynchronize(s->upload);
    if (he != hipSuccess) {
        swe_destroy(d);
        return set_error(SWE_E_HIP, std::string("request start: ") + hipGetErrorString(he));
    }
    *out = d;
    return SWE_OK;
}

std::vector<swe_domain *> active_domains(swe_server *s)
{
    std::vector<swe_domain *> v;
    for (auto &a : s->active) v.push_back(a.dom);
    return v;
}

// An idle server gives its work-queue blocks back, so that the arena is
// whole for the next admission.
void release_queue_blocks(swe_server *s)
{
    drop_ensemble(s);
    if (s->ens_bytes) s->arena.release(s->ens_off, s->ens_bytes);
    if (s->ens_new_bytes) s->arena.release(s->ens_new_off, s->ens_new_bytes);
    s->ens_bytes = s->ens_new_bytes = 0;
    s->dirty = false;
}

// The head of the queue does not fit even in an empty arena (its workspace
// plus its work queue): it completes at once with SWE_E_NOMEM.
int refuse_head(swe_server *s, std::unique_ptr<Pending> q)
{
    swe_completion c{};
    c.id = q->r.id;
    c.tick = s->ticks;
    c.status = SWE_E_NOMEM;
    s->done.push_back(c);
    s->completed += 1;
    return SWE_OK;
}

std::unique_ptr<Pending> pop_pending(swe_server *s)
{
    std::lock_guard<std::mutex> g(s->qlock);
    if (s->pending.empty()) return nullptr;
    auto q = std::move(s->pending.front());
    s->pending.pop_front();
    return q;
}

void push_back_front(swe_server *s, std::unique_ptr<Pending> q)
{
    std::lock_guard<std::mutex> g(s->qlock);
    s->pending.push_front(std::move(q));
}

// Admit waiting requests in arrival order while a slot is free and both the
// request's workspace and the (possibly grown) ensemble queue fit in the
// arena.  Runs while the current tick's steps execute: nothing the running
// ensemble uses is touched (a grown queue block is carved beside the old
// one and swapped in at the next rebuild).
int admit(swe_server *s)
{
    std::vector<std::pair<int, int>> shapes;
    for (auto &a : s->active) shapes.emplace_back(a.dom->p.nx, a.dom->p.ny);
    while ((int)s->active.size() < s->max_active) {
        std::unique_ptr<Pending> q = pop_pending(s);
        if (!q) break;
        // one ensemble launch runs one kernel variant: a request of another
        // kind (north-vector projection, compensated state) than the active
        // set waits at the head of the queue until the active set has drained
        if (!s->active.empty()) {
            const swe_params &a = s->active.front().dom->p, &b = q->r.params;
            if (a.north_projection != b.north_projection || a.compensated_state != b.compensated_state) {
                push_back_front(s, std::move(q));
                break;
            }
        }
        size_t off;
        if (!s->arena.alloc(q->bytes, &off)) {
            if (s->active.empty()) return refuse_head(s, std::move(q));  // could never start
            push_back_front(s, std::move(q));
            break;
        }
        // the queue size depends only on the members' shapes
        shapes.emplace_back(q->r.params.nx, q->r.params.ny);
        const size_t need = ensemble_bytes_for_shapes(shapes, s->rows);
        size_t have = s->ens_new_bytes ? s->ens_new_bytes : s->ens_bytes;
        size_t grow_off = 0, grow_bytes = 0;
        if (need > have) {
            grow_bytes = align_up(need + need / 2, kAlign);
            if (!s->arena.alloc(grow_bytes, &grow_off)) {
                grow_bytes = align_up(need, kAlign);
                if (!s->arena.alloc(grow_bytes, &grow_off)) {
                    s->arena.release(off, q->bytes);
                    shapes.pop_back();
                    if (s->active.empty()) return refuse_head(s, std::move(q));
                    push_back_front(s, std::move(q));
                    break;
                }
            }
        }
        swe_domain *d = nullptr;
        int rc = start_request(s, q.get(), off, &d);
        if (rc) {
            s->arena.release(off, q->bytes);
            if (grow_bytes) s->arena.release(grow_off, grow_bytes);
            shapes.pop_back();
            if (rc == SWE_E_HIP) return rc;  // a runtime failure stops the server
            // the request itself was refused (its inputs): report it, go on
            swe_completion c{};
            c.id = q->r.id;
            c.tick = s->ticks;
            c.status = rc;
            s->done.push_back(c);
            s->completed += 1;
            continue;
        }
        if (grow_bytes) {
            if (s->ens_new_bytes) s->arena.release(s->ens_new_off, s->ens_new_bytes);
            s->ens_new_off = grow_off;
            s->ens_new_bytes = grow_bytes;
        }
        Active a;
        a.bytes = q->bytes;
        a.req = std::move(q);
        a.dom = d;
        a.off = off;
        s->active.push_back(std::move(a));
        s->admitted += 1;
        s->dirty = true;
    }
    return SWE_OK;
}

int rebuild(swe_server *s)
{
    drop_ensemble(s);
    s->dirty = false;
    if (s->ens_new_bytes) {
        if (s->ens_bytes) s->arena.release(s->ens_off, s->ens_bytes);
        s->ens_off = s->ens_new_off;
        s->ens_bytes = s->ens_new_bytes;
        s->ens_new_bytes = 0;
    }
    if (s->active.empty()) return SWE_OK;
    std::vector<swe_domain *> doms = active_domains(s);
    int rc = swe_ensemble_create(doms.data(), (int)doms.size(), s->arena_base + s->ens_off, s->ens_bytes, s->stream,
                                 s->rows, s->chunk, &s->ens);
    if (rc) return rc;
    return swe_ensemble_use_graphs(s->ens, 0);
}

// Copies a finished request's state to the caller's buffers and records it.
int complete(swe_server *s, Active &a, double t, int64_t steps, int status)
{
    const swe_request &r = a.req->r;
    if (r.out_eta && r.out_hu && r.out_hv) {
        double tt, dtn;
        int rr = swe_read_state(a.dom, r.out_eta, r.out_hu, r.out_hv, &tt, &dtn);
        if (rr && rr != SWE_E_UNSTABLE) return rr;
    }
    swe_completion c{};
    c.id = r.id;
    c.t = t;
    c.steps = steps;
    c.tick = s->ticks;
    c.status = status;
    s->done.push_back(c);
    s->completed += 1;
    return SWE_OK;
}

}  // namespace

extern "C" {

int swe_server_create(void *dev_arena, size_t arena_bytes, void *hip_stream, void *upload_stream, int32_t max_active,
                      int32_t steps_per_tick, int32_t rows_per_wave, int32_t chunk, swe_server **out)
{
    if (!out || !dev_arena || arena_bytes < kAlign || max_active < 1 || max_active > 65536 || steps_per_tick < 1 ||
        rows_per_wave < 0 || rows_per_wave > 4096 || chunk < 0 || chunk > 1024)
        return set_error(SWE_E_ARG, "bad server arguments");
    if (((uintptr_t)dev_arena) % kAlign) return set_error(SWE_E_ARG, "arena must be 256-byte aligned");
    swe_server *s = new (std::nothrow) swe_server();
    if (!s) return set_error(SWE_E_NOMEM, "host allocation failed");
    s->arena_base = (char *)dev_arena;
    s->arena.reset(arena_bytes / kAlign * kAlign);
    s->stream = (hipStream_t)hip_stream;
    s->upload = (hipStream_t)upload_stream;
    s->max_active = max_active;
    s->steps_per_tick = steps_per_tick;
    s->rows = rows_per_wave;
    s->chunk = chunk;
    hipError_t he = hipHostMalloc((void **)&s->heads, sizeof(CtrlHead) * (size_t)max_active, hipHostMallocDefault);
    if (he != hipSuccess) {
        delete s;
        return set_error(SWE_E_HIP, std::string("hipHostMalloc: ") + hipGetErrorString(he));
    }
    *out = s;
    return SWE_OK;
}

int swe_server_submit(swe_server *s, const swe_request *r)
{
    if (!s || !r) return set_error(SWE_E_ARG, "NULL argument");
    if (!r->Hc || !r->f || !r->eta || !r->hu || !r->hv) return set_error(SWE_E_ARG, "missing request input");
    if (!std::isfinite(r->horizon) || r->horizon < 0) return set_error(SWE_E_ARG, "horizon must be finite and >= 0");
    if (r->n_wind < 0 || r->n_bnd < 0 || (r->n_wind > 0 && (!r->wind_t || !r->wind_tau)) ||
        (r->n_bnd > 0 && (!r->bnd_t || !r->bnd)))
        return set_error(SWE_E_ARG, "bad forcing arguments");
    auto q = std::make_unique<Pending>();
    q->max_wind = std::max<int>(1, r->n_wind);
    int rc = swe_workspace_bytes(&r->params, q->max_wind, r->n_bnd, &q->bytes);
    if (rc) return rc;
    if (align_up(q->bytes, kAlign) > s->arena.size()) return set_error(SWE_E_NOMEM, "request larger than the arena");
    copy_request(r, q.get());
    std::lock_guard<std::mutex> g(s->qlock);
    s->pending.push_back(std::move(q));
    s->submitted += 1;
    return SWE_OK;
}

int swe_server_tick(swe_server *s, int32_t *n_active, int32_t *n_pending)
{
    if (!s) return set_error(SWE_E_ARG, "server is NULL");
    using clk = std::chrono::steady_clock;
    auto secs = [](clk::time_point a, clk::time_point b) { return std::chrono::duration<double>(b - a).count(); };
    int rc;
    auto t0 = clk::now();
    if (s->dirty && (rc = rebuild(s))) return rc;
    auto t1 = clk::now();
    // 1. the active set advances (asynchronously) ...
    if (s->ens && (rc = swe_ensemble_step(s->ens, s->steps_per_tick))) return rc;
    auto t2 = clk::now();
    // 2. ... while waiting requests are uploaded on the other stream
    const size_t n_before = s->active.size();
    if ((rc = admit(s))) return rc;
    auto t3 = clk::now();
    // 3. read back the control heads of the members that took part
    for (size_t k = 0; k < n_before; ++k)
        SHIP(hipMemcpyAsync(&s->heads[k], s->active[k].dom->dom.ctrl, sizeof(CtrlHead), hipMemcpyDeviceToHost,
                            s->stream));
    SHIP(hipStreamSynchronize(s->stream));
    auto t4 = clk::now();
    s->t_rebuild += secs(t0, t1);
    s->t_launch += secs(t1, t2);
    s->t_admit += secs(t2, t3);
    s->t_wait += secs(t3, t4);
    s->ticks += 1;
    // 4. retire finished (or failed) requests; newly admitted ones join at
    //    the next tick (a zero horizon completes at once)
    std::vector<Active> keep, gone;
    keep.reserve(s->active.size());
    for (size_t k = 0; k < s->active.size(); ++k) {
        Active &a = s->active[k];
        const double horizon = a.req->r.horizon;
        if (k < n_before) {
            const CtrlHead &h = s->heads[k];
            const int64_t ncell = (int64_t)a.req->r.params.nx * a.req->r.params.ny;
            const double t = h.t[a.dom->parity];
            s->cell_steps += (h.steps - a.steps_seen) * ncell;
            a.steps_seen = h.steps;
            if (h.flags || t >= horizon) {
                if ((rc = complete(s, a, t, h.steps, h.flags ? SWE_E_UNSTABLE : SWE_OK))) return rc;
                gone.push_back(std::move(a));
                continue;
            }
        } else if (horizon <= 0.0) {
            if ((rc = complete(s, a, 0.0, 0, SWE_OK))) return rc;
            gone.push_back(std::move(a));
            continue;
        }
        keep.push_back(std::move(a));
    }
    if (!gone.empty()) {
        drop_ensemble(s);  // the ensemble borrows its members: release it first
        for (auto &a : gone) {
            swe_destroy(a.dom);
            s->arena.release(a.off, a.bytes);
        }
        s->dirty = true;
    }
    s->active = std::move(keep);
    if (s->active.empty()) release_queue_blocks(s);
    s->t_retire += secs(t4, clk::now());
    if (n_active) *n_active = (int32_t)s->active.size();
    if (n_pending) {
        std::lock_guard<std::mutex> g(s->qlock);
        *n_pending = (int32_t)s->pending.size();
    }
    return SWE_OK;
}

int swe_server_poll(swe_server *s, swe_completion *out, int32_t max, int32_t *n)
{
    if (!s || !n || max < 0 || (max > 0 && !out)) return set_error(SWE_E_ARG, "bad poll arguments");
    int32_t k = 0;
    while (k < max && !s->done.empty()) {
        out[k++] = s->done.front();
        s->done.pop_front();
    }
    *n = k;
    return SWE_OK;
}

int swe_server_get_stats(swe_server *s, swe_server_stats *st)
{
    if (!s || !st) return set_error(SWE_E_ARG, "NULL argument");
    std::lock_guard<std::mutex> g(s->qlock);
    st->submitted = s->submitted;
    st->admitted = s->admitted;
    st->completed = s->completed;
    st->ticks = s->ticks;
    st->cell_steps = s->cell_steps;
    st->arena_bytes = s->arena.size();
    st->arena_used = s->arena.used();
    st->arena_peak = s->arena.peak();
    st->active = (int32_t)s->active.size();
    st->pending = (int32_t)s->pending.size();
    st->host_rebuild_s = s->t_rebuild;
    st->host_launch_s = s->t_launch;
    st->host_admit_s = s->t_admit;
    st->host_wait_s = s->t_wait;
    st->host_retire_s = s->t_retire;
    return SWE_OK;
}

void swe_server_destroy(swe_server *s)
{
    if (!s) return;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    drop_ensemble(s);
    for (auto &a : s->active) swe_destroy(a.dom);
    if (s->heads) (void)hipHostFree(s->heads);
    delete s;
}

}  // extern "C"
