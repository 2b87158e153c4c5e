// Query server with continuous batching.
//
// The folded CSD of every baseline stays resident (caller-owned device memory);
// the seeds of each (baseline, nside) are built on first use and cached.  A
// query names a baseline, a resolution and a contiguous band of bins; its
// answer is the broadband pair Xbb, Gbb of that band (Sec. V): the band sums
// of the narrowband maps (Eqs. eq_dirtymap, eq_fisher split per bin), computed
// without writing those maps by sgwb_broadband_maps (the band summed first
// through per-segment delay tables, or the dirty map's tiles adding up their
// strips' rows, whichever its cost estimate favours; Gbb is the band-summed
// weights against gamma^2, so no beam GEMM runs).
//
// A worker thread owns the device side:
//   * admission (serve_policy.h): cost-aware -- at most one heavy query (one
//     that fills the GPU alone) runs at a time, heavy queries start in arrival
//     order, light ones run beside it in the other slots (one HIP stream each)
//     and pass a heavy query waiting for its turn; every query needs its HBM
//     footprint to fit in the arena (a first-fit allocator over one allocation
//     made at creation, so serving never calls the device allocator);
//   * each admitted query's kernels are queued on its slot's stream, so work of
//     queries that arrive while others run overlaps on the device;
//   * completion is detected with an event per slot; the workspace goes back
//     to the arena at once, the broadband pair when the caller releases the
//     ticket.
// Results do not depend on the mix: every kernel has a fixed summation order.
#include <math.h>
#include <stdlib.h>
#include <stdio.h>
#include <string.h>
#include <sys/prctl.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "serve_policy.h"
#include "broadband.h"
#include "sgwb_internal.h"

using namespace sgwb;

namespace {

using Clock = std::chrono::steady_clock;

using serve::Arena;

struct Geom {
    float *gamma = nullptr;
    double *tau = nullptr;
    char *seeds = nullptr;  // seed-side products of the matrix-core dirty map
    bool seeded = false;    // seeds holds them (a matrix-core form applies)
    hipEvent_t ready = nullptr;
    int32_t npix = 0;
};

enum class QState { Pending, Running, Done };

struct Query {
    sgwb_query q;
    uint64_t ticket = 0;
    QState state = QState::Pending;
    int status = SGWB_OK;
    int slot = -1;
    Clock::time_point t_submit, t_start, t_done;
    char *ws = nullptr;                    // workspace (arena)
    float *Xbb = nullptr, *Gbb = nullptr;  // result (arena)
    size_t ws_bytes = 0;
    int32_t npix = 0;
    double cost = 0.0;  // map terms: segments x bins x pixels
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    uint64_t ticket = 0;  // 0 = free
    bool heavy = false;   // the running query is a heavy one
};

}  // namespace

struct sgwb_server {
    std::vector<sgwb_dataset> data;
    std::vector<double> tau_bound;  // per dataset: its baseline's chord / c
    std::vector<Slot> slots;
    int32_t queue_capacity = 0;
    Arena arena;
    char *arena_base = nullptr;
    std::map<std::pair<int, int>, Geom> geoms;
    std::map<uint64_t, Query> queries;
    std::deque<uint64_t> pending;
    uint64_t next_ticket = 1;
    std::mutex mu;
    std::condition_variable cv;
    std::thread worker;
    std::atomic<bool> stop{false};
    Clock::time_point t0;
    double heavy_terms = serve::kHeavyTermsDefault;
    int max_heavy = 1;  // heavy queries at a time
    // statistics
    uint64_t n_done = 0, n_failed = 0;
    double terms_done = 0.0;
    size_t peak_used = 0;
};

namespace {

double secs(const sgwb_server *s, Clock::time_point t)
{
    return std::chrono::duration<double>(t - s->t0).count();
}

size_t query_footprint(const sgwb_server *s, const sgwb_query &q, size_t *ws_bytes)
{
    const sgwb_dataset &d = s->data[q.dataset];
    const int64_t npix = 12LL * q.nside * q.nside;
    const int32_t nf = q.k_hi - q.k_lo;
    *ws_bytes = sgwb_broadband_maps_workspace_size(d.tg.nt, nf, (int32_t)npix, SGWB_MAPS_ANTIPODAL, &d.fg, 0, nf,
                                                   s->tau_bound[q.dataset]);
    auto up = [](size_t n) { return (n + 255) / 256 * 256; };
    return up(*ws_bytes) + 2 * up(npix * sizeof(float));
}

size_t geom_bytes(const sgwb_dataset &d, int nside)
{
    const size_t npix = 12ull * nside * nside;
    auto up = [](size_t n) { return (n + 255) / 256 * 256; };
    return up(npix * d.tg.nt * sizeof(float)) + up(npix * d.tg.nt * sizeof(double)) +
           up(xm_seed_bytes(d.tg.nt, (int32_t)npix));
}

// Build (or find) the seeds of (dataset, nside) and the dirty map's seed-side
// products (its form record and Bessel amplitudes), once; queued on stream st.
int ensure_geometry(sgwb_server *s, int ds, int nside, hipStream_t st, Geom **out)
{
    auto key = std::make_pair(ds, nside);
    auto it = s->geoms.find(key);
    if (it != s->geoms.end()) {
        *out = &it->second;
        return SGWB_OK;
    }
    const sgwb_dataset &d = s->data[ds];
    Geom g;
    g.npix = 12 * nside * nside;
    g.gamma = reinterpret_cast<float *>(s->arena.alloc((size_t)g.npix * d.tg.nt * sizeof(float)));
    g.tau = reinterpret_cast<double *>(s->arena.alloc((size_t)g.npix * d.tg.nt * sizeof(double)));
    g.seeds = s->arena.alloc(xm_seed_bytes(d.tg.nt, g.npix));
    if (!g.gamma || !g.tau || !g.seeds) {
        s->arena.release(reinterpret_cast<char *>(g.gamma));
        s->arena.release(reinterpret_cast<char *>(g.tau));
        s->arena.release(g.seeds);
        return set_error(SGWB_ENOMEM, "server: no room for the seeds of dataset %d at nside %d", ds, nside);
    }
    int rc = sgwb_build_geometry(&d.bl, nside, &d.tg, g.gamma, g.tau, st);
    if (!rc)
        rc = seed_products(d.C, d.w, d.ldc, d.tg.nt, d.nf, &d.fg, d.k0, g.gamma, g.tau, g.npix, g.seeds, st,
                           &g.seeded);
    if (!rc && (hipEventCreateWithFlags(&g.ready, hipEventDisableTiming) != hipSuccess ||
                hipEventRecord(g.ready, st) != hipSuccess))
        rc = check_hip(hipGetLastError(), "server: geometry event");
    if (rc) {
        // nothing was queued that writes the blocks (the build refused its
        // arguments on the host, or the event failed after it): make sure, then free
        (void)hipStreamSynchronize(st);
        if (g.ready) (void)hipEventDestroy(g.ready);
        s->arena.release(reinterpret_cast<char *>(g.gamma));
        s->arena.release(reinterpret_cast<char *>(g.tau));
        s->arena.release(g.seeds);
        return rc;
    }
    auto ins = s->geoms.emplace(key, g);
    *out = &ins.first->second;
    return SGWB_OK;
}

void fail_query(sgwb_server *s, Query &q, int status)
{
    q.status = status;
    q.state = QState::Done;
    q.t_start = q.t_done = Clock::now();
    s->n_failed++;
}

// Queue one admitted query on slot k.  Called with the lock held.
int launch_query(sgwb_server *s, Query &q, int k)
{
    Slot &sl = s->slots[k];
    const sgwb_dataset &d = s->data[q.q.dataset];
    const int nside = q.q.nside;
    Geom *g = nullptr;
    int rc = ensure_geometry(s, q.q.dataset, nside, sl.stream, &g);
    if (rc) return rc;
    if (hipStreamWaitEvent(sl.stream, g->ready, 0) != hipSuccess)
        return check_hip(hipGetLastError(), "server: wait for seeds");
    const int32_t nf = q.q.k_hi - q.q.k_lo;
    const int32_t npix = g->npix;
    q.ws = s->arena.alloc(q.ws_bytes);
    q.Xbb = reinterpret_cast<float *>(s->arena.alloc(npix * sizeof(float)));
    q.Gbb = reinterpret_cast<float *>(s->arena.alloc(npix * sizeof(float)));
    if (!q.ws || !q.Xbb || !q.Gbb)
        return set_error(SGWB_ENOMEM, "server: arena exhausted");
    q.npix = npix;
    const float *C = d.C + 2 * (int64_t)q.q.k_lo;
    const float *w = d.w + q.q.k_lo;
    // the broadband maps alone (no narrowband row, no beam GEMM), by the route
    // sgwb_broadband_maps picks for the query: the delay tables, or the strips
    // with the dirty map's seed-side products from the geometry cache
    rc = broadband_maps_seeded(C, w, d.ldc, d.tg.nt, nf, &d.fg, d.k0 + q.q.k_lo, g->gamma, g->tau, npix,
                               SGWB_MAPS_ANTIPODAL, s->tau_bound[q.q.dataset], d.H + q.q.k_lo, 0, nf, q.Xbb, q.Gbb,
                               q.ws, q.ws_bytes, g->seeded ? g->seeds : nullptr, sl.stream);
    if (rc) return rc;
    if (hipEventRecord(sl.done, sl.stream) != hipSuccess) return check_hip(hipGetLastError(), "server: record");
    sl.ticket = q.ticket;
    q.slot = k;
    q.state = QState::Running;
    q.t_start = Clock::now();
    return SGWB_OK;
}

void release_workspace(sgwb_server *s, Query &q)
{
    s->arena.release(q.ws);
    q.ws = nullptr;
}

void worker_loop(sgwb_server *s)
{
    // the 20 us polls below would otherwise be stretched by the default 50 us
    // timer slack of a Linux thread, and each query's completion seen that late
    (void)prctl(PR_SET_TIMERSLACK, 1000UL, 0UL, 0UL, 0UL);
    std::unique_lock<std::mutex> lk(s->mu);
    while (!s->stop.load()) {
        bool progressed = false;
        // retire finished queries
        for (auto &sl : s->slots) {
            if (!sl.ticket) continue;
            const hipError_t e = hipEventQuery(sl.done);
            if (e == hipErrorNotReady) continue;
            Query &q = s->queries[sl.ticket];
            q.t_done = Clock::now();
            q.state = QState::Done;
            if (e != hipSuccess) {
                q.status = check_hip(e, "server: query kernels");
                s->n_failed++;
            } else {
                s->n_done++;
                s->terms_done += (double)s->data[q.q.dataset].tg.nt * (q.q.k_hi - q.q.k_lo) * q.npix;
            }
            release_workspace(s, q);
            sl.ticket = 0;
            sl.heavy = false;
            progressed = true;
            s->cv.notify_all();
        }
        // admit pending queries (serve_policy.h: cost-aware, see the header)
        for (;;) {
            int free_slot = -1, nfree = 0;
            bool any_running = false;
            int heavy_running = 0;
            for (size_t k = 0; k < s->slots.size(); ++k) {
                if (!s->slots[k].ticket) {
                    if (free_slot < 0) free_slot = (int)k;
                    ++nfree;
                } else {
                    any_running = true;
                    heavy_running += s->slots[k].heavy ? 1 : 0;
                }
            }
            if (free_slot < 0 || s->pending.empty()) break;
            std::vector<serve::PendingView> views;
            views.reserve(s->pending.size());
            bool failed = false;
            for (size_t i = 0; i < s->pending.size(); ++i) {
                Query &q = s->queries[s->pending[i]];
                size_t need = query_footprint(s, q.q, &q.ws_bytes);
                if (!s->geoms.count(std::make_pair(q.q.dataset, q.q.nside)))
                    need += geom_bytes(s->data[q.q.dataset], q.q.nside);
                if (need > s->arena.size()) {  // can never run: fail it now, without device work
                    s->pending.erase(s->pending.begin() + (ptrdiff_t)i);
                    fail_query(s, q, set_error(SGWB_ENOMEM, "server: query needs %zu bytes, arena holds %zu", need,
                                               s->arena.size()));
                    failed = true;
                    break;
                }
                views.push_back({q.cost, need});
            }
            if (failed) {
                progressed = true;
                s->cv.notify_all();
                continue;
            }
            // with nothing running a query is tried even if the free ranges look
            // short (launch_query then reports SGWB_ENOMEM for it)
            const int idx = serve::pick_admission(views, serve::RunningView{nfree, heavy_running}, s->heavy_terms,
                                                  [&](size_t i) {
                                                      const size_t n = views[i].need;
                                                      return !any_running ||
                                                             (s->arena.size() - s->arena.used() >= n &&
                                                              s->arena.fits(n));
                                                  },
                                                  s->max_heavy);
            if (idx == serve::kAdmitNone) break;
            const uint64_t ticket = s->pending[(size_t)idx];
            s->pending.erase(s->pending.begin() + idx);
            Query &q = s->queries[ticket];
            const int rc = launch_query(s, q, free_slot);
            if (rc) {
                // kernels of this query may already be queued on the slot's
                // stream (seeds, maps): let them finish before the blocks go back
                (void)hipStreamSynchronize(s->slots[free_slot].stream);
                release_workspace(s, q);
                s->arena.release(reinterpret_cast<char *>(q.Xbb));
                s->arena.release(reinterpret_cast<char *>(q.Gbb));
                q.Xbb = q.Gbb = nullptr;
                fail_query(s, q, rc);
                s->cv.notify_all();
            } else {
                s->slots[free_slot].heavy = q.cost >= s->heavy_terms;
            }
            s->peak_used = std::max(s->peak_used, s->arena.used());
            progressed = true;
        }
        if (!progressed) {
            bool running = false;
            for (auto &sl : s->slots) running |= sl.ticket != 0;
            // poll running work every 20 us; sleep until a submit otherwise
            if (running)
                s->cv.wait_for(lk, std::chrono::microseconds(20));
            else
                s->cv.wait_for(lk, std::chrono::milliseconds(50));
        }
    }
}

}  // namespace

extern "C" {

int sgwb_server_create(const sgwb_server_cfg *cfg, sgwb_server **out)
{
    if (!out) return set_error(SGWB_EINVAL, "server_create: null out");
    *out = nullptr;
    if (!cfg || !cfg->datasets || cfg->ndatasets < 1) return set_error(SGWB_EINVAL, "server_create: no datasets");
    if (cfg->slots < 1 || cfg->slots > 16) return set_error(SGWB_EINVAL, "server_create: slots must be 1..16");
    for (int i = 0; i < cfg->ndatasets; ++i) {
        const sgwb_dataset &d = cfg->datasets[i];
        if (!d.C || !d.w || !d.H) return set_error(SGWB_EINVAL, "server_create: dataset %d: null pointer", i);
        if (d.tg.nt < 1 || d.nf < 1 || d.ldc < d.nf || d.k0 < 0)
            return set_error(SGWB_EINVAL, "server_create: dataset %d: bad shape", i);
        if (!isfinite(d.fg.f0_hz) || !isfinite(d.fg.df_hz) || d.fg.df_hz <= 0.0 || !isfinite(d.tg.stride_s) ||
            !isfinite(d.tg.t0_s) || !isfinite(d.tg.seg_dur_s))
            return set_error(SGWB_EINVAL, "server_create: dataset %d: bad grid", i);
    }
    sgwb_server *s = new sgwb_server();
    s->data.assign(cfg->datasets, cfg->datasets + cfg->ndatasets);
    for (const sgwb_dataset &d : s->data) s->tau_bound.push_back(sgwb_baseline_delay_bound(&d.bl));
    s->queue_capacity = cfg->queue_capacity > 0 ? cfg->queue_capacity : 1 << 20;
    size_t budget = cfg->hbm_budget_bytes;
    if (budget == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
            delete s;
            return check_hip(hipGetLastError(), "server_create: hipMemGetInfo");
        }
        budget = fr / 10 * 6;
    }
    budget = budget / 256 * 256;
    if (hipMalloc(&s->arena_base, budget) != hipSuccess) {
        delete s;
        return set_error(SGWB_ENOMEM, "server_create: cannot reserve %zu bytes of HBM", budget);
    }
    s->arena.init(s->arena_base, budget);
    s->slots.resize(cfg->slots);
    for (auto &sl : s->slots) {
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) {
            sgwb_server_destroy(s);
            return check_hip(hipGetLastError(), "server_create: streams");
        }
    }
    s->t0 = Clock::now();
    if (const char *e = getenv("SGWB_SERVER_HEAVY_TERMS")) {
        const double v = atof(e);
        if (v > 0.0) s->heavy_terms = v;
    }
    if (const char *e = getenv("SGWB_SERVER_MAX_HEAVY")) {
        const int v = atoi(e);
        if (v >= 1 && v <= 64) s->max_heavy = v;
    }
    int dev = 0;
    (void)hipGetDevice(&dev);
    s->worker = std::thread([s, dev] {
        (void)hipSetDevice(dev);
        worker_loop(s);
    });
    *out = s;
    return SGWB_OK;
}

int sgwb_server_submit(sgwb_server *s, const sgwb_query *q, uint64_t *ticket)
{
    if (!s || !q || !ticket) return set_error(SGWB_EINVAL, "server_submit: null argument");
    if (q->dataset < 0 || q->dataset >= (int)s->data.size())
        return set_error(SGWB_EINVAL, "server_submit: no dataset %d", q->dataset);
    if (!is_pow2_nside(q->nside)) return set_error(SGWB_EINVAL, "server_submit: bad nside %d", q->nside);
    const sgwb_dataset &d = s->data[q->dataset];
    if (!(0 <= q->k_lo && q->k_lo < q->k_hi && q->k_hi <= d.nf))
        return set_error(SGWB_EINVAL, "server_submit: band [%d, %d) outside the dataset's %d bins", q->k_lo, q->k_hi,
                         d.nf);
    std::lock_guard<std::mutex> lk(s->mu);
    if ((int64_t)s->pending.size() >= s->queue_capacity) return set_error(SGWB_EBUSY, "server_submit: queue full");
    Query qq;
    qq.q = *q;
    // cost in map-term equivalents: the route's time estimate at the strips
    // route's rate (4.2e13 terms/s), so that a band-first query counts for
    // what it costs, not for its nt x band x npix terms
    const int32_t npix = 12 * q->nside * q->nside, nb = q->k_hi - q->k_lo;
    const double est = broadband_cost_seconds(d.tg.nt, nb, npix, SGWB_MAPS_ANTIPODAL, &d.fg, 0, nb,
                                              s->tau_bound[q->dataset]);
    qq.cost = est >= 0.0 ? est * 4.2e13 : (double)d.tg.nt * nb * (double)npix;
    qq.ticket = s->next_ticket++;
    qq.t_submit = Clock::now();
    s->queries.emplace(qq.ticket, qq);
    s->pending.push_back(qq.ticket);
    *ticket = qq.ticket;
    s->cv.notify_all();
    return SGWB_OK;
}

int sgwb_server_poll(sgwb_server *s, uint64_t ticket, sgwb_result *out)
{
    if (!s || !out) return set_error(SGWB_EINVAL, "server_poll: null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->queries.find(ticket);
    if (it == s->queries.end()) return set_error(SGWB_EINVAL, "server_poll: unknown ticket");
    const Query &q = it->second;
    if (q.state != QState::Done) return SGWB_EAGAIN;
    out->status = q.status;
    out->npix = q.npix;
    out->Xbb = q.Xbb;
    out->Gbb = q.Gbb;
    out->t_submit_s = secs(s, q.t_submit);
    out->t_start_s = secs(s, q.t_start);
    out->t_done_s = secs(s, q.t_done);
    return SGWB_OK;
}

int sgwb_server_fetch(sgwb_server *s, uint64_t ticket, float *Xbb, float *Gbb, hipStream_t stream)
{
    if (!s || !Xbb || !Gbb) return set_error(SGWB_EINVAL, "server_fetch: null argument");
    const float *xs, *gs;
    size_t n;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->queries.find(ticket);
        if (it == s->queries.end()) return set_error(SGWB_EINVAL, "server_fetch: unknown ticket");
        const Query &q = it->second;
        if (q.state != QState::Done) return SGWB_EAGAIN;
        if (q.status != SGWB_OK) return q.status;
        xs = q.Xbb;
        gs = q.Gbb;
        n = (size_t)q.npix * sizeof(float);
    }
    hipError_t e = hipMemcpyAsync(Xbb, xs, n, hipMemcpyDefault, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(Gbb, gs, n, hipMemcpyDefault, stream);
    return check_hip(e, "server_fetch: copy");
}

int sgwb_server_release(sgwb_server *s, uint64_t ticket)
{
    if (!s) return set_error(SGWB_EINVAL, "server_release: null server");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->queries.find(ticket);
    if (it == s->queries.end()) return set_error(SGWB_EINVAL, "server_release: unknown ticket");
    if (it->second.state != QState::Done) return set_error(SGWB_EINVAL, "server_release: query not finished");
    s->arena.release(reinterpret_cast<char *>(it->second.Xbb));
    s->arena.release(reinterpret_cast<char *>(it->second.Gbb));
    s->queries.erase(it);
    s->cv.notify_all();
    return SGWB_OK;
}

int sgwb_server_stats(sgwb_server *s, char *buf, size_t len)
{
    if (!s || !buf || !len) return set_error(SGWB_EINVAL, "server_stats: bad arguments");
    std::lock_guard<std::mutex> lk(s->mu);
    size_t running = 0;
    for (auto &sl : s->slots) running += sl.ticket != 0;
    const int n = snprintf(buf, len,
                           "{\"done\": %llu, \"failed\": %llu, \"pending\": %zu, \"running\": %zu, \"terms_done\": %.6e, "
                           "\"arena_bytes\": %zu, \"arena_used\": %zu, \"arena_peak\": %zu, \"geometries\": %zu, "
                           "\"slots\": %zu, \"heavy_terms\": %.6e, \"uptime_s\": %.6f}",
                           (unsigned long long)s->n_done, (unsigned long long)s->n_failed, s->pending.size(), running,
                           s->terms_done, s->arena.size(), s->arena.used(), s->peak_used, s->geoms.size(),
                           s->slots.size(), s->heavy_terms, secs(s, Clock::now()));
    if (n < 0 || (size_t)n >= len) return set_error(SGWB_ENOMEM, "server_stats: buffer too small");
    return SGWB_OK;
}

void sgwb_server_destroy(sgwb_server *s)
{
    if (!s) return;
    s->stop.store(true);
    s->cv.notify_all();
    if (s->worker.joinable()) s->worker.join();
    for (auto &sl : s->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    for (auto &kv : s->geoms)
        if (kv.second.ready) (void)hipEventDestroy(kv.second.ready);
    if (s->arena_base) (void)hipFree(s->arena_base);
    delete s;
}

}  // extern "C"
