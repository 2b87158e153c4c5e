// Batched plans: several map jobs (baselines, resolutions, uneven bands) in one
// persistent dirty-map launch and one persistent beam launch, captured with the
// per-job operand preparation and broadband reductions in a HIP graph.
//
// plan_create validates the jobs, owns the per-job workspaces and the device
// job tables, picks the tunables (tile order and grid of the dirty-map launch,
// wave-tile shape and grid of the beam launch) with the autotuner (cache in tune.hip)
// (timed on the device, cached on disk), and captures the graph.
// plan_launch replays the graph on the caller's stream: no allocation, no host
// synchronisation.  The tuner also decides whether the beams run on a branch of
// their own beside the dirty maps (two graph branches, joined before the
// broadband sums) or after them on the one stream.  Every tunable changes only the schedule, never an output's
// summation order, so all choices give bitwise identical maps.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "sgwb_internal.h"

using namespace sgwb;

struct sgwb_plan {
    std::vector<sgwb_job> jobs;
    std::vector<MapArgs> args;
    // dirty map
    std::vector<XJob> xjobs;  // host copy, tile_begin filled; antipodal jobs first
    XJob *d_xjobs = nullptr;
    int64_t x_tiles = 0;
    int32_t nx_pair = 0;         // xjobs[0, nx_pair) use antipodal pairs
    int64_t x_tiles_pair = 0;    // tiles of those jobs
    // dirty map on the matrix cores (jobs where that form applies)
    std::vector<XmJob> xmjobs;
    XmJob *d_xmjobs = nullptr;
    int64_t xm_tiles = 0;
    // beam
    std::vector<BJob> bjobs;
    BJob *d_bjobs = nullptr;
    int64_t b_wgs = 0;
    // band: per job, the dirty map's per-strip partial sums (matrix-core jobs)
    // and the scratch of the weight-side broadband Fisher diagonal
    std::vector<size_t> band_off;
    std::vector<char> use_xm;
    // memory
    void *beam_ws = nullptr, *band_ws = nullptr, *xm_ws = nullptr;
    size_t beam_bytes = 0, band_bytes = 0, xm_bytes = 0;
    Tunables tun;
    bool tuned = false, from_cache = false;
    std::vector<double> tune_ms;
    std::string tune_key;
    int num_cus = 0;
    int device = 0;
    hipStream_t cap = nullptr;
    hipStream_t side = nullptr;  // second branch (beams) of the branched schedule
    hipEvent_t fork = nullptr, join = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace sgwb {

int validate_job(const sgwb_job &j, MapArgs *a)
{
    int rc = check_maps_args_f32(j.C, j.w, j.ldc, j.nt, j.nf, &j.fg, j.k0, j.gamma, j.tau, j.npix, j.flags, a);
    if (rc) return rc;
    if (!j.X && !j.Gam) return set_error(SGWB_EINVAL, "plan: job computes nothing (X and Gam are NULL)");
    const bool band = j.Xbb || j.Gbb;
    if (band) {
        if (!(0 <= j.band_lo && j.band_lo <= j.band_hi && j.band_hi <= j.nf))
            return set_error(SGWB_EINVAL, "plan: band rows out of range");
        if ((j.Xbb && !j.X) || (j.Gbb && (!j.Gam || !j.H)))
            return set_error(SGWB_EINVAL, "plan: broadband output without its narrowband input");
    }
    return SGWB_OK;
}

// (Re)build the device job tables for the current tunables.
static int upload_tables(sgwb_plan *p)
{
    // each pairing class is its own launch, so each numbers its tiles from 0
    int64_t t = 0;
    for (size_t i = 0; i < p->xjobs.size(); ++i) {
        if ((int32_t)i == p->nx_pair) {
            p->x_tiles_pair = t;
            t = 0;
        }
        XJob &x = p->xjobs[i];
        x.strip_major = p->tun.x_strip_major;
        x.tile_begin = t;
        t += xjob_tiles(x);
    }
    if ((size_t)p->nx_pair == p->xjobs.size()) {
        p->x_tiles_pair = t;
        t = 0;
    }
    p->x_tiles = p->x_tiles_pair + t;
    int64_t tx = 0;
    for (auto &x : p->xmjobs) {
        x.tile_begin = tx;
        tx += xmjob_tiles(x);
    }
    p->xm_tiles = tx;
    int64_t wg = 0;
    for (auto &b : p->bjobs) {
        b.wg_begin = wg;
        const int64_t n = bjob_workgroups(b, p->tun.beam_shape);
        wg += (n + 7) / 8 * 8;  // keep every job's range XCD-aligned
    }
    p->b_wgs = wg;
    hipError_t e = hipSuccess;
    if (!p->xjobs.empty())
        e = hipMemcpy(p->d_xjobs, p->xjobs.data(), p->xjobs.size() * sizeof(XJob), hipMemcpyHostToDevice);
    if (e == hipSuccess && !p->xmjobs.empty())
        e = hipMemcpy(p->d_xmjobs, p->xmjobs.data(), p->xmjobs.size() * sizeof(XmJob), hipMemcpyHostToDevice);
    if (e == hipSuccess && !p->bjobs.empty())
        e = hipMemcpy(p->d_bjobs, p->bjobs.data(), p->bjobs.size() * sizeof(BJob), hipMemcpyHostToDevice);
    return check_hip(e, "plan: upload job tables");
}

// Queue the whole plan on stream s (used for capture and for timing).
static hipError_t enqueue(sgwb_plan *p, hipStream_t s, int parts)
{
    hipError_t e = hipSuccess;
    if (parts & 2) {
        for (auto &b : p->bjobs)
            if ((e = launch_beam_prep(b, s)) != hipSuccess) return e;
    }
    if ((parts & 1) && p->xm_tiles > 0) {
        for (auto &x : p->xmjobs)
            if ((e = launch_xm_prep(x, s)) != hipSuccess) return e;
        if (p->tun.xm_per_job) {
            // the single-call kernel per job: the same tiles, so the same bits
            for (auto &x : p->xmjobs)
                if ((e = launch_xm_main(x, s)) != hipSuccess) return e;
        } else {
            const int64_t grid = xm_batched_grid(p->xmjobs.data(), (int32_t)p->xmjobs.size());
            if ((e = launch_xm_batched(p->d_xmjobs, (int32_t)p->xmjobs.size(), grid, s)) != hipSuccess)
                return e;
        }
    }
    if (parts & 1) {
        const int64_t cap = (int64_t)p->num_cus * p->tun.x_grid_per_cu;
        const int64_t tp = p->x_tiles_pair, tn = p->x_tiles - p->x_tiles_pair;
        if (tp > 0 && (e = launch_dirty_map_batched(p->d_xjobs, p->nx_pair, tp, std::min(tp, cap), true, s)) !=
                          hipSuccess)
            return e;
        const int32_t nn = (int32_t)p->xjobs.size() - p->nx_pair;
        if (tn > 0 && (e = launch_dirty_map_batched(p->d_xjobs + p->nx_pair, nn, tn, std::min(tn, cap), false, s)) !=
                          hipSuccess)
            return e;
    }
    if ((parts & 2) && p->b_wgs > 0) {
        // 0 workgroups per CU: one workgroup per tile group, no persistent loop
        int64_t grid = p->tun.beam_grid_per_cu > 0
                           ? std::min<int64_t>(p->b_wgs, (int64_t)p->num_cus * p->tun.beam_grid_per_cu)
                           : p->b_wgs;
        grid = (grid + 7) / 8 * 8;
        if ((e = launch_beam_gemm_batched(p->d_bjobs, (int32_t)p->bjobs.size(), p->b_wgs, grid, p->tun.beam_shape,
                                          s)) != hipSuccess)
            return e;
    }
    if (parts & 4) {
        // the same broadband forms as sgwb_make_maps_band, so the bits agree
        for (size_t i = 0; i < p->jobs.size(); ++i) {
            const sgwb_job &j = p->jobs[i];
            if (!j.Xbb && !j.Gbb) continue;
            char *ws = reinterpret_cast<char *>(p->band_ws) + p->band_off[i];
            size_t xpart = 0;
            if (j.Xbb) {
                if (p->use_xm[i]) {
                    xpart = (size_t)xm_band_rows(p->args[i]) * j.npix * sizeof(double);
                    e = launch_band_partial_finish(reinterpret_cast<double *>(ws), xm_band_rows(p->args[i]), j.npix,
                                                   j.Xbb, s);
                } else {
                    e = launch_band<float>(j.X, nullptr, nullptr, j.nf, j.npix, j.band_lo, j.band_hi, j.Xbb, nullptr,
                                           nullptr, 0, s);
                }
                if (e != hipSuccess) return e;
            }
            if (j.Gbb) {
                double *scratch = reinterpret_cast<double *>(ws + (xpart + 255) / 256 * 256);
                e = launch_band_gamma(j.w, j.ldc, j.nt, j.H, j.band_lo, j.band_hi, j.gamma, j.npix, scratch, j.Gbb, s);
                if (e != hipSuccess) return e;
            }
        }
    }
    return hipGetLastError();
}

// The whole plan.  Branched schedule: the beams go on a second stream forked
// from s (an event) and joined back before the broadband sums, so they can
// run beside the dirty maps; under capture the fork becomes two graph branches.
static hipError_t enqueue_all(sgwb_plan *p, hipStream_t s, int parts)
{
    const bool branch = p->tun.branches && (parts & 3) == 3 && !p->bjobs.empty() &&
                        (p->xm_tiles > 0 || p->x_tiles > 0);
    if (!branch) return enqueue(p, s, parts);
    hipError_t e = hipEventRecord(p->fork, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(p->side, p->fork, 0);
    if (e == hipSuccess) e = enqueue(p, p->side, 2);
    if (e == hipSuccess) e = hipEventRecord(p->join, p->side);
    if (e == hipSuccess) e = enqueue(p, s, 1);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, p->join, 0);
    if (e == hipSuccess && (parts & 4)) e = enqueue(p, s, 4);
    return e;
}

double time_parts(sgwb_plan *p, hipStream_t s, int parts, int reps)
{
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    double best = 1e30;
    for (int r = 0; r < reps; ++r) {
        (void)hipEventRecord(a, s);
        if (enqueue_all(p, s, parts) != hipSuccess) {
            best = -1.0;
            break;
        }
        (void)hipEventRecord(b, s);
        (void)hipEventSynchronize(b);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, a, b);
        best = std::min(best, (double)ms);
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return best;
}

int plan_set_tunables(sgwb_plan *p, const Tunables &t)
{
    p->tun = t;
    return upload_tables(p);
}

std::string plan_signature(const sgwb_plan *p)
{
    // jobs described by what changes the schedule: resolution, segments, strips
    std::string s;
    char buf[96];
    for (const auto &x : p->xjobs) {
        snprintf(buf, sizeof buf, "x%lld.%d.%lld;", (long long)x.a.npix, x.a.nt, (long long)x.nstrips);
        s += buf;
    }
    for (const auto &x : p->xmjobs) {
        snprintf(buf, sizeof buf, "m%lld.%d.%lld;", (long long)x.x.a.npix, x.x.a.nt, (long long)x.x.nstrips);
        s += buf;
    }
    for (const auto &b : p->bjobs) {
        snprintf(buf, sizeof buf, "b%lld.%lld.%lld;", (long long)b.fm.nblk, (long long)b.fn.nblk, (long long)b.fm.nks);
        s += buf;
    }
    return s;
}

// Pick the tunables: from the cache, by timing the candidates on the device, or
// the defaults when tuning is off.
int autotune_plan(sgwb_plan *p, bool tune)
{
    Tunables t;
    p->tune_key = device_key() + ":" + plan_signature(p);
    if (!tune) return plan_set_tunables(p, t);
    if (tune_cache_load(p->tune_key, &t)) {
        p->tuned = true;
        p->from_cache = true;
        return plan_set_tunables(p, t);
    }
    hipStream_t s = p->cap;
    int rc;
    // dirty map: tile order x persistent grid
    Tunables best = t;
    double best_ms = 1e30;
    if (!p->xjobs.empty()) {
        for (int order = 1; order >= 0; --order)
            for (int g : {2, 4, 8}) {
                Tunables c = best;
                c.x_strip_major = order;
                c.x_grid_per_cu = g;
                if ((rc = plan_set_tunables(p, c))) return rc;
                const double ms = time_parts(p, s, 1, 1);
                if (ms < 0) return check_hip(hipGetLastError(), "autotune: dirty-map launch");
                p->tune_ms.push_back(ms);
                if (ms < best_ms) {
                    best_ms = ms;
                    best.x_strip_major = order;
                    best.x_grid_per_cu = g;
                }
            }
    }
    if (!p->xmjobs.empty()) {
        // matrix-core dirty maps: one multi-job launch, or the single-call kernel per job
        best_ms = 1e30;
        int pick = 0;
        for (int per_job : {0, 1}) {
            Tunables c = best;
            c.xm_per_job = per_job;
            if ((rc = plan_set_tunables(p, c))) return rc;
            const double ms = time_parts(p, s, 1, 1);
            if (ms < 0) return check_hip(hipGetLastError(), "autotune: dirty-map launch");
            p->tune_ms.push_back(ms);
            if (ms < best_ms) {
                best_ms = ms;
                pick = per_job;
            }
        }
        best.xm_per_job = pick;
    }
    if (!p->bjobs.empty()) {
        best_ms = 1e30;
        Tunables bb = best;
        for (int shape : {kBeamShape2x4, kBeamShape4x4})
            for (int g : {2, 4, 8, 0}) {
                Tunables c = best;
                c.beam_shape = shape;
                c.beam_grid_per_cu = g;
                if ((rc = plan_set_tunables(p, c))) return rc;
                const double ms = time_parts(p, s, 2, 1);
                if (ms < 0) return check_hip(hipGetLastError(), "autotune: beam launch");
                p->tune_ms.push_back(ms);
                if (ms < best_ms) {
                    best_ms = ms;
                    bb.beam_shape = shape;
                    bb.beam_grid_per_cu = g;
                }
            }
        best = bb;
    }
    if (!p->bjobs.empty() && (p->xm_tiles > 0 || p->x_tiles > 0)) {
        // the whole plan, sequential or with the beams on a branch of their own
        best_ms = 1e30;
        int pick = 0;
        for (int br : {0, 1}) {
            Tunables c = best;
            c.branches = br;
            if ((rc = plan_set_tunables(p, c))) return rc;
            const double ms = time_parts(p, s, 7, 2);
            if (ms < 0) return check_hip(hipGetLastError(), "autotune: whole plan");
            p->tune_ms.push_back(ms);
            if (ms < best_ms) {
                best_ms = ms;
                pick = br;
            }
        }
        best.branches = pick;
    }
    p->tuned = true;
    tune_cache_store(p->tune_key, best);
    return plan_set_tunables(p, best);
}

}  // namespace sgwb

static void plan_free(sgwb_plan *p)
{
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->cap) (void)hipStreamDestroy(p->cap);
    if (p->side) (void)hipStreamDestroy(p->side);
    if (p->fork) (void)hipEventDestroy(p->fork);
    if (p->join) (void)hipEventDestroy(p->join);
    if (p->d_xjobs) (void)hipFree(p->d_xjobs);
    if (p->d_xmjobs) (void)hipFree(p->d_xmjobs);
    if (p->xm_ws) (void)hipFree(p->xm_ws);
    if (p->d_bjobs) (void)hipFree(p->d_bjobs);
    if (p->beam_ws) (void)hipFree(p->beam_ws);
    if (p->band_ws) (void)hipFree(p->band_ws);
    delete p;
}

extern "C" {

int sgwb_plan_create(const sgwb_job *jobs, int32_t njobs, uint32_t flags, sgwb_plan **out)
{
    if (!out) return set_error(SGWB_EINVAL, "plan_create: null out");
    *out = nullptr;
    if (!jobs || njobs < 1 || njobs > 4096) return set_error(SGWB_EINVAL, "plan_create: need 1..4096 jobs");
    if (flags & ~(SGWB_PLAN_AUTOTUNE | SGWB_PLAN_NO_GRAPH)) return set_error(SGWB_EINVAL, "plan_create: unknown flags");
    sgwb_plan *p = new sgwb_plan();
    int rc = SGWB_OK;
    p->jobs.assign(jobs, jobs + njobs);
    p->args.resize(njobs);
    for (int i = 0; i < njobs && !rc; ++i) rc = validate_job(p->jobs[i], &p->args[i]);
    if (rc) {
        plan_free(p);
        return rc;
    }
    (void)hipGetDevice(&p->device);
    (void)hipDeviceGetAttribute(&p->num_cus, hipDeviceAttributeMultiprocessorCount, p->device);
    if (p->num_cus <= 0) p->num_cus = 256;

    // workspaces
    std::vector<size_t> beam_off(njobs, 0), xm_off(njobs, 0);
    std::vector<bool> use_xm(njobs, false);
    p->band_off.assign(njobs, 0);
    p->use_xm.assign(njobs, 0);
    for (int i = 0; i < njobs; ++i) {
        const sgwb_job &j = p->jobs[i];
        if (j.X && xm_eligible(p->args[i]) && !(j.flags & SGWB_MAPS_VALU_X)) {
            use_xm[i] = true;
            p->use_xm[i] = 1;
            xm_off[i] = p->xm_bytes;
            p->xm_bytes += (xm_workspace_bytes(j.k0, j.nt, j.nf, j.npix) + 255) / 256 * 256;
        }
        if (j.Gam) {
            beam_off[i] = p->beam_bytes;
            const int64_t ncol = p->args[i].nside > 0 ? j.npix / 2 : j.npix;
            p->beam_bytes += (beam_workspace_bytes(j.nt, j.nf, (int32_t)ncol) + 255) / 256 * 256;
        }
        if (j.Xbb || j.Gbb) {
            p->band_off[i] = p->band_bytes;
            size_t n = 0;
            if (j.Xbb && use_xm[i]) n += (size_t)xm_band_rows(p->args[i]) * j.npix * sizeof(double);
            n = (n + 255) / 256 * 256;
            if (j.Gbb) n += band_gamma_scratch_bytes(j.nt, j.npix);
            p->band_bytes += (n + 255) / 256 * 256;
        }
    }
    hipError_t e = hipSuccess;
    if (p->beam_bytes) e = hipMalloc(&p->beam_ws, p->beam_bytes);
    if (e == hipSuccess && p->band_bytes) e = hipMalloc(&p->band_ws, p->band_bytes);
    if (e == hipSuccess && p->xm_bytes) e = hipMalloc(&p->xm_ws, p->xm_bytes);
    if (e != hipSuccess) {
        rc = set_error(SGWB_ENOMEM, "plan_create: workspace allocation failed: %s", hipGetErrorString(e));
        plan_free(p);
        return rc;
    }
    // job tables: longest jobs (most segments) first
    std::vector<int> order(njobs);
    for (int i = 0; i < njobs; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return p->jobs[x].nt > p->jobs[y].nt; });
    for (int pass = 0; pass < 2; ++pass)
        for (int i : order) {
            const sgwb_job &j = p->jobs[i];
            const bool pair = p->args[i].nside > 0;
            if (j.X && !use_xm[i] && pair == (pass == 0)) {
                XJob x;
                fill_xjob(&x, p->args[i], j.C, j.w, j.gamma, j.tau, j.X, true);
                p->xjobs.push_back(x);
                if (pair) p->nx_pair++;
            }
        }
    for (int i : order) {
        const sgwb_job &j = p->jobs[i];
        if (use_xm[i]) {
            XmJob x;
            fill_xmjob(&x, p->args[i], j.C, j.w, j.gamma, j.tau, j.X, reinterpret_cast<char *>(p->xm_ws) + xm_off[i]);
            if (j.Xbb) {  // the tiles write per-strip band sums
                x.x.a.band_part = reinterpret_cast<double *>(reinterpret_cast<char *>(p->band_ws) + p->band_off[i]);
                x.x.a.band_lo = j.band_lo;
                x.x.a.band_hi = j.band_hi;
            }
            p->xmjobs.push_back(x);
        }
        if (j.Gam) {
            BJob b;
            fill_bjob(&b, p->args[i], j.w, j.gamma, j.Gam, reinterpret_cast<char *>(p->beam_ws) + beam_off[i]);
            p->bjobs.push_back(b);
        }
    }
    if (!p->xjobs.empty()) e = hipMalloc(&p->d_xjobs, p->xjobs.size() * sizeof(XJob));
    if (e == hipSuccess && !p->xmjobs.empty()) e = hipMalloc(&p->d_xmjobs, p->xmjobs.size() * sizeof(XmJob));
    if (e == hipSuccess && !p->bjobs.empty()) e = hipMalloc(&p->d_bjobs, p->bjobs.size() * sizeof(BJob));
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->join, hipEventDisableTiming);
    if (e != hipSuccess) {
        rc = set_error(SGWB_EDEVICE, "plan_create: %s", hipGetErrorString(e));
        plan_free(p);
        return rc;
    }

    // tunables
    rc = autotune_plan(p, (flags & SGWB_PLAN_AUTOTUNE) != 0);
    if (rc) {
        plan_free(p);
        return rc;
    }

    if (!(flags & SGWB_PLAN_NO_GRAPH)) {
        e = hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipError_t qe = enqueue_all(p, p->cap, 7);
            e = hipStreamEndCapture(p->cap, &p->graph);
            if (qe != hipSuccess) e = qe;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            rc = set_error(SGWB_EDEVICE, "plan_create: graph capture failed: %s", hipGetErrorString(e));
            plan_free(p);
            return rc;
        }
    }
    *out = p;
    return SGWB_OK;
}

int sgwb_plan_launch(sgwb_plan *p, hipStream_t stream)
{
    if (!p) return set_error(SGWB_EINVAL, "plan_launch: null plan");
    if (p->exec) return check_hip(hipGraphLaunch(p->exec, stream), "plan_launch: hipGraphLaunch");
    return check_hip(enqueue_all(p, stream, 7), "plan_launch: enqueue");
}

void sgwb_plan_destroy(sgwb_plan *p) { plan_free(p); }

int sgwb_plan_describe(const sgwb_plan *p, char *buf, size_t len)
{
    if (!p || !buf || len == 0) return set_error(SGWB_EINVAL, "plan_describe: bad arguments");
    std::string ms;
    for (size_t i = 0; i < p->tune_ms.size(); ++i) {
        char b[32];
        snprintf(b, sizeof b, "%s%.4f", i ? ", " : "", p->tune_ms[i]);
        ms += b;
    }
    int n = snprintf(buf, len,
                     "{\"jobs\": %zu, \"x_tiles\": %lld, \"xm_tiles\": %lld, \"beam_workgroups\": %lld, \"x_strip_major\": %d, "
                     "\"x_grid_per_cu\": %d, \"xm_per_job\": %d, \"beam_shape\": \"%s\", \"beam_grid_per_cu\": %d, "
                     "\"branches\": %d, \"tuned\": %s, "
                     "\"from_cache\": %s, \"tune_ms\": [%s], \"graph\": %s, \"key\": \"%s\"}",
                     p->jobs.size(), (long long)p->x_tiles, (long long)p->xm_tiles, (long long)p->b_wgs, p->tun.x_strip_major,
                     p->tun.x_grid_per_cu, p->tun.xm_per_job, p->tun.beam_shape == kBeamShape2x4 ? "2x4" : "4x4",
                     p->tun.beam_grid_per_cu, p->tun.branches,
                     p->tuned ? "true" : "false", p->from_cache ? "true" : "false", ms.c_str(),
                     p->exec ? "true" : "false", p->tune_key.c_str());
    if (n < 0 || (size_t)n >= len) return set_error(SGWB_ENOMEM, "plan_describe: buffer too small");
    return SGWB_OK;
}

}  // extern "C"
