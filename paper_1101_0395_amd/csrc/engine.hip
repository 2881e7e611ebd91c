// Serving engine: continuous batching of whole-quantizer jobs.  Jobs join and
// leave the set in flight between steps; every step drives the same batched
// phases as cq_quantize_batch (histogram and initialization of the newly
// admitted jobs, Lloyd iterations of all jobs in flight, palette and pixel map
// of the jobs that stopped).  Each job keeps all of its device state in its
// own pool slot and each kernel's work for a job depends only on that job,
// so a job's results do not depend on what else is in flight.
#include <stdio.h>

#include <deque>
#include <new>
#include <utility>
#include <vector>

#include "batch.h"
#include "pool.h"

namespace cq {

struct EngineJob {
    int64_t ticket = 0;
    cq_job spec{};
    size_t off = 0;     // slot offset in the pool
    size_t bytes = 0;   // slot size
    JobDev dev{};       // descriptor (pointers into the slot)
    int32_t it = 0;     // iterations enqueued since admission
};

}  // namespace cq

struct cq_engine {
    int32_t max_jobs = 0;
    char* desc = nullptr;       // descriptor region for max_jobs jobs
    char* pool_base = nullptr;  // slots
    cq::ExtentPool pool;
    hipStream_t s = nullptr;
    bool failed = false;
    int64_t next_ticket = 1;
    std::deque<cq::EngineJob> queue;   // submitted, waiting for a slot
    std::vector<cq::EngineJob> active;  // in flight, in admission order
    std::deque<cq::HostBuf> staged;  // upload snapshots of a finished phase, kept until the stream drains
};

namespace cq {

static size_t engine_desc_bytes(int32_t max_jobs) { return align256(desc_bytes(max_jobs)); }

// Moves queued jobs into the set in flight while the oldest one fits; returns
// the indices (into e->active) of the jobs admitted.
static std::vector<int> engine_admit(cq_engine* e)
{
    std::vector<int> fresh;
    while (!e->queue.empty() && int32_t(e->active.size()) < e->max_jobs) {
        EngineJob& q = e->queue.front();
        size_t off = 0;
        if (!e->pool.alloc(q.bytes, &off)) break;
        q.off = off;
        const cq_job& j = q.spec;
        fill_quantize_job(q.dev, j.img, j.H, j.W, j.row_stride_bytes, j.subsample, j.K, int(j.scheme), j.seed, j.max_iters,
                          j.tol, j.prune, j.palette, j.out_idx, j.out_rgb, e->pool_base + off);
        q.it = 0;
        fresh.push_back(int(e->active.size()));
        e->active.push_back(q);
        e->queue.pop_front();
    }
    return fresh;
}

// Histogram, initialization and k-means set-up of the jobs just admitted.
static cq_status engine_prefill(cq_engine* e, const std::vector<int>& fresh)
{
    Batch b(int(fresh.size()), e->desc, e->s);
    for (int i = 0; i < b.B; ++i) b.h[i] = e->active[fresh[i]].dev;
    CQ_TRY(run_histogram(b));
    CQ_TRY(collect(b));
    std::vector<int64_t> n(size_t(b.B));
    for (int i = 0; i < b.B; ++i) n[i] = b.res[i].n_unique;
    set_counts(b, n);
    CQ_TRY(run_init(b));  // leaves the final descriptors uploaded
    CQ_TRY(launch_kmeans_begin(b.d_jobs(), b.B, b.s));
    for (int i = 0; i < b.B; ++i) e->active[fresh[i]].dev = b.h[i];
    for (auto& v : b.staged) e->staged.push_back(std::move(v));  // copies may still be pending
    return CQ_OK;
}

// `iters` iterations of every job in flight, each at its own iteration
// number: a job's first iteration is a full search, later ones of a pruned
// job walk the sorted table; a pruned job's update regroups its records on
// the iterations that the device-side schedule regroups.  A job that has
// stopped on the device keeps its blocks until the host learns of it; they
// return at once.
static cq_status engine_iterate(cq_engine* e, Batch& d, int32_t iters)
{
    const int B = d.B;
    auto iterating = [&](int j) {
        const EngineJob& x = e->active[j];
        return x.dev.n > x.dev.K && x.it < x.dev.max_iters;
    };
    auto assign_blocks = [&](int j) {
        const JobDev& J = e->active[j].dev;
        return iterating(j) ? int((J.n + J.chunk - 1) / J.chunk) : 0;
    };
    bool uploaded = false;
    std::vector<int> sent;
    for (int32_t q = 0; q < iters; ++q) {
        const int full = d.set_map(kMapAssignFull, [&](int j) {
            const EngineJob& x = e->active[j];
            return (x.it == 0 || !x.dev.prune) ? assign_blocks(j) : 0;
        });
        const int walk = d.set_map(kMapAssignWalk, [&](int j) {
            const EngineJob& x = e->active[j];
            return (x.it > 0 && x.dev.prune) ? assign_blocks(j) : 0;
        });
        const int update = d.set_map(kMapUpdate, [&](int j) {
            if (!iterating(j)) return 0;
            const EngineJob& x = e->active[j];
            const bool regroup = x.dev.prune && regroup_at(x.it + 1, x.dev.regroup_period);
            return update_table_blocks(x.dev.K, x.dev.prune) + (regroup ? int(regroup_blocks(x.dev.n, x.dev.chunk)) : 0);
        });
        if (full + walk == 0) break;
        if (!uploaded || d.maps != sent) {
            CQ_TRY(upload(d));
            sent = d.maps;
            uploaded = true;
        }
        CQ_TRY(launch_kmeans_iter(d.d_jobs(), d.d_maps(), B, false, 0, full, walk, update, true, 0, d.s));
        for (int j = 0; j < B; ++j)
            if (iterating(j)) ++e->active[j].it;
    }
    if (!uploaded) CQ_TRY(upload(d));  // the descriptors the control-block readback uses
    return CQ_OK;
}

// Palette, pixel map and statistics of the jobs that stopped; their slots
// return to the pool.
static cq_status engine_finish(cq_engine* e, const Batch& d, cq_engine_done* done, int32_t* n_done)
{
    std::vector<int> fin;
    for (int j = 0; j < d.B; ++j)
        if (d.res[j].done) fin.push_back(j);
    *n_done = 0;
    if (fin.empty()) return CQ_OK;
    Batch f(int(fin.size()), e->desc, e->s);
    for (int i = 0; i < f.B; ++i) f.h[i] = e->active[fin[i]].dev;
    CQ_TRY(upload(f));
    CQ_TRY(launch_palette(f.d_jobs(), f.B, f.s));
    CQ_TRY(run_map(f, true, true));
    CQ_TRY(collect(f));
    for (int i = 0; i < f.B; ++i) {
        const EngineJob& x = e->active[fin[i]];
        cq_engine_done& o = done[i];
        memset(&o, 0, sizeof o);
        o.ticket = x.ticket;
        o.status = f.res[i].sync_error ? CQ_EDEVICE : f.res[i].bad_input ? CQ_EINVAL : CQ_OK;
        fill_stats(f.h[i], f.res[i], o.stats, true);
        e->pool.release(x.off, x.bytes);
    }
    *n_done = f.B;
    std::vector<EngineJob> keep;
    keep.reserve(e->active.size() - fin.size());
    size_t k = 0;
    for (int j = 0; j < d.B; ++j) {
        if (k < fin.size() && fin[k] == j) {
            ++k;
            continue;
        }
        keep.push_back(e->active[j]);
    }
    e->active.swap(keep);
    return CQ_OK;
}

static cq_status engine_step(cq_engine* e, int32_t iters, cq_engine_done* done, int32_t* n_done)
{
    const std::vector<int> fresh = engine_admit(e);
    if (!fresh.empty()) CQ_TRY(engine_prefill(e, fresh));
    if (e->active.empty()) return CQ_OK;
    Batch d(int(e->active.size()), e->desc, e->s);
    for (int j = 0; j < d.B; ++j) d.h[j] = e->active[j].dev;
    CQ_TRY(engine_iterate(e, d, iters));
    CQ_TRY(collect(d));
    e->staged.clear();  // the stream has drained
    return engine_finish(e, d, done, n_done);
}

}  // namespace cq

using namespace cq;

extern "C" {

size_t cq_engine_job_bytes(int32_t H, int32_t W)
{
    if (H <= 0 || W <= 0 || int64_t(H) * W > kMaxPixels) return 0;
    cq_job j{};
    j.H = H;
    j.W = W;
    return slot_bytes(j);
}

size_t cq_engine_workspace_bytes(int32_t max_jobs, size_t pool_bytes)
{
    if (max_jobs < 1 || max_jobs > kMaxBatch) return 0;
    return engine_desc_bytes(max_jobs) + align256(pool_bytes);
}

cq_status cq_engine_create(int32_t max_jobs, void* ws, size_t ws_bytes, void* stream, cq_engine** engine)
{
    clear_error();
    if (!engine) return einval("engine is null");
    *engine = nullptr;
    if (max_jobs < 1 || max_jobs > kMaxBatch) return einval("max_jobs = %d outside [1, %d]", max_jobs, kMaxBatch);
    const size_t head = engine_desc_bytes(max_jobs);
    CQ_TRY(check_ws(ws, ws_bytes, head));
    cq_engine* e = new (std::nothrow) cq_engine;
    if (!e) {
        set_error("out of host memory");
        return CQ_EDEVICE;
    }
    e->max_jobs = max_jobs;
    e->desc = static_cast<char*>(ws);
    e->pool_base = static_cast<char*>(ws) + head;
    e->pool = ExtentPool(ws_bytes - head, 256);
    e->s = static_cast<hipStream_t>(stream);
    *engine = e;
    return CQ_OK;
}

cq_status cq_engine_submit(cq_engine* e, const cq_job* job, int64_t* ticket)
{
    clear_error();
    if (!e || !job || !ticket) return einval("engine/job/ticket is null");
    if (e->failed) {
        set_error("the engine stopped after a device error");
        return CQ_EDEVICE;
    }
    CQ_TRY(check_job(*job, 0));
    EngineJob q;
    q.spec = *job;
    q.bytes = slot_bytes(*job);
    if (e->pool.round(q.bytes) > e->pool.total()) {
        set_error("job needs %zu pool bytes, the pool has %zu", q.bytes, e->pool.total());
        return CQ_ECAPACITY;
    }
    q.ticket = e->next_ticket++;
    *ticket = q.ticket;
    e->queue.push_back(q);
    return CQ_OK;
}

cq_status cq_engine_step(cq_engine* e, int32_t iters, cq_engine_done* done, int32_t capacity, int32_t* n_done)
{
    clear_error();
    if (!e || !done || !n_done) return einval("engine/done/n_done is null");
    *n_done = 0;
    if (e->failed) {
        set_error("the engine stopped after a device error");
        return CQ_EDEVICE;
    }
    if (iters < 0 || iters > kMaxIters) return einval("iters = %d outside [0, %d]", iters, kMaxIters);
    if (capacity < e->max_jobs) return einval("capacity %d < max_jobs %d", capacity, e->max_jobs);
    const cq_status st = engine_step(e, iters, done, n_done);
    if (st != CQ_OK) e->failed = true;  // the jobs in flight are in an unknown state
    return st;
}

cq_status cq_engine_pending(const cq_engine* e, int32_t* queued, int32_t* running, size_t* pool_used)
{
    clear_error();
    if (!e) return einval("engine is null");
    if (queued) *queued = int32_t(e->queue.size());
    if (running) *running = int32_t(e->active.size());
    if (pool_used) *pool_used = e->pool.used();
    return CQ_OK;
}

void cq_engine_destroy(cq_engine* e)
{
    if (!e) return;
    if (!e->staged.empty()) (void)hipStreamSynchronize(e->s);  // after a failed step: let pending copies end
    delete e;
}

}  // extern "C"
