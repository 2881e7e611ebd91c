// C-ABI entry points of libcq: argument validation, workspace carving, the
// batch descriptors every kernel reads, and the host side of the iteration
// loop.  The single-image calls run as batches of one job.
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <deque>
#include <map>
#include <mutex>
#include <vector>

#include "batch.h"

namespace cq {

// ---------------------------------------------------------------- errors
static thread_local char g_error[512];

void set_error(const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_error, sizeof g_error, fmt, ap);
    va_end(ap);
}

void clear_error() { g_error[0] = '\0'; }

cq_status check_launch(const char* what)
{
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("%s launch failed: %s", what, hipGetErrorString(e));
        return CQ_EDEVICE;
    }
    return CQ_OK;
}

cq_status einval(const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_error, sizeof g_error, fmt, ap);
    va_end(ap);
    return CQ_EINVAL;
}

// ---------------------------------------------------------------- kernel timer
struct KernelTimer {
    bool enabled = false;
    bool armed = false;  // the current launch is bracketed
    char name[64] = {0};
    int32_t capacity = 0;
    int32_t used = 0;
    int32_t every = 1;
    int64_t seen = 0;
    hipEvent_t* start = nullptr;
    hipEvent_t* stop = nullptr;
};
static KernelTimer g_timer;

void timer_begin(const char* kernel, hipStream_t s)
{
    if (!g_timer.enabled || strcmp(kernel, g_timer.name) != 0) return;
    g_timer.armed = g_timer.seen++ % g_timer.every == 0 && g_timer.used < g_timer.capacity;
    if (g_timer.armed) (void)hipEventRecord(g_timer.start[g_timer.used], s);
}

void timer_end(const char* kernel, hipStream_t s)
{
    if (!g_timer.enabled || !g_timer.armed || strcmp(kernel, g_timer.name) != 0) return;
    (void)hipEventRecord(g_timer.stop[g_timer.used], s);
    ++g_timer.used;
    g_timer.armed = false;
}

static void timer_release()
{
    for (int32_t i = 0; i < g_timer.capacity; ++i) {
        (void)hipEventDestroy(g_timer.start[i]);
        (void)hipEventDestroy(g_timer.stop[i]);
    }
    delete[] g_timer.start;
    delete[] g_timer.stop;
    g_timer = KernelTimer{};
}

// ---------------------------------------------------------------- checks
static cq_status check_image(const uint8_t* img, int32_t H, int32_t W, int64_t row_stride)
{
    if (!img) return einval("img is null");
    if (H <= 0 || W <= 0) return einval("image size %d x %d must be positive", H, W);
    if (int64_t(H) * W > kMaxPixels) return einval("image has more than 2^28 pixels");
    if (row_stride < 3 * int64_t(W)) return einval("row stride %lld < 3 W", (long long)row_stride);
    return CQ_OK;
}

static cq_status check_subsample(int32_t subsample)
{
    if (subsample != 0 && subsample != 1) return einval("subsample = %d is not 0 or 1", subsample);
    return CQ_OK;
}

cq_status check_ws(const void* ws, size_t ws_bytes, size_t need)
{
    if (!ws) {
        set_error("workspace is null");
        return CQ_EWORKSPACE;
    }
    if ((reinterpret_cast<uintptr_t>(ws) & 255u) != 0) {
        set_error("workspace must be 256-byte aligned");
        return CQ_EWORKSPACE;
    }
    if (ws_bytes < need) {
        set_error("workspace has %zu bytes, %zu needed", ws_bytes, need);
        return CQ_EWORKSPACE;
    }
    return CQ_OK;
}

static cq_status check_k(int32_t K)
{
    if (K < 1 || K > kMaxK) return einval("K = %d outside [1, 256]", K);
    return CQ_OK;
}

static cq_status check_iters_tol(int32_t max_iters, double tol)
{
    if (max_iters < 1 || max_iters > kMaxIters) return einval("max_iters = %d outside [1, %d]", max_iters, kMaxIters);
    if (!(tol >= 0.0) || tol > 1e300) return einval("tol must be a finite value >= 0");
    return CQ_OK;
}

// ---------------------------------------------------------------- batches
// Points the workspace-backed fields of a job at one slot with layout L.
static void bind_slot(JobDev& J, char* slot, const Layout& L)
{
    J.lut = to_dev(reinterpret_cast<uint8_t*>(slot + L.lut));
    J.meta = to_dev(reinterpret_cast<Meta*>(slot + L.meta));
    J.trace = to_dev(reinterpret_cast<double*>(slot + L.trace));
    J.rec = to_dev(reinterpret_cast<Rec*>(slot + L.rec));
    J.prow = to_dev(reinterpret_cast<uint32_t*>(slot + L.prow));
    J.ord = to_dev(reinterpret_cast<uint8_t*>(slot + L.ord));
    J.sums = to_dev(reinterpret_cast<unsigned long long*>(slot + L.sums));
    J.cprev = to_dev(reinterpret_cast<double*>(slot + L.cprev));
    J.hkeys = to_dev(reinterpret_cast<uint16_t*>(slot + L.hkeys));
    J.hk2 = to_dev(reinterpret_cast<uint16_t*>(slot + L.hk2));
    J.hcnt = to_dev(reinterpret_cast<uint32_t*>(slot + L.hcnt));
    J.hmat = to_dev(reinterpret_cast<uint32_t*>(slot + L.hmat));
    J.hnu = to_dev(reinterpret_cast<uint32_t*>(slot + L.hnu));
    J.hbs = to_dev(reinterpret_cast<uint32_t*>(slot + L.hbs));
    J.part = to_dev(reinterpret_cast<unsigned long long*>(slot + L.part));
    J.vals = to_dev(reinterpret_cast<uint64_t*>(slot + L.chunks));
    J.d2 = to_dev(reinterpret_cast<uint32_t*>(slot + L.work));
    J.grp = to_dev(reinterpret_cast<uint64_t*>(slot + L.work));
}

// The image, and the view of it that the histogram counts: all of it, or with
// subsampling its pixels at even row and column (ceil(H/2) x ceil(W/2) pixels,
// twice the row and pixel steps).
static void set_image(JobDev& J, const uint8_t* img, int32_t H, int32_t W, int64_t stride, bool subsample)
{
    J.img = to_dev(img);
    J.H = H;
    J.W = W;
    J.stride = stride;
    J.packed = (stride == 3 * int64_t(W) && (reinterpret_cast<uintptr_t>(img) & 3u) == 0) ? 1 : 0;
    J.hH = subsample ? (H + 1) / 2 : H;
    J.hW = subsample ? (W + 1) / 2 : W;
    J.hstride = subsample ? 2 * stride : stride;
    J.hpitch = subsample ? 6 : 3;
    J.hpacked = subsample ? 0 : J.packed;
    J.map_direct = subsample ? 1 : 0;
}

// ------------------------------------------------------------ host buffers
namespace {
constexpr int kHostClasses = 24;  // size classes 1 KiB << c

// Never destroyed, so a buffer released during process exit (an engine freed
// late) still finds its list.
struct HostPool {
    std::mutex mu;
    std::vector<void*> free_list[kHostClasses];
};
HostPool& host_pool()
{
    static HostPool* pool = new HostPool;
    return *pool;
}

int host_class(size_t n)
{
    int c = 0;
    while (c < kHostClasses && (size_t(1024) << c) < n) ++c;
    return c;
}
}  // namespace

HostBuf::HostBuf(size_t n)
{
    const int c = host_class(n);
    if (c < kHostClasses) {
        cap_ = size_t(1024) << c;
        {
            HostPool& pool = host_pool();
            std::lock_guard<std::mutex> lock(pool.mu);
            if (!pool.free_list[c].empty()) {
                p_ = pool.free_list[c].back();
                pool.free_list[c].pop_back();
                pinned_ = true;
                return;
            }
        }
        if (hipHostMalloc(&p_, cap_, hipHostMallocDefault) == hipSuccess) {
            pinned_ = true;
            return;
        }
        (void)hipGetLastError();  // fall back to pageable memory
        p_ = nullptr;
    }
    cap_ = n;
    p_ = malloc(n);
    pinned_ = false;
}

void HostBuf::release()
{
    if (!p_) return;
    if (pinned_) {
        HostPool& pool = host_pool();
        std::lock_guard<std::mutex> lock(pool.mu);
        pool.free_list[host_class(cap_)].push_back(p_);
    } else {
        free(p_);
    }
    p_ = nullptr;
}

// Copies the job descriptors and block maps to the device in one copy, laid
// out as in the descriptor region.  Each upload reads its own host snapshot,
// which outlives the asynchronous copy.
cq_status upload(Batch& b)
{
    const size_t jb = sizeof(JobDev) * size_t(b.B), mo = desc_maps_off(b.B), mb = sizeof(int) * b.maps.size();
    char* snap = nullptr;
    if (b.host_stage) {
        if (mo + mb > b.host_stage_bytes) {
            set_error("descriptor upload of %zu bytes exceeds the host staging area", mo + mb);
            return CQ_EDEVICE;
        }
        snap = b.host_stage;
    } else {
        b.staged.emplace_back(mo + mb);
        snap = b.staged.back().data();
    }
    if (!snap) {
        set_error("out of host memory");
        return CQ_EDEVICE;
    }
    memcpy(snap, b.h.data(), jb);
    memset(snap + jb, 0, mo - jb);
    memcpy(snap + mo, b.maps.data(), mb);
    CQ_HIP_TRY(hipMemcpyAsync(b.desc, snap, mo + mb, hipMemcpyHostToDevice, b.s));
    return CQ_OK;
}

__global__ void k_collect(const JobDev* __restrict__ jobs, int B, JobResult* __restrict__ out)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= B) return;
    const Meta* m = gp(jobs[j].meta);
    JobResult r;
    r.n_unique = m->n_unique;
    r.ndc = m->ndc;
    r.near_ties = m->near_ties;
    r.sq_err = m->sq_err;
    r.total_w = m->total_w;
    r.sse_last = m->sse_last;
    r.done = m->done;
    r.iters = m->iters;
    r.converged = m->converged;
    r.bad_input = m->bad_input;
    r.sync_error = m->sync_error;
    r.pad_ = 0;
    out[j] = r;
}

__global__ void k_zero_sq_err(const JobDev* __restrict__ jobs, int B)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < B) gp(jobs[j].meta)->sq_err = 0;
}

// Gathers every job's control block into b.res (synchronizes the stream).
cq_status collect(Batch& b)
{
    CQ_TIMED_LAUNCH("k_collect", b.s, k_collect<<<(b.B + 63) / 64, 64, 0, b.s>>>(b.d_jobs(), b.B, b.d_results()));
    const size_t rb = sizeof(JobResult) * size_t(b.B);
    if (b.host_stage) {
        if (rb > b.host_stage_bytes) {
            set_error("status readback of %zu bytes exceeds the host staging area", rb);
            return CQ_EDEVICE;
        }
        CQ_HIP_TRY(hipMemcpyAsync(b.host_stage, b.d_results(), rb, hipMemcpyDeviceToHost, b.s));
        CQ_HIP_TRY(hipStreamSynchronize(b.s));
        memcpy(b.res.data(), b.host_stage, rb);
        return CQ_OK;
    }
    HostBuf out(rb);
    if (!out.data()) {
        set_error("out of host memory");
        return CQ_EDEVICE;
    }
    CQ_HIP_TRY(hipMemcpyAsync(out.data(), b.d_results(), rb, hipMemcpyDeviceToHost, b.s));
    CQ_HIP_TRY(hipStreamSynchronize(b.s));
    memcpy(b.res.data(), out.data(), rb);
    b.staged.clear();  // every upload before this point has completed
    return CQ_OK;
}

// Stream (one per device, default priority) for readbacks that must not
// queue behind later work on the caller's stream; destroyed only by
// cq_release_resources.
namespace {
std::mutex g_side_mu;
std::map<int, hipStream_t>& side_streams()
{
    static std::map<int, hipStream_t>* m = new std::map<int, hipStream_t>;
    return *m;
}
}  // namespace

cq_status side_stream(hipStream_t* out)
{
    int dev = 0;
    CQ_HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_side_mu);
    std::map<int, hipStream_t>& streams = side_streams();
    auto it = streams.find(dev);
    if (it == streams.end()) {
        hipStream_t st = nullptr;
        CQ_HIP_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        it = streams.emplace(dev, st).first;
    }
    *out = it->second;
    return CQ_OK;
}

cq_status collect_async(Batch& b, int slot, hipEvent_t done)
{
    CQ_TIMED_LAUNCH("k_collect", b.s, k_collect<<<(b.B + 63) / 64, 64, 0, b.s>>>(b.d_jobs(), b.B, b.d_results(slot)));
    CQ_HIP_TRY(hipEventRecord(done, b.s));
    return CQ_OK;
}

cq_status read_results(Batch& b, int slot, hipEvent_t done)
{
    hipStream_t side = nullptr;
    CQ_TRY(side_stream(&side));
    CQ_HIP_TRY(hipStreamWaitEvent(side, done, 0));
    const size_t rb = sizeof(JobResult) * size_t(b.B);
    if (b.host_stage) {
        // a copy to pageable memory returns once complete; the area is free
        // again before the next upload
        if (rb > b.host_stage_bytes) {
            set_error("status readback of %zu bytes exceeds the host staging area", rb);
            return CQ_EDEVICE;
        }
        CQ_HIP_TRY(hipMemcpyAsync(b.host_stage, b.d_results(slot), rb, hipMemcpyDeviceToHost, side));
        CQ_HIP_TRY(hipStreamSynchronize(side));
        memcpy(b.res.data(), b.host_stage, rb);
        return CQ_OK;
    }
    HostBuf out(rb);
    if (!out.data()) {
        set_error("out of host memory");
        return CQ_EDEVICE;
    }
    CQ_HIP_TRY(hipMemcpyAsync(out.data(), b.d_results(slot), rb, hipMemcpyDeviceToHost, side));
    CQ_HIP_TRY(hipStreamSynchronize(side));
    memcpy(b.res.data(), out.data(), rb);
    return CQ_OK;
}

// Two events without timing, destroyed with the object.
struct EventPair {
    hipEvent_t ev[2] = {nullptr, nullptr};
    cq_status create()
    {
        for (auto& e : ev) CQ_HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        return CQ_OK;
    }
    ~EventPair()
    {
        for (auto e : ev)
            if (e) (void)hipEventDestroy(e);
    }
};

// ---------------------------------------------------------------- phases
cq_status run_histogram(Batch& b)
{
    const int total = b.set_map(kMapHist, [&](int j) { return hist_blocks(hist_pixels(b.h[j])); });
    // Counting blocks: 256 or more per job, so that a few images fill the
    // chip; 64 or more where the batch needs many rounds of resident blocks
    // anyway (about 1024 of them), since a small image's blocks mostly find
    // empty buckets and each block has a fixed cost; the pairs are then
    // emitted four buckets per wave for the same reason.
    int64_t at256 = 0;
    for (const JobDev& J : b.h) at256 += hist_count_blocks(hist_pixels(J), 256);
    const int cmin = at256 >= 8 * 1024 ? 64 : 256;
    const int count = b.set_map(kMapHistCount, [&](int j) { return hist_count_blocks(hist_pixels(b.h[j]), cmin); });
    int64_t max_tiles = 1;
    for (const JobDev& J : b.h) max_tiles = hist_tiles(hist_pixels(J)) > max_tiles ? hist_tiles(hist_pixels(J)) : max_tiles;
    CQ_TRY(upload(b));
    return launch_histogram(b.d_jobs(), b.d_maps(), b.B, total, count, int(max_tiles), cmin == 64 ? 4 : 1, b.s);
}

// Once N' is known (from the histogram or from the caller).
// The launch schedule follows the colours of the jobs that iterate.
void set_counts(Batch& b, const std::vector<int64_t>& n)
{
    int64_t colours = 0;
    for (int j = 0; j < b.B; ++j)
        if (n[j] > b.h[j].K) colours += n[j];
    const cq_schedule sched = schedule_for(colours);
    for (int j = 0; j < b.B; ++j) {
        JobDev& J = b.h[j];
        J.n = n[j];
        J.chunk = assign_chunk(J.n, sched.assign_chunk);
        J.regroup_period = sched.regroup_period;
        J.map_k = int32_t(J.n < J.K ? J.n : J.K);
    }
}

// LBG: the centroid (one iteration of a single centre from zero), then the
// doubling stages, each refined by k-means with the threshold kLbgTol.  The
// jobs still doubling form a batch of their own in the same descriptor
// region; the batch's own descriptors are uploaded again at the end.
static cq_status run_lbg(Batch& b)
{
    std::vector<int> jobs;
    for (int j = 0; j < b.B; ++j)
        if (b.h[j].scheme == CQ_INIT_LBG && b.h[j].n > b.h[j].K) jobs.push_back(j);
    if (jobs.empty()) return CQ_OK;
    std::vector<int32_t> have(jobs.size(), 0);  // centres so far (0: not even the centroid)
    while (true) {
        std::vector<int> act;
        for (size_t i = 0; i < jobs.size(); ++i)
            if (have[i] < b.h[jobs[i]].K) act.push_back(int(i));
        if (act.empty()) break;
        Batch st(int(act.size()), b.desc, b.s);
        st.host_stage = b.host_stage;
        st.host_stage_bytes = b.host_stage_bytes;
        st.fixed_events = b.fixed_events;
        for (int q = 0; q < st.B; ++q) {
            const int i = act[q];
            JobDev J = b.h[jobs[i]];
            const int32_t m = have[i];
            const int32_t next = m == 0 ? 1 : (2 * m <= J.K ? 2 * m : J.K);
            J.init_C = m;
            J.K = next;
            J.prune = m == 0 ? 0 : 1;
            J.max_iters = m == 0 ? 1 : kLbgMaxIters;
            J.tol = kLbgTol;
            st.h[q] = J;
            have[i] = next;
        }
        CQ_TRY(upload(st));
        CQ_TRY(launch_lbg_stage(st.d_jobs(), st.B, st.s));
        CQ_TRY(run_kmeans(st, false));
        CQ_TRY(check_kmeans(st));
        for (auto& v : st.staged) b.staged.push_back(std::move(v));
    }
    return upload(b);
}

cq_status run_init(Batch& b)
{
    bool any_forgy = false, any_sff = false;
    std::vector<int64_t> coop_n(size_t(b.B), 0);
    for (int j = 0; j < b.B; ++j) {
        JobDev& J = b.h[j];
        J.init_blocks = 0;
        if (J.n <= J.K) continue;
        if (J.scheme == CQ_INIT_FORGY) any_forgy = true;
        if (J.scheme == CQ_INIT_MAXMIN || J.scheme == CQ_INIT_KMEANSPP) coop_n[j] = J.n;
        if (J.scheme == CQ_INIT_SFF) {
            any_sff = true;
            J.init_C = sff_subset(J.K, J.n);
            // CQ_SFF_SEQUENTIAL=1 takes the draws one at a time (the path for a
            // rejected draw), for tests; read on every call
            const char* e = getenv("CQ_SFF_SEQUENTIAL");
            J.init_blocks = (e && atoi(e) > 0) ? 1 : 0;
        }
    }
    auto var_job = [&](int j) { return b.h[j].scheme == CQ_INIT_VAR && b.h[j].n > b.h[j].K; };
    const int var_tiles = b.set_map(kMapVarTiles, [&](int j) { return var_job(j) ? var_tile_count(b.h[j].n) : 0; });
    const int var_groups = b.set_map(kMapVarGroups, [&](int j) { return var_job(j) ? b.h[j].K : 0; });
    auto den_job = [&](int j) { return b.h[j].scheme == CQ_INIT_DEN && b.h[j].n > b.h[j].K; };
    const int den_tiles = b.set_map(kMapDenTiles, [&](int j) { return den_job(j) ? den_tile_count(b.h[j].n) : 0; });
    const int den_centres = b.set_map(kMapDenCentres, [&](int j) { return den_job(j) ? b.h[j].K : 0; });
    const int wu_blocks = b.set_map(kMapWu, [&](int j) {
        const JobDev& J = b.h[j];
        return J.scheme == CQ_INIT_WU && J.n > J.K ? wu_accum_blocks(J.n) : 0;
    });
    CQ_TRY(upload(b));
    CQ_TRY(launch_init_begin(b.d_jobs(), b.B, b.s));
    if (any_forgy) CQ_TRY(launch_forgy(b.d_jobs(), b.B, b.s));
    if (var_tiles > 0) CQ_TRY(launch_var(b.d_jobs(), b.d_maps(), b.B, var_tiles, var_groups, b.s));
    if (any_sff) CQ_TRY(launch_sff(b.d_jobs(), b.B, b.s));
    if (wu_blocks > 0) CQ_TRY(launch_wu(b.d_jobs(), b.d_maps(), b.B, wu_blocks, b.s));
    if (den_tiles > 0) CQ_TRY(launch_den(b.d_jobs(), b.d_maps(), b.B, den_tiles, den_centres, b.s));
    std::vector<CoopLaunch> plan;
    CQ_TRY(plan_coop(coop_n, plan));
    for (const CoopLaunch& w : plan) {
        for (int j = 0; j < b.B; ++j) b.h[j].init_blocks = 0;
        for (size_t q = 0; q < w.jobs.size(); ++q) {
            JobDev& J = b.h[w.jobs[q]];
            J.init_blocks = w.blocks[q];
            J.init_C = (J.n + w.blocks[q] - 1) / w.blocks[q];
        }
        const int total = b.set_map(kMapInit, [&](int j) { return b.h[j].init_blocks; });
        CQ_TRY(upload(b));
        CQ_TRY(launch_init_coop(b.d_jobs(), b.d_maps() + kMapInit * (b.B + 1), b.B, total, w.variant, b.s));
    }
    return run_lbg(b);
}

// Iterations of every job until all have stopped.  Iterations are enqueued
// in groups; a stopped job's blocks return at once, so one readback per group
// suffices.
cq_status run_kmeans(Batch& b, bool memberships, bool check)
{
    // every job iterates in step with the launches and all share the
    // schedule's regrouping period, so the host knows which iterations
    // regroup (the same rule as on the device)
    const int period = b.B > 0 ? b.h[0].regroup_period : 1;
    int max_iters = 0;
    for (const JobDev& J : b.h) max_iters = J.max_iters > max_iters ? J.max_iters : max_iters;
    // jobs the host knows to be still iterating; a job that stopped gets no
    // more blocks once the host has read so
    std::vector<char> active(size_t(b.B), 1);
    int assign_total = 0, full_total = 0, walk_total = 0, update_total = 0, table_total = 0;
    auto set_iteration_maps = [&]() {
        auto assign_blocks = [&](int j) {
            const JobDev& J = b.h[j];
            return (J.n <= J.K || !active[size_t(j)]) ? 0 : int((J.n + J.chunk - 1) / J.chunk);
        };
        assign_total = b.set_map(kMapAssign, assign_blocks);
        full_total = b.set_map(kMapAssignFull, [&](int j) { return b.h[j].prune ? 0 : assign_blocks(j); });
        walk_total = b.set_map(kMapAssignWalk, [&](int j) { return b.h[j].prune ? assign_blocks(j) : 0; });
        update_total = b.set_map(kMapUpdate, [&](int j) {
            const JobDev& J = b.h[j];
            if (J.n <= J.K || !active[size_t(j)]) return 0;
            return update_table_blocks(J.K, J.prune) + (J.prune ? int(regroup_blocks(J.n, J.chunk)) : 0);
        });
        table_total = b.set_map(kMapUpdateTable, [&](int j) {
            const JobDev& J = b.h[j];
            return (J.n <= J.K || !active[size_t(j)]) ? 0 : update_table_blocks(J.K, J.prune);
        });
    };
    set_iteration_maps();
    CQ_TRY(upload(b));
    CQ_TRY(launch_kmeans_begin(b.d_jobs(), b.B, b.s));
    if (check) CQ_TRY(launch_check_colours(b.d_jobs(), b.d_maps(), b.B, assign_total, b.s));
    if (assign_total == 0) return collect(b);
    // The status of group g is read while group g + 1 runs: the device never
    // waits for the host, and the group enqueued after the last job stopped
    // costs only early returns.
    EventPair own;
    hipEvent_t* ev_pair = b.fixed_events;
    if (!ev_pair) {
        CQ_TRY(own.create());
        ev_pair = own.ev;
    }
    // As jobs stop, the colours still iterating shrink, and the schedule for
    // that smaller count may take fewer colours per assignment block (which
    // changes no result: the blocks only partition each job's colours; the
    // regrouping period stays, since it fixes which record buffer each
    // iteration reads).  New block counts and maps are uploaded behind the
    // group already queued, so they apply from the group after it.
    auto replan = [&]() -> cq_status {
        int64_t colours = 0;
        for (int j = 0; j < b.B; ++j)
            if (active[size_t(j)] && b.h[j].n > b.h[j].K) colours += b.h[j].n;
        const cq_schedule sched = schedule_for(colours);
        for (int j = 0; j < b.B; ++j)
            if (active[size_t(j)]) b.h[j].chunk = assign_chunk(b.h[j].n, sched.assign_chunk);
        set_iteration_maps();
        return upload(b);
    };
    const int group = 8;
    bool all_done = false, replanned = false;
    for (int it = 1, g = 0; it <= max_iters; it += group, ++g) {
        const int n_it = it + group - 1 <= max_iters ? group : max_iters - it + 1;
        for (int q = 0; q < n_it; ++q)
            CQ_TRY(launch_kmeans_iter(b.d_jobs(), b.d_maps(), b.B, it + q == 1, assign_total, full_total,
                                      walk_total, update_total, regroup_at(it + q, period), table_total,
                                      b.s));
        CQ_TRY(collect_async(b, g & 1, ev_pair[g & 1]));
        if (g == 0) continue;
        CQ_TRY(read_results(b, (g - 1) & 1, ev_pair[(g - 1) & 1]));
        all_done = true;
        bool stopped = false;
        for (int j = 0; j < b.B; ++j) {
            all_done = all_done && b.res[size_t(j)].done;
            if (b.res[size_t(j)].done && active[size_t(j)]) {
                active[size_t(j)] = 0;
                stopped = true;
            }
        }
        if (all_done) break;
        if (stopped && it + group <= max_iters) {
            CQ_TRY(replan());
            replanned = true;
        }
    }
    if (replanned) {
        // every job's blocks again, for the passes after the iterations
        // (the key-order memberships, the colour table)
        std::fill(active.begin(), active.end(), 1);
        set_iteration_maps();
        CQ_TRY(upload(b));
    }
    if (!all_done) CQ_TRY(collect(b));  // the state after the last group
    // the memberships in key order, for callers that return them (a pruned
    // run holds them in its regrouped records until now)
    bool grouped = false;
    for (const JobDev& J : b.h) grouped = grouped || (J.prune && J.n > J.K);
    if (memberships && grouped) CQ_TRY(launch_unpermute(b.d_jobs(), b.d_maps(), b.B, assign_total, b.s));
    return CQ_OK;
}

cq_status run_map(Batch& b, bool with_err, bool from_records)
{
    // a job whose table covers every colour of its image maps through it and
    // sums the squared error over the colours; one that searches the palette
    // per pixel sums it over the pixels in the map kernel.  A pruned job just
    // out of its k-means run searches from its colours' clusters, through
    // its palette's sorted distance rows.
    for (JobDev& J : b.h) J.lut_rec = (from_records && J.prune && !J.map_direct && J.n > J.K) ? 1 : 0;
    const int rows_total = b.set_map(kMapPalRows, [&](int j) {
        const JobDev& J = b.h[j];
        return J.lut_rec ? pal_rows_blocks(J.map_k) : 0;
    });
    const int lut_total = b.set_map(kMapLut, [&](int j) {
        const JobDev& J = b.h[j];
        return J.map_direct ? 0 : int((J.n + J.chunk - 1) / J.chunk);
    });
    const int pix_total = b.set_map(kMapPix, [&](int j) {
        const JobDev& J = b.h[j];
        const bool pass = J.out_idx || J.out_rgb || (with_err && J.map_direct);
        return pass ? map_blocks(int64_t(J.H) * J.W) : 0;
    });
    CQ_TRY(upload(b));
    if (with_err) CQ_TIMED_LAUNCH("k_zero_sq_err", b.s, k_zero_sq_err<<<(b.B + 63) / 64, 64, 0, b.s>>>(b.d_jobs(), b.B));
    if (rows_total > 0) CQ_TRY(launch_pal_rows(b.d_jobs(), b.d_maps(), b.B, rows_total, b.s));
    if (lut_total > 0) CQ_TRY(launch_lut(b.d_jobs(), b.d_maps(), b.B, lut_total, with_err ? 1 : 0, b.s));
    if (pix_total > 0) CQ_TRY(launch_map(b.d_jobs(), b.d_maps(), b.B, pix_total, with_err ? 1 : 0, b.s));
    return CQ_OK;
}

void fill_stats(const JobDev& J, const JobResult& r, cq_stats& st, bool with_img)
{
    memset(&st, 0, sizeof st);
    st.iters = r.iters;
    st.converged = r.converged;
    st.k_used = int32_t(J.n < J.K ? J.n : J.K);
    st.prune = J.prune ? 1 : 0;
    st.n_unique = J.n;
    st.ndc_total = int64_t(r.ndc);
    st.near_ties = int64_t(r.near_ties);
    st.sse_final = r.sse_last;
    st.mse_float = r.total_w ? r.sse_last / double(r.total_w) : 0.0;
    st.mse_img = with_img ? double(r.sq_err) / (double(J.H) * double(J.W)) : 0.0;
}

// After the initialization: a team barrier that gave up is a device error.
cq_status check_init(const Batch& b)
{
    for (int j = 0; j < b.B; ++j) {
        if (b.res[j].sync_error) {
            set_error("job %d: a barrier of the cooperative initialization timed out", j);
            return CQ_EDEVICE;
        }
    }
    return CQ_OK;
}

// After the iterations (fields written by the k-means begin kernel).
cq_status check_kmeans(const Batch& b)
{
    for (int j = 0; j < b.B; ++j) {
        const int bad = b.res[j].bad_input;
        if (bad & 1) return einval("job %d: initial centres contain a non-finite value", j);
        if (bad & 2) return einval("job %d: a colour key is not below 2^24", j);
        if (bad & 4) return einval("job %d: the counts sum to more than 2^28", j);
    }
    return CQ_OK;
}

// Whole quantizer for a filled batch (histogram -> init -> k-means ->
// palette -> map); fills stats (nullable, one per job).
cq_status run_quantize(Batch& b, cq_stats* stats)
{
    CQ_TRY(run_histogram(b));
    CQ_TRY(collect(b));
    std::vector<int64_t> n(size_t(b.B));
    for (int j = 0; j < b.B; ++j) n[j] = b.res[j].n_unique;
    set_counts(b, n);
    CQ_TRY(run_init(b));
    CQ_TRY(run_kmeans(b, false));
    CQ_TRY(check_init(b));
    CQ_TRY(check_kmeans(b));
    CQ_TRY(launch_palette(b.d_jobs(), b.B, b.s));
    CQ_TRY(run_map(b, true, true));
    CQ_TRY(collect(b));
    if (stats)
        for (int j = 0; j < b.B; ++j) fill_stats(b.h[j], b.res[j], stats[j], true);
    return CQ_OK;
}

void fill_quantize_job(JobDev& J, const uint8_t* img, int32_t H, int32_t W, int64_t stride, int32_t subsample,
                       int32_t K, int scheme, uint64_t seed, int32_t max_iters, double tol, int32_t prune,
                       uint8_t* palette, uint8_t* out_idx, uint8_t* out_rgb, char* slot)
{
    const int64_t npix = int64_t(H) * W;
    const Layout L = make_layout(npix, npix, true);
    set_image(J, img, H, W, stride, subsample != 0);
    bind_slot(J, slot, L);
    J.keys = to_dev(reinterpret_cast<uint32_t*>(slot + L.keys));
    J.counts = to_dev(reinterpret_cast<uint32_t*>(slot + L.counts));
    J.assign = to_dev(reinterpret_cast<uint8_t*>(slot + L.assign));
    J.centers = to_dev(reinterpret_cast<double*>(slot + L.centers));
    J.capacity = npix;
    J.K = K;
    J.scheme = scheme;
    J.seed = seed;
    J.max_iters = max_iters;
    J.tol = tol;
    J.prune = prune ? 1 : 0;
    J.palette = to_dev(palette);
    J.out_idx = to_dev(out_idx);
    J.out_rgb = to_dev(out_rgb);
    J.packed = J.packed && (reinterpret_cast<uintptr_t>(out_idx) & 3u) == 0 &&
               (reinterpret_cast<uintptr_t>(out_rgb) & 3u) == 0;
}

size_t slot_bytes(const cq_job& j) { return align256(make_layout(int64_t(j.H) * j.W, int64_t(j.H) * j.W, true).total); }

cq_status check_job(const cq_job& j, int idx)
{
    cq_status s = check_image(j.img, j.H, j.W, j.row_stride_bytes);
    if (s == CQ_OK) s = check_subsample(j.subsample);
    if (s == CQ_OK) s = check_k(j.K);
    if (s == CQ_OK && !j.palette) s = einval("palette is null");
    if (s == CQ_OK && (int(j.scheme) < CQ_INIT_FORGY || int(j.scheme) > CQ_INIT_DEN || j.scheme == CQ_INIT_USER))
        s = einval("scheme must be FORGY, MAXMIN, KMEANSPP, VAR, SFF, WU, LBG or DEN");
    if (s == CQ_OK) s = check_iters_tol(j.max_iters, j.tol);
    if (s != CQ_OK) {
        char msg[512];
        snprintf(msg, sizeof msg, "job %d: %s", idx, g_error);
        snprintf(g_error, sizeof g_error, "%s", msg);
    }
    return s;
}

// cq_quantize on a given workspace; host_stage / events (nullable) make the
// call use a fixed host staging area and fixed readback events instead of
// pooled pinned buffers and new events.
cq_status quantize_into(const uint8_t* img, int32_t H, int32_t W, int64_t row_stride_bytes, int32_t subsample,
                        int32_t K, cq_init_t scheme, uint64_t seed, int32_t max_iters, double tol, int32_t prune,
                        uint8_t* palette, uint8_t* out_idx, uint8_t* out_rgb, cq_stats* stats, void* ws,
                        size_t ws_bytes, void* stream, char* host_stage, size_t host_stage_bytes,
                        hipEvent_t* events)
{
    CQ_TRY(check_image(img, H, W, row_stride_bytes));
    CQ_TRY(check_subsample(subsample));
    CQ_TRY(check_k(K));
    if (!palette) return einval("palette is null");
    if (int(scheme) < CQ_INIT_FORGY || int(scheme) > CQ_INIT_DEN || scheme == CQ_INIT_USER)
        return einval("cq_quantize needs scheme FORGY, MAXMIN, KMEANSPP, VAR, SFF, WU, LBG or DEN");
    CQ_TRY(check_iters_tol(max_iters, tol));
    const int64_t npix = int64_t(H) * W;
    const Layout L = make_layout(npix, npix, true);
    CQ_TRY(check_ws(ws, ws_bytes, L.total));
    Batch b(1, at<char>(ws, L.desc), static_cast<hipStream_t>(stream));
    b.host_stage = host_stage;
    b.host_stage_bytes = host_stage_bytes;
    b.fixed_events = events;
    fill_quantize_job(b.h[0], img, H, W, row_stride_bytes, subsample, K, int(scheme), seed, max_iters, tol, prune,
                      palette, out_idx, out_rgb, static_cast<char*>(ws));
    return run_quantize(b, stats);
}

// The library's process-wide objects: pooled pinned host buffers, readback
// streams, the kernel timer's events and the allocation-free entry point's
// per-device events.  Re-created on demand by later calls.
void release_resources()
{
    {
        HostPool& pool = host_pool();
        std::lock_guard<std::mutex> lock(pool.mu);
        for (auto& list : pool.free_list) {
            for (void* p : list) (void)hipHostFree(p);
            list.clear();
        }
    }
    {
        std::lock_guard<std::mutex> lock(g_side_mu);
        for (auto& kv : side_streams()) (void)hipStreamDestroy(kv.second);
        side_streams().clear();
    }
    timer_release();
    noalloc_release();
}

}  // namespace cq

using namespace cq;

extern "C" {

size_t cq_workspace_bytes(int32_t H, int32_t W, int32_t K)
{
    if (H <= 0 || W <= 0 || K < 1 || K > kMaxK) return 0;
    const int64_t npix = int64_t(H) * W;
    if (npix > kMaxPixels) return 0;
    return make_layout(npix, npix, true).total;
}

cq_status cq_workspace_prepare(void* ws, size_t ws_bytes, void* stream)
{
    clear_error();
    const Layout L = make_layout(0, 0, false);
    CQ_TRY(check_ws(ws, ws_bytes, L.fixed_end));
    (void)stream;  // no region needs clearing between calls
    return CQ_OK;
}

cq_status cq_histogram(const uint8_t* img, int32_t H, int32_t W, int64_t row_stride_bytes,
                       int32_t subsample, uint32_t* keys, uint32_t* counts, int64_t capacity, int64_t* n_unique,
                       void* ws, size_t ws_bytes, void* stream)
{
    clear_error();
    CQ_TRY(check_image(img, H, W, row_stride_bytes));
    CQ_TRY(check_subsample(subsample));
    if (!n_unique) return einval("n_unique is null");
    if (capacity < 0) return einval("capacity is negative");
    if (capacity > 0 && (!keys || !counts)) return einval("keys/counts are null");
    const Layout L = make_layout(int64_t(H) * W, 0, false);
    CQ_TRY(check_ws(ws, ws_bytes, L.total));
    Batch b(1, at<char>(ws, L.desc), static_cast<hipStream_t>(stream));
    JobDev& J = b.h[0];
    set_image(J, img, H, W, row_stride_bytes, subsample != 0);
    bind_slot(J, static_cast<char*>(ws), L);
    J.keys = to_dev(keys);
    J.counts = to_dev(counts);
    J.capacity = capacity;
    CQ_TRY(run_histogram(b));
    CQ_TRY(collect(b));
    const int64_t n = b.res[0].n_unique;
    *n_unique = n;
    if (n > capacity) {
        set_error("%lld unique colours exceed capacity %lld", (long long)n, (long long)capacity);
        return CQ_ECAPACITY;
    }
    return CQ_OK;
}

cq_status cq_pixel_keys(const uint8_t* img, int32_t H, int32_t W, int64_t row_stride_bytes, uint32_t* keys,
                        uint32_t* counts, void* stream)
{
    clear_error();
    CQ_TRY(check_image(img, H, W, row_stride_bytes));
    if (!keys || !counts) return einval("keys/counts are null");
    return launch_pixel_keys(img, H, W, row_stride_bytes, keys, counts, static_cast<hipStream_t>(stream));
}

cq_status cq_init(const uint32_t* keys, const uint32_t* counts, int64_t n_unique, int32_t K,
                  cq_init_t scheme, uint64_t seed, double* centers, int32_t* k_used, void* ws,
                  size_t ws_bytes, void* stream)
{
    clear_error();
    CQ_TRY(check_k(K));
    if (!keys || !counts || !centers) return einval("keys/counts/centers is null");
    if (n_unique < 1 || n_unique > kMaxPixels) return einval("n_unique = %lld out of range", (long long)n_unique);
    if (int(scheme) < CQ_INIT_FORGY || int(scheme) > CQ_INIT_DEN) return einval("unknown init scheme %d", int(scheme));
    const Layout L = make_layout(0, n_unique, false);
    CQ_TRY(check_ws(ws, ws_bytes, L.total));
    Batch b(1, at<char>(ws, L.desc), static_cast<hipStream_t>(stream));
    JobDev& J = b.h[0];
    bind_slot(J, static_cast<char*>(ws), L);
    J.keys = to_dev(const_cast<uint32_t*>(keys));
    J.counts = to_dev(const_cast<uint32_t*>(counts));
    J.centers = to_dev(centers);
    J.assign = to_dev(reinterpret_cast<uint8_t*>(static_cast<char*>(ws) + L.assign));
    J.K = K;
    J.scheme = int(scheme);
    J.seed = seed;
    set_counts(b, {n_unique});
    CQ_TRY(run_init(b));
    if (k_used) {
        CQ_TRY(collect(b));
        CQ_TRY(check_init(b));
        *k_used = int32_t(n_unique < K ? n_unique : K);
    }
    return CQ_OK;
}

cq_status cq_kmeans(const uint32_t* keys, const uint32_t* counts, int64_t n_unique, int32_t K,
                    double* centers, int32_t max_iters, double tol, int32_t prune, uint8_t* assign,
                    uint8_t* palette, double* sse_trace, cq_stats* stats, void* ws, size_t ws_bytes,
                    void* stream)
{
    clear_error();
    CQ_TRY(check_k(K));
    if (!keys || !counts || !centers || !assign) return einval("keys/counts/centers/assign is null");
    if (n_unique < 1 || n_unique > kMaxPixels) return einval("n_unique = %lld out of range", (long long)n_unique);
    CQ_TRY(check_iters_tol(max_iters, tol));
    // a pruned run keeps two packed records per colour in the workspace
    const Layout L = make_layout(0, prune ? n_unique : 0, false);
    CQ_TRY(check_ws(ws, ws_bytes, prune ? L.total : L.fixed_end));
    Batch b(1, at<char>(ws, L.desc), static_cast<hipStream_t>(stream));
    JobDev& J = b.h[0];
    bind_slot(J, static_cast<char*>(ws), L);
    J.keys = to_dev(const_cast<uint32_t*>(keys));
    J.counts = to_dev(const_cast<uint32_t*>(counts));
    J.centers = to_dev(centers);
    J.assign = to_dev(assign);
    J.palette = to_dev(palette);
    J.K = K;
    J.max_iters = max_iters;
    J.tol = tol;
    J.prune = prune ? 1 : 0;
    set_counts(b, {n_unique});
    CQ_TRY(run_kmeans(b, true, true));
    CQ_TRY(check_kmeans(b));
    if (palette) CQ_TRY(launch_palette(b.d_jobs(), 1, b.s));
    const JobResult r = b.res[0];
    if (sse_trace && r.iters > 0) {
        CQ_HIP_TRY(hipMemcpyAsync(sse_trace, from_dev(J.trace), sizeof(double) * size_t(r.iters), hipMemcpyDeviceToHost, b.s));
    }
    CQ_HIP_TRY(hipStreamSynchronize(b.s));
    if (stats) fill_stats(J, r, *stats, false);
    return CQ_OK;
}

cq_status cq_map(const uint8_t* img, int32_t H, int32_t W, int64_t row_stride_bytes,
                 const uint32_t* keys, const uint32_t* counts, int64_t n_unique,
                 const uint8_t* palette, int32_t K, uint8_t* out_idx, uint8_t* out_rgb,
                 uint64_t* sq_err_sum, void* ws, size_t ws_bytes, void* stream)
{
    clear_error();
    CQ_TRY(check_image(img, H, W, row_stride_bytes));
    CQ_TRY(check_k(K));
    if (!keys || !palette) return einval("keys/palette is null");
    if (n_unique < 1 || n_unique > int64_t(H) * W) return einval("n_unique = %lld out of range", (long long)n_unique);
    if (sq_err_sum && !counts) return einval("sq_err_sum needs counts");
    const Layout L = make_layout(0, 0, false);
    CQ_TRY(check_ws(ws, ws_bytes, L.fixed_end));
    Batch b(1, at<char>(ws, L.desc), static_cast<hipStream_t>(stream));
    JobDev& J = b.h[0];
    set_image(J, img, H, W, row_stride_bytes, false);
    bind_slot(J, static_cast<char*>(ws), L);
    J.keys = to_dev(const_cast<uint32_t*>(keys));
    J.counts = to_dev(const_cast<uint32_t*>(counts));
    J.palette = to_dev(const_cast<uint8_t*>(palette));
    J.out_idx = to_dev(out_idx);
    J.out_rgb = to_dev(out_rgb);
    J.K = K;
    set_counts(b, {n_unique});
    J.map_k = K;
    J.packed = J.packed && (reinterpret_cast<uintptr_t>(out_idx) & 3u) == 0 &&
               (reinterpret_cast<uintptr_t>(out_rgb) & 3u) == 0;
    CQ_TRY(run_map(b, sq_err_sum != nullptr, false));
    if (sq_err_sum) {
        CQ_TRY(collect(b));
        *sq_err_sum = b.res[0].sq_err;
    }
    return CQ_OK;
}

cq_status cq_quantize(const uint8_t* img, int32_t H, int32_t W, int64_t row_stride_bytes, int32_t subsample,
                      int32_t K, cq_init_t scheme, uint64_t seed, int32_t max_iters, double tol, int32_t prune,
                      uint8_t* palette, uint8_t* out_idx, uint8_t* out_rgb, cq_stats* stats, void* ws,
                      size_t ws_bytes, void* stream)
{
    clear_error();
    return quantize_into(img, H, W, row_stride_bytes, subsample, K, scheme, seed, max_iters, tol, prune, palette,
                         out_idx, out_rgb, stats, ws, ws_bytes, stream, nullptr, 0, nullptr);
}

size_t cq_batch_workspace_bytes(const cq_job* jobs, int32_t n_jobs)
{
    if (!jobs || n_jobs < 1 || n_jobs > kMaxBatch) return 0;
    size_t total = align256(desc_bytes(n_jobs));
    for (int32_t i = 0; i < n_jobs; ++i) {
        const cq_job& j = jobs[i];
        if (j.H <= 0 || j.W <= 0 || int64_t(j.H) * j.W > kMaxPixels) return 0;
        total += slot_bytes(j);
    }
    return total;
}

cq_status cq_batch_workspace_prepare(const cq_job* jobs, int32_t n_jobs, void* ws, size_t ws_bytes, void* stream)
{
    clear_error();
    const size_t need = cq_batch_workspace_bytes(jobs, n_jobs);
    if (need == 0) return einval("invalid batch description");
    CQ_TRY(check_ws(ws, ws_bytes, need));
    (void)stream;  // no region needs clearing between calls
    return CQ_OK;
}

cq_status cq_quantize_batch(const cq_job* jobs, int32_t n_jobs, cq_stats* stats, void* ws, size_t ws_bytes,
                            void* stream)
{
    clear_error();
    if (!jobs || n_jobs < 1 || n_jobs > kMaxBatch) return einval("n_jobs must be in [1, %d]", kMaxBatch);
    for (int32_t i = 0; i < n_jobs; ++i) CQ_TRY(check_job(jobs[i], i));
    const size_t need = cq_batch_workspace_bytes(jobs, n_jobs);
    CQ_TRY(check_ws(ws, ws_bytes, need));
    Batch b(n_jobs, static_cast<char*>(ws), static_cast<hipStream_t>(stream));
    char* slot = static_cast<char*>(ws) + align256(desc_bytes(n_jobs));
    for (int32_t i = 0; i < n_jobs; ++i) {
        const cq_job& j = jobs[i];
        fill_quantize_job(b.h[i], j.img, j.H, j.W, j.row_stride_bytes, j.subsample, j.K, int(j.scheme), j.seed, j.max_iters,
                          j.tol, j.prune, j.palette, j.out_idx, j.out_rgb, slot);
        slot += slot_bytes(j);
    }
    return run_quantize(b, stats);
}

cq_status cq_set_schedule(const cq_schedule* table, int32_t n)
{
    clear_error();
    return set_schedule(table, n);
}

cq_status cq_get_schedule(cq_schedule* table, int32_t capacity, int32_t* n)
{
    clear_error();
    return get_schedule(table, capacity, n);
}

cq_status cq_timer_enable(const char* kernel, int32_t max_launches, int32_t every)
{
    clear_error();
    if (!kernel || !kernel[0] || strlen(kernel) >= sizeof g_timer.name) return einval("bad kernel name");
    if (max_launches < 1 || max_launches > (1 << 22)) return einval("max_launches out of range");
    if (every < 1) return einval("every must be at least 1");
    timer_release();
    g_timer.start = new hipEvent_t[max_launches];
    g_timer.stop = new hipEvent_t[max_launches];
    for (int32_t i = 0; i < max_launches; ++i) {
        if (hipEventCreate(&g_timer.start[i]) != hipSuccess || hipEventCreate(&g_timer.stop[i]) != hipSuccess) {
            g_timer.capacity = i;  // release what was created
            timer_release();
            set_error("hipEventCreate failed");
            return CQ_EDEVICE;
        }
        g_timer.capacity = i + 1;
    }
    strncpy(g_timer.name, kernel, sizeof g_timer.name - 1);
    g_timer.used = 0;
    g_timer.every = every;
    g_timer.seen = 0;
    g_timer.armed = false;
    g_timer.enabled = true;
    return CQ_OK;
}

cq_status cq_timer_read(int64_t* launches, double* total_ms, int64_t* seen)
{
    clear_error();
    if (!launches || !total_ms) return einval("null output");
    double total = 0.0;
    for (int32_t i = 0; i < g_timer.used; ++i) {
        CQ_HIP_TRY(hipEventSynchronize(g_timer.stop[i]));
        float ms = 0.f;
        CQ_HIP_TRY(hipEventElapsedTime(&ms, g_timer.start[i], g_timer.stop[i]));
        total += double(ms);
    }
    *launches = g_timer.used;
    *total_ms = total;
    if (seen) *seen = g_timer.seen;
    return CQ_OK;
}

cq_status cq_timer_disable(void)
{
    clear_error();
    timer_release();
    return CQ_OK;
}

void cq_release_resources(void) { release_resources(); }

const char* cq_last_error(void) { return g_error; }

}  // extern "C"
