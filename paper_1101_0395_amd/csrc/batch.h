// Host side of a batch: the job descriptors and block maps of one launch
// sequence, and the phases of the quantizer over a batch (defined in
// api.hip; the serving engine in engine.hip drives the same phases over the
// jobs it has in flight).
#pragma once

#include <string.h>

#include <deque>
#include <vector>

#include "coop_plan.h"
#include "cq_internal.h"

namespace cq {

// A host buffer for asynchronous copies: pinned memory (hipHostMalloc) from
// per-size free lists kept for the life of the process (a pageable source or
// destination makes the runtime stage every copy), or pageable memory if no
// pinned memory can be had.  The memory returns to its list on destruction.
class HostBuf {
public:
    HostBuf() = default;
    explicit HostBuf(size_t n);
    HostBuf(HostBuf&& o) noexcept : p_(o.p_), cap_(o.cap_), pinned_(o.pinned_) { o.p_ = nullptr; }
    HostBuf& operator=(HostBuf&& o) noexcept
    {
        if (this != &o) {
            release();
            p_ = o.p_;
            cap_ = o.cap_;
            pinned_ = o.pinned_;
            o.p_ = nullptr;
        }
        return *this;
    }
    HostBuf(const HostBuf&) = delete;
    HostBuf& operator=(const HostBuf&) = delete;
    ~HostBuf() { release(); }
    char* data() const { return static_cast<char*>(p_); }

private:
    void release();
    void* p_ = nullptr;
    size_t cap_ = 0;
    bool pinned_ = false;
};

// Host view of one launch sequence: job descriptors, block maps, and the
// device descriptor region they are copied to.
struct Batch {
    int B = 0;
    char* desc = nullptr;
    hipStream_t s = nullptr;
    std::vector<JobDev> h;
    std::vector<int> maps;
    std::vector<JobResult> res;
    std::deque<HostBuf> staged;  // host copies behind the uploads, kept until the stream is synchronized
    // When set, uploads and readbacks go through this pageable host area
    // instead of pooled pinned buffers (the path that allocates nothing): a
    // copy from pageable memory has consumed its source when the call
    // returns, and a copy to it has completed, so the area is reused at once.
    char* host_stage = nullptr;
    size_t host_stage_bytes = 0;
    // events of the pipelined status readback, owned elsewhere when set
    hipEvent_t* fixed_events = nullptr;

    Batch(int nb, char* d, hipStream_t st)
        : B(nb), desc(d), s(st), h(size_t(nb)), maps(size_t(kNumMaps) * (nb + 1), 0), res(size_t(nb))
    {
        memset(static_cast<void*>(h.data()), 0, sizeof(JobDev) * h.size());
    }
    JobDev* d_jobs() const { return reinterpret_cast<JobDev*>(desc); }
    int* d_maps() const { return reinterpret_cast<int*>(desc + desc_maps_off(B)); }
    JobResult* d_results(int slot = 0) const
    {
        return reinterpret_cast<JobResult*>(desc + desc_results_off(B) + size_t(slot) * align256(sizeof(JobResult) * size_t(B)));
    }

    // map `id` from per-job block counts; returns the total
    template <typename F>
    int set_map(int id, F blocks_of)
    {
        int* m = maps.data() + size_t(id) * (B + 1);
        m[0] = 0;
        for (int j = 0; j < B; ++j) m[j + 1] = m[j] + blocks_of(j);
        return m[B];
    }
};

// kernels launched from the other translation units
int hist_blocks(int64_t npix);
int hist_count_blocks(int64_t npix, int min_blocks);
cq_status launch_pixel_keys(const uint8_t* img, int32_t H, int32_t W, int64_t row_stride, uint32_t* keys,
                            uint32_t* counts, hipStream_t s);
cq_status launch_histogram(const JobDev* jobs, const int* maps, int B, int total_hist_blocks, int total_count,
                           int max_tiles, int emit_per_wave, hipStream_t s);
// One cooperative initialization launch: the kernel variant (8 or 32
// colours per thread in registers; 0: D^2 in global memory), its jobs and
// their team sizes.
int coop_capacity(int variant);
int64_t coop_reg_colours(int R);
cq_status plan_coop(const std::vector<int64_t>& n, std::vector<CoopLaunch>& plan);
cq_status launch_init_begin(const JobDev* jobs, int B, hipStream_t s);
cq_status launch_forgy(const JobDev* jobs, int B, hipStream_t s);
cq_status launch_var(const JobDev* jobs, const int* maps, int B, int tiles, int groups, hipStream_t s);
int var_tile_count(int64_t n);
int wu_accum_blocks(int64_t n);
cq_status launch_wu(const JobDev* jobs, const int* maps, int B, int accum_blocks, hipStream_t s);
cq_status launch_lbg_stage(const JobDev* jobs, int B, hipStream_t s);
int den_tile_count(int64_t n);
cq_status launch_den(const JobDev* jobs, const int* maps, int B, int tiles, int centres, hipStream_t s);
cq_status launch_sff(const JobDev* jobs, int B, hipStream_t s);
int64_t sff_subset(int32_t K, int64_t n);
cq_status launch_init_coop(const JobDev* jobs, const int* map, int B, int total, int variant, hipStream_t s);
cq_status launch_kmeans_begin(const JobDev* jobs, int B, hipStream_t s);
cq_status launch_check_colours(const JobDev* jobs, const int* maps, int B, int blocks, hipStream_t s);
cq_status launch_kmeans_iter(const JobDev* jobs, const int* maps, int B, bool first, int all_blocks,
                             int full_blocks, int walk_blocks, int update_blocks, bool regroup,
                             int table_blocks, hipStream_t s);
int update_table_blocks(int K, int prune);
cq_status launch_palette(const JobDev* jobs, int B, hipStream_t s);
int64_t assign_chunk(int64_t n, int32_t scheduled);
cq_schedule schedule_for(int64_t colours);
cq_status set_schedule(const cq_schedule* table, int32_t n);
cq_status get_schedule(cq_schedule* table, int32_t capacity, int32_t* n);
int64_t regroup_blocks(int64_t n, int64_t chunk);
cq_status launch_unpermute(const JobDev* jobs, const int* maps, int B, int blocks, hipStream_t s);
int map_blocks(int64_t npix);
cq_status launch_lut(const JobDev* jobs, const int* maps, int B, int total, int with_err, hipStream_t s);
int pal_rows_blocks(int K);
cq_status launch_pal_rows(const JobDev* jobs, const int* maps, int B, int total, hipStream_t s);
cq_status launch_map(const JobDev* jobs, const int* maps, int B, int total, int with_err, hipStream_t s);

// argument checks (set the thread's error text)
cq_status einval(const char* fmt, ...);
cq_status check_ws(const void* ws, size_t ws_bytes, size_t need);
cq_status check_job(const cq_job& j, int idx);

// phases over a filled batch
cq_status upload(Batch& b);
cq_status collect(Batch& b);  // every job's control block into b.res; synchronizes the stream
// Copies every job's control block to result slot `slot` and records `done`
// on the batch stream; read_results waits for that event only (not for work
// enqueued after it) and fills b.res from the slot.
cq_status collect_async(Batch& b, int slot, hipEvent_t done);
cq_status read_results(Batch& b, int slot, hipEvent_t done);
cq_status run_histogram(Batch& b);
void set_counts(Batch& b, const std::vector<int64_t>& n);
cq_status run_init(Batch& b);
// memberships: write the final memberships in key order (cq_kmeans);
// check: validate caller-supplied colours first (keys below 2^24, counts
// summing to at most 2^28; a job that fails runs no iteration and
// check_kmeans reports it).
cq_status run_kmeans(Batch& b, bool memberships, bool check = false);
// from_records: the jobs come straight from their k-means runs, so a pruned
// job's colour table may start each colour at its final cluster.
cq_status run_map(Batch& b, bool with_err, bool from_records);
cq_status run_quantize(Batch& b, cq_stats* stats);  // histogram -> init -> k-means -> palette -> map
cq_status quantize_into(const uint8_t* img, int32_t H, int32_t W, int64_t row_stride_bytes, int32_t subsample,
                        int32_t K, cq_init_t scheme, uint64_t seed, int32_t max_iters, double tol, int32_t prune,
                        uint8_t* palette, uint8_t* out_idx, uint8_t* out_rgb, cq_stats* stats, void* ws,
                        size_t ws_bytes, void* stream, char* host_stage, size_t host_stage_bytes,
                        hipEvent_t* events);
// Releases the per-device set-up of the allocation-free entry point.
void noalloc_release();
// The device's readback stream (created on first use).
cq_status side_stream(hipStream_t* out);
cq_status check_init(const Batch& b);
cq_status check_kmeans(const Batch& b);
void fill_stats(const JobDev& J, const JobResult& r, cq_stats& st, bool with_img);

// one whole-quantizer job in a slot of slot_bytes(j) bytes
size_t slot_bytes(const cq_job& j);
void fill_quantize_job(JobDev& J, const uint8_t* img, int32_t H, int32_t W, int64_t stride, int32_t subsample,
                       int32_t K, int scheme, uint64_t seed, int32_t max_iters, double tol, int32_t prune,
                       uint8_t* palette, uint8_t* out_idx, uint8_t* out_rgb, char* slot);

#define CQ_TRY(expr)                     \
    do {                                 \
        cq_status st_ = (expr);          \
        if (st_ != CQ_OK) return st_;    \
    } while (0)

}  // namespace cq
