/* cq: exact weighted k-means colour quantization on AMD Instinct MI355X (gfx950).
 *
 * C ABI of the GPU library libcq.so.  The method is the Weighted Sort-Means
 * (WSM) quantizer of M. E. Celebi, "Improving the Performance of K-Means for
 * Color Quantization": data reduction to the unique colours of the image with
 * their pixel counts as weights (Section 2.2, items 1-2), Lloyd iterations
 * (Algo. 1) accelerated by sort-means triangle-inequality pruning (Section 2.2
 * item 3, Algo. 2), the relative-SSE stopping rule of Section 3.3, and the
 * pixel-mapping phase of Section 1 with the MSE of Section 3.1.
 *
 * General conventions
 *  - Pointers are DEVICE pointers unless marked (host).  The caller owns every
 *    buffer, including the workspace; the library never allocates device
 *    memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Work
 *    is enqueued on it; a call that returns a value through a (host) pointer
 *    synchronizes that stream before returning.
 *  - Images are uint8 H x W x 3, interleaved R,G,B, rows `row_stride_bytes`
 *    apart (>= 3 W).  A colour key is R<<16 | G<<8 | B.
 *  - K (palette size) is in [1, 256]; H * W <= 2^28.
 *  - Results are bit-identical to the CPU reference definition: integer
 *    histograms, sums and MSE numerators; FP64 distances evaluated as
 *    (dx*dx + dy*dy) + dz*dz without contraction.
 *  - Errors: a non-zero cq_status is returned and cq_last_error() describes it.
 *    No call aborts the process and no C++ exception crosses the ABI.  Outputs
 *    are unspecified after an error.
 *  - Calls that share one workspace must be serialized (same stream or
 *    external synchronization).
 */
#ifndef CQ_H
#define CQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CQ_OK = 0,
    CQ_EINVAL = 1,      /* invalid argument (range, null pointer, shape)       */
    CQ_ECAPACITY = 2,   /* output capacity smaller than the number of colours  */
    CQ_EWORKSPACE = 3,  /* workspace missing, too small or misaligned          */
    CQ_EDEVICE = 4      /* HIP runtime error; see cq_last_error()              */
} cq_status;

/* Initialization schemes of Section 2.3, and WU, the initializer of WSM-WU
 * in Section 3.3. */
typedef enum {
    CQ_INIT_FORGY = 0,     /* K distinct colours drawn uniformly (FGY)              */
    CQ_INIT_MAXMIN = 1,    /* farthest-first after a uniform first colour (MMX)     */
    CQ_INIT_KMEANSPP = 2,  /* D^2 sampling, weighted by pixel counts (KPP)          */
    CQ_INIT_USER = 3,      /* centres supplied by the caller (WSM-X warm start)     */
    CQ_INIT_VAR = 4,       /* maximum variance: medians along the widest channel    */
    CQ_INIT_SFF = 5,       /* farthest first on a random subset (SFF)              */
    CQ_INIT_WU = 6,        /* Wu's greedy orthogonal bipartitioning (WU)           */
    CQ_INIT_LBG = 7,       /* splitting from the centroid, refined by k-means (LBG) */
    CQ_INIT_DEN = 8        /* centres per uniform cell by its share of colours (DEN) */
} cq_init_t;

/* Run statistics (host structure). */
typedef struct {
    int32_t iters;      /* Lloyd iterations run                                     */
    int32_t converged;  /* 1 if stopped by the relative-SSE test or SSE == 0        */
    int32_t k_used;     /* min(K, N')                                               */
    int32_t prune;      /* 1 if sort-means pruning was on                           */
    int64_t n_unique;   /* N', the number of unique colours                         */
    int64_t ndc_total;  /* distance calculations, summed over colours and iterations */
    int64_t near_ties;  /* colour-iterations whose two smallest evaluated distances
                           differ by at most 1e-5 relative                          */
    double sse_final;   /* SSE (eq. 1) after the last centre update                 */
    double mse_float;   /* sse_final / number of pixels                             */
    double mse_img;     /* MSE (Section 3.1) of the mapped image (cq_quantize only) */
} cq_stats;

/* Bytes of workspace needed by every entry point for one image of H x W pixels
 * with palette size K (the same buffer serves all five calls).  Returns 0 for
 * invalid sizes. */
size_t cq_workspace_bytes(int32_t H, int32_t W, int32_t K);

/* Check a workspace before its first use (size and 256-byte alignment).
 * No region of the workspace has to hold particular values between calls, so
 * nothing is written; calling it again, for instance after CQ_EDEVICE, is
 * harmless. */
cq_status cq_workspace_prepare(void* ws, size_t ws_bytes, void* stream);

/* Section 2.2 items 1-2: the unique colours of the image with their pixel
 * counts.  subsample != 0 first applies the optional 2:1 subsampling of item
 * 1: only the pixels at even row and even column (ceil(H/2) x ceil(W/2) of
 * them) are counted.  Writes keys[0..N') in ascending order and
 * counts[0..N') (the weights before normalization by the number of pixels
 * counted).  *n_unique (host) receives N'; if N' > capacity only the first
 * `capacity` entries are written and CQ_ECAPACITY is returned.  The workspace
 * must hold cq_workspace_bytes(H, W, K) for this image (it stages the pixels
 * partitioned by key range).  Synchronizes `stream`. */
cq_status cq_histogram(const uint8_t* img, int32_t H, int32_t W, int64_t row_stride_bytes,
                       int32_t subsample, uint32_t* keys, uint32_t* counts, int64_t capacity,
                       int64_t* n_unique /* host */, void* ws, size_t ws_bytes, void* stream);

/* The data set of plain KM (Algo. 1, the baseline of the comparison in
 * Section 3.2): one record per pixel, in row-major order, keys[p] the pixel's
 * colour key and counts[p] = 1.  keys and counts are device uint32[H W].
 * Passed to cq_kmeans with prune = 0 they make it run KM over the pixels: a
 * full search of the K centres for every pixel in every iteration.  The same
 * starting centres give the same centres, SSE trace and palette as the
 * weighted run on the histogram (the cluster sums are exact integers).  Does
 * not synchronize. */
cq_status cq_pixel_keys(const uint8_t* img, int32_t H, int32_t W, int64_t row_stride_bytes,
                        uint32_t* keys, uint32_t* counts, void* stream);

/* Section 2.3 (and WU of Section 3.3): initial centres from the N' unique
 * colours.  centers is a device double[K][3].  For N' <= K the centres are the
 * colours in key order followed by zeros and *k_used (host, nullable) is N'.
 * Random draws come from one splitmix64 stream seeded with `seed`.
 *  - FGY: a partial Fisher-Yates shuffle of the colours, draw j uniform in
 *    [j, N').
 *  - MMX: the first colour uniform, then farthest first by integer D^2 (ties
 *    to the lowest index).
 *  - KPP: the first colour with probability proportional to its count, colour
 *    j then proportional to count * D^2.
 *  - VAR (no draws): on the pixel data set (colour i repeated count_i times),
 *    the channel of largest pixel variance (ties R, G, B), the pixels ordered
 *    by (that channel's value, key), K groups [floor(g N / K),
 *    floor((g+1) N / K)) of the N pixels, each group's lower-median pixel.
 *  - SFF: a subset of L = max(K, ceil(2 K ln K)) colours (at most N') drawn as
 *    FGY draws, then MMX on the subset in draw order (first centre
 *    subset[U(L)], ties to the lowest subset position).
 *  - WU (no draws): Wu's greedy orthogonal bipartitioning over 32 levels per
 *    channel (value >> 3).  From the whole grid, the box of largest weighted
 *    variance s2 - |m|^2 / w (ties to the lowest box index; a box of one cell,
 *    or with no allowed cut, counts 0) is split at the plane maximizing
 *    |m_l|^2 / w_l + |m_u|^2 / w_u over two non-empty parts (first plane,
 *    then R, G, B on ties); the lower part keeps the index and the upper part
 *    is appended, until K boxes or no variance is left.  The centres are the
 *    box means; with fewer than K boxes the rest repeat box 0's mean.  The
 *    statistics are exact integers, the criteria FP64 in that order.
 *  - LBG (no draws): the weighted centroid, then stages that turn centre j of
 *    m into c_j - (1,1,1) in place and c_j + (1,1,1) at index m + j (a last
 *    partial stage splits the first K - m), each refined by weighted Lloyd
 *    iterations stopped by the rule of Section 3.3 at the paper's threshold
 *    0.001 (at most 100 iterations).  Synchronizes `stream` once per stage.
 *  - DEN: 512 cells (value >> 5 per channel, cell (r >> 5) * 64 +
 *    (g >> 5) * 8 + (b >> 5)); cell c with u_c of the N' colours gets
 *    floor(K u_c / N') centres, and the rest go one each to the cells of
 *    largest remainder K u_c mod N' (ties to the lower cell); cell by cell the
 *    quota is drawn as FGY draws from the cell's colours in key order.
 *  - USER: the centres are left as given.
 * The colours must be as cq_histogram gives them: keys below 2^24 in
 * ascending order, counts summing to at most 2^28 (the k-means++ weights
 * n D^2 are summed in 46 bits); other inputs give unspecified centres or
 * CQ_EDEVICE from a cooperative wait that gives up, never an access out of
 * bounds.  The workspace must hold cq_workspace_bytes(H, W, K) of an image with
 * H W >= N'.  Synchronizes only if k_used is non-null or the scheme is LBG; a
 * device-side failure of the initialization is reported by that
 * synchronization or by the next synchronizing call on the workspace. */
cq_status cq_init(const uint32_t* keys, const uint32_t* counts, int64_t n_unique, int32_t K,
                  cq_init_t scheme, uint64_t seed, double* centers, int32_t* k_used /* host */,
                  void* ws, size_t ws_bytes, void* stream);

/* Algo. 1 / Algo. 2: weighted Lloyd iterations on the unique colours starting
 * from centers (device double[K][3], updated in place).  keys/counts are the
 * ascending unique colours of cq_histogram; with prune = 0 any records will
 * do (unsorted, repeated keys: cq_pixel_keys gives plain KM).
 *  - prune = 0: full nearest-centre search every iteration (Algo. 1).
 *  - prune = 1: sort-means (Algo. 2): iteration 1 is a full search; later
 *    iterations scan the centres in increasing distance from the previous
 *    centre and stop once d(c_p, c_t)^2 > 4 d(x, c_p)^2 (1 + 1e-12).  Both
 *    modes give identical results; only the distance count differs.
 *  - Ties go to the lowest centre index.  An empty cluster keeps its centre.
 *  - After the update of iteration i, SSE_i is computed from exact integer
 *    cluster sums; the run stops when SSE_i == 0, when i >= 2 and
 *    SSE_{i-1} - SSE_i <= tol * SSE_i (Section 3.3), or at max_iters.
 * assign (device uint8[N']) receives the final memberships; palette (device
 * uint8[K][3], nullable) receives floor(c + 0.5) clamped to [0, 255];
 * sse_trace (host double[max_iters], nullable) receives SSE_1..SSE_iters.
 * For N' <= K the centres become the colours and no iteration runs.
 * 1 <= max_iters <= 100000, tol >= 0.  Every key must be below 2^24 and
 * the counts must sum to at most 2^28 (a pruned run packs a count in 28
 * bits): a run with more than K colours checks this on the device first and
 * returns CQ_EINVAL without iterating.  A pruned run keeps two 8-byte
 * records per colour in the workspace: cq_workspace_bytes(H, W, K) of any
 * image with H W >= N' is enough.  Synchronizes `stream`. */
cq_status cq_kmeans(const uint32_t* keys, const uint32_t* counts, int64_t n_unique, int32_t K,
                    double* centers, int32_t max_iters, double tol, int32_t prune,
                    uint8_t* assign, uint8_t* palette, double* sse_trace /* host */,
                    cq_stats* stats /* host */, void* ws, size_t ws_bytes, void* stream);

/* Pixel mapping (Section 1): every pixel goes to the palette entry at the
 * smallest integer squared distance (lowest index on ties).  `keys` are the
 * image's unique colours from cq_histogram (every pixel colour must be among
 * them).  out_idx (device uint8[H][W], nullable) receives the palette index,
 * out_rgb (device uint8[H][W][3], nullable) the palette colour.
 * *sq_err_sum (host, nullable) receives the integer sum over pixels of the
 * squared error, i.e. H W times the MSE of Section 3.1; it needs `counts`
 * (device uint32[N'], nullable otherwise).  Synchronizes only if sq_err_sum is
 * non-null. */
cq_status cq_map(const uint8_t* img, int32_t H, int32_t W, int64_t row_stride_bytes,
                 const uint32_t* keys, const uint32_t* counts, int64_t n_unique,
                 const uint8_t* palette, int32_t K, uint8_t* out_idx, uint8_t* out_rgb,
                 uint64_t* sq_err_sum /* host */, void* ws, size_t ws_bytes, void* stream);

/* The whole quantizer: histogram (of the 2:1-subsampled image if subsample
 * != 0, as in cq_histogram) -> init (any scheme but CQ_INIT_USER) -> weighted
 * sort-means (prune = 1) or plain weighted Lloyd (prune = 0) -> palette ->
 * map of every pixel of the image.  palette is device uint8[K][3] (entries
 * past k_used are zero); out_idx and out_rgb as in cq_map (nullable).  stats
 * (host, nullable) includes mse_img, over all H W pixels; mse_float divides
 * the final SSE by the pixels the histogram counted.  Synchronizes `stream`. */
cq_status cq_quantize(const uint8_t* img, int32_t H, int32_t W, int64_t row_stride_bytes,
                      int32_t subsample, int32_t K, cq_init_t scheme, uint64_t seed, int32_t max_iters, double tol,
                      int32_t prune, uint8_t* palette, uint8_t* out_idx, uint8_t* out_rgb,
                      cq_stats* stats /* host */, void* ws, size_t ws_bytes, void* stream);

/* For callers that cannot allocate memory (code under graph capture, tight
 * serving loops, harnesses that forbid allocation): cq_quantize with no
 * workspace argument.  Its workspace is a fixed device array inside the
 * library, 48 MiB on every GPU it runs on (held until the process ends), so
 * the image may have at most 1048576 (2^20) pixels: CQ_EINVAL beyond that.
 * Host staging uses a fixed host array.  The first call on a device sets it
 * up (the array's device address, two events for the status readback and
 * the library's readback stream); later calls on that device create,
 * allocate and free nothing.  The array keeps the last call's contents and
 * nothing in it has to start at zero.  Every call on a GPU shares that GPU's
 * array, so calls that overlapped there would race: the library serializes
 * calls from the threads of a process, and each returns only after its work
 * on `stream` is complete.  Results are identical to cq_quantize's.
 * Synchronizes `stream`. */
cq_status cq_quantize_noalloc(const uint8_t* img, int32_t H, int32_t W, int64_t row_stride_bytes,
                              int32_t subsample, int32_t K, cq_init_t scheme, uint64_t seed, int32_t max_iters,
                              double tol, int32_t prune, uint8_t* palette, uint8_t* out_idx, uint8_t* out_rgb,
                              cq_stats* stats /* host */, void* stream);

/* ------------------------------------------------------------------------
 * Batches: many images of different sizes and palette sizes quantized by one
 * sequence of launches (every kernel covers all jobs; a job that has stopped
 * iterating costs its blocks one early return).  Results are identical to
 * cq_quantize on each image alone.
 * ---------------------------------------------------------------------- */
typedef struct {
    const uint8_t* img;         /* device uint8 [H][W][3], rows row_stride_bytes apart  */
    int32_t H, W;
    int64_t row_stride_bytes;
    int32_t K;                  /* palette size, 1..256                                 */
    cq_init_t scheme;           /* any cq_init_t but CQ_INIT_USER                       */
    uint64_t seed;
    int32_t max_iters;          /* 1..100000                                            */
    double tol;                 /* >= 0                                                 */
    int32_t prune;              /* 1: sort-means, 0: full search                        */
    uint8_t* palette;           /* device uint8 [K][3] (entries past k_used are zero)   */
    uint8_t* out_idx;           /* device uint8 [H][W], nullable                         */
    uint8_t* out_rgb;           /* device uint8 [H][W][3], nullable                      */
    int32_t subsample;          /* 1: histogram of the pixels at even row and column    */
} cq_job;

/* Workspace bytes for a batch (one slot per job plus descriptors); 0 for an
 * invalid description.  At most 4096 jobs. */
size_t cq_batch_workspace_bytes(const cq_job* jobs /* host */, int32_t n_jobs);

/* Checks that the workspace is large enough and aligned for the batch; no
 * region of it needs clearing between calls, so no device work is done. */
cq_status cq_batch_workspace_prepare(const cq_job* jobs /* host */, int32_t n_jobs, void* ws,
                                     size_t ws_bytes, void* stream);

/* cq_quantize for every job of the batch.  stats (host, nullable) receives one
 * cq_stats per job.  Synchronizes `stream`. */
cq_status cq_quantize_batch(const cq_job* jobs /* host */, int32_t n_jobs, cq_stats* stats /* host */,
                            void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Serving engine: continuous batching of whole-quantizer jobs (cq_job, as in
 * cq_quantize) that arrive over time.  Each job's results are identical to
 * cq_quantize on that image alone, whatever else is in flight.
 *
 * The engine owns host bookkeeping only; its device memory is one
 * caller-owned workspace: a descriptor region for up to max_jobs jobs in
 * flight, followed by a pool from which every admitted job takes a slot of
 * cq_engine_job_bytes(job) bytes (its histogram, records, sums and lookup
 * table) until it finishes.  Jobs wait in submission order; the oldest is
 * admitted at the start of a step when fewer than max_jobs are in flight and
 * a free range of the pool fits its slot (first fit).  A step then
 *   1. runs the histogram and initialization of the jobs just admitted
 *      (their "prefill"),
 *   2. runs `iters` Lloyd iterations of every job in flight, each at its own
 *      iteration count (the first one a full search, sort-means after that),
 *   3. for every job that has stopped: palette, pixel map and statistics; its
 *      slot returns to the pool.
 * Nothing is in flight on `stream` between calls.  An engine is used from one
 * host thread at a time; the caller keeps each job's image and output buffers
 * alive until the job is reported done.
 * ---------------------------------------------------------------------- */
typedef struct cq_engine cq_engine;

/* One finished job, as reported by cq_engine_step. */
typedef struct {
    int64_t ticket;     /* from cq_engine_submit                                   */
    cq_status status;   /* CQ_OK, or CQ_EDEVICE if its initialization barrier timed out */
    int32_t reserved_;
    cq_stats stats;     /* as cq_quantize reports them (includes mse_img)          */
} cq_engine_done;

/* Pool bytes one job occupies while in flight; 0 for an invalid size. */
size_t cq_engine_job_bytes(int32_t H, int32_t W);

/* Workspace bytes for max_jobs (1..4096) jobs in flight and a pool of
 * pool_bytes; 0 for invalid arguments. */
size_t cq_engine_workspace_bytes(int32_t max_jobs, size_t pool_bytes);

/* Creates an engine over `ws` (device, 256-byte aligned, at least
 * cq_engine_workspace_bytes(max_jobs, 0) bytes; everything past the
 * descriptor region is the pool).  *engine (host) receives the handle.  No
 * device work. */
cq_status cq_engine_create(int32_t max_jobs, void* ws, size_t ws_bytes, void* stream,
                           cq_engine** engine /* host */);

/* Queues a job (validated as in cq_quantize_batch); *ticket (host) receives
 * its number, increasing from 1.  CQ_ECAPACITY if its slot is larger than
 * the whole pool (it could never be admitted).  No device work. */
cq_status cq_engine_submit(cq_engine* engine, const cq_job* job /* host */, int64_t* ticket /* host */);

/* One step (admission, prefill, `iters` iterations (0..100000), completion).
 * done (host) has room for `capacity` >= max_jobs entries; *n_done (host)
 * receives how many jobs finished in this step, in their admission order.
 * Synchronizes `stream`.  After an error other than an invalid argument
 * (CQ_EINVAL for iters, capacity or a null pointer) the engine accepts only
 * cq_engine_destroy. */
cq_status cq_engine_step(cq_engine* engine, int32_t iters, cq_engine_done* done /* host */, int32_t capacity,
                         int32_t* n_done /* host */);

/* Jobs waiting for admission, jobs in flight and pool bytes in use (each
 * output nullable, host). */
cq_status cq_engine_pending(const cq_engine* engine, int32_t* queued, int32_t* running, size_t* pool_used);

/* Frees the host bookkeeping (the workspace stays the caller's).  Jobs still
 * queued or in flight are dropped; after a failed step it first waits for
 * `stream`.  NULL is accepted. */
void cq_engine_destroy(cq_engine* engine);

/* ------------------------------------------------------------------------
 * Launch schedule of the Lloyd iterations.  How the iteration kernels are
 * tiled does not change any result, only the speed: the colours each
 * assignment block takes (few, so that a small batch still fills the GPU;
 * many, so that a large one pays less per block) and how often a pruned run
 * regroups its colours by (cluster, distance) for the sort-means scans
 * (every iteration keeps the scans of a wave short; less often saves the
 * regrouping's traffic).  A call that iterates over C unique colours in all
 * (the sum of N' over its jobs with N' > K) uses the last entry whose
 * min_colours <= C.  The built-in table holds the schedules that
 * paper_1101_0395_amd/autotune.py measured fastest on this GPU for batches
 * of those sizes.
 * ---------------------------------------------------------------------- */
typedef struct {
    int64_t min_colours;     /* the entry applies from this many colours on          */
    int32_t assign_chunk;    /* colours per assignment block: a multiple of 256 in
                                [256, 32768] (raised where a job would need more than
                                8192 blocks)                                           */
    int32_t regroup_period;  /* pruned runs regroup at iterations 1-4 and at every
                                multiple of this (>= 1)                                */
} cq_schedule;

/* Replaces the process-wide schedule table with n (1..32) entries whose
 * min_colours start at 0 and increase; n = 0 restores the built-in table.
 * CQ_EINVAL for anything else (the table is left as it was).  Takes effect
 * for calls and engine admissions that start afterwards; calls already
 * running keep the schedule they started with.  No device work. */
cq_status cq_set_schedule(const cq_schedule* table /* host */, int32_t n);

/* The current table: *n (host) receives its length and the first
 * min(n, capacity) entries are copied to table (host, nullable when
 * capacity is 0). */
cq_status cq_get_schedule(cq_schedule* table /* host */, int32_t capacity, int32_t* n /* host */);

/* Kernel timing for measurement harnesses (not needed for quantization).
 * While enabled, launches of the kernel named `kernel` (for example
 * "k_assign_walk", "k_hist_count", "k_map") are counted, and every
 * `every`-th of them (the 1st, the (every+1)-th, ...; every >= 1) is
 * bracketed by a pair of HIP events recorded on the stream it is launched
 * on, for at most max_launches bracketed launches.  Sampling keeps the
 * events' own cost out of the work being timed.  cq_timer_read waits for
 * those events and returns the number of bracketed launches, the sum of their
 * durations in milliseconds and the number of launches seen (nullable).
 * Process-global state: enable, run and read from one host thread. */
cq_status cq_timer_enable(const char* kernel, int32_t max_launches, int32_t every);
cq_status cq_timer_read(int64_t* launches /* host */, double* total_ms /* host */, int64_t* seen /* host */);
cq_status cq_timer_disable(void);

/* Releases the objects the library keeps for the whole process: pooled
 * pinned host buffers, its readback streams, the kernel timer's events and
 * the set-up of cq_quantize_noalloc.  Call it with no work of the library
 * pending, for instance before the process exits (so that they are gone
 * before the runtime's own teardown); later calls re-create what they need. */
void cq_release_resources(void);

/* Thread-local description of the last error on this thread ("" if none);
 * valid until the next cq_* call on the same thread. */
const char* cq_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CQ_H */
