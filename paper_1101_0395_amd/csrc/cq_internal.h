// Internal definitions shared by the HIP sources of libcq: workspace layout,
// the device-side control block, and small device helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/cq.h"

namespace cq {

constexpr uint32_t kNumKeys = 1u << 24;          // all 24-bit colours
constexpr int kMaxK = 256;
constexpr int kMaxIters = 100000;
constexpr int64_t kMaxPixels = int64_t(1) << 28;
constexpr int kMaxBatch = 4096;
constexpr int kMaxAssignBlocks = 8192;  // assignment blocks of one job (so a block has at most 32768 colours)

// Histogram: keys split into kHistBuckets buckets of kHistLow consecutive keys
// (bucket = key >> kHistLowBits); pixels are taken kHistTile at a time.
constexpr int kHistLowBits = 13;
constexpr int kHistLow = 1 << kHistLowBits;
constexpr int kHistBuckets = 1 << (24 - kHistLowBits);
constexpr int kHistTile = 32768;

__host__ __device__ __forceinline__ int64_t hist_tiles(int64_t npix)
{
    const int64_t t = (npix + kHistTile - 1) / kHistTile;
    return t > 0 ? t : 1;
}

// Cooperative initialization: at most kInitMaxBlocks blocks of kInitThreads
// threads per team.  Thread t of a block owns a run of R consecutive colours;
// every round the block publishes a tagged value and each thread the sum of
// its run (both for two round parities).
constexpr int kInitMaxBlocks = 256;
constexpr int kInitThreads = 1024;

// Sorted centre table: row stride (entries) independent of K.
constexpr int kRow = kMaxK;

// One entry of a sorted table row: the centre (c0, c1, c2) and its squared
// distance d from the row's own centre, so that a scan needs no second lookup.
struct alignas(32) Rec {
    double c0, c1, c2, d;
};

// Entries a row walk reads per round, and the padding past the last row that
// lets the final round of any row read whole rounds.
constexpr int kWalk = 4;      // table entries per round of a sort-means walk
constexpr int kTablePad = 8;  // entries after the last row: a walk's last round (and the one loaded ahead) may reach past its row

// Cluster statistics of one iteration (uint64 each): n_k, S_k (3 per
// cluster), Q_k, then the number of unique colours and the counting-sort
// cursor of every (cluster, distance bucket) pair, pair index k kBuckets + b.
// Two such blocks alternate between iterations.
constexpr int kBuckets = 16;
constexpr int kSumN = 0;
constexpr int kSumS = kMaxK;
constexpr int kSumQ = 4 * kMaxK;
// (u64 slot offsets) the colour counts and the regrouping cursors per
// (cluster, bucket) pair are uint32 (a count is below 2^28), two per slot
constexpr int kSumColours = 5 * kMaxK;
constexpr int kSumCursor = kSumColours + kMaxK * kBuckets / 2;
// (pruned runs) the largest squared distance of a cluster's colours to the
// centre they were assigned to, as the bit pattern of a non-negative double
// (such patterns order as the values do)
constexpr int kSumMaxD = kSumCursor + kMaxK * kBuckets / 2;
constexpr int kSumStride = kSumMaxD + kMaxK;

// Device-side control block, one per workspace.
struct Meta {
    uint64_t rng;         // splitmix64 state of the init draws
    uint64_t ndc;         // distance calculations, accumulated over iterations
    uint64_t near_ties;   // near-tie colour-iterations, accumulated
    uint64_t sq_err;      // pixel-map squared-error sum
    uint64_t total_w;     // k-means: sum of the colour weights (pixels)
    int64_t n_unique;     // result of the histogram compaction
    int64_t chosen;       // init: colour index picked in the current round
    int32_t done;         // k-means: 1 once the stopping rule has fired
    int32_t iters;        // k-means: iterations run
    int32_t converged;    // k-means: stopped by the SSE test
    int32_t bad_input;    // k-means: a non-finite initial centre was seen
    double sse_prev;      // SSE of the previous iteration
    double sse_last;      // SSE of the last iteration
    uint32_t barrier;     // arrival counter of the grid barrier of a cooperative launch
    int32_t sync_error;   // set when a grid barrier waited past its spin limit
    int32_t cur_it;       // k-means: iteration whose cluster sums are being built
    uint32_t pick_epoch;  // init: rounds whose pick has been published
    uint32_t pad0;
    int64_t pick_slot[2]; // init: published pick (colour index) by round parity
    uint32_t pad[38];
};
static_assert(sizeof(Meta) <= 512, "Meta must fit its slot");

constexpr size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// ---------------------------------------------------------------- jobs
// One image of a launch.  Every kernel takes a device array of jobs and, where
// jobs need different numbers of blocks, a prefix map of B + 1 block offsets
// (block b belongs to the job j with map[j] <= b < map[j + 1]).
// Device code sees the buffers of a job descriptor as global-memory pointers,
// so loads through them are global or scalar loads rather than generic ones;
// host code sees plain pointers of the same size.
#if defined(__HIP_DEVICE_COMPILE__)
#define CQ_GLOBAL __attribute__((address_space(1)))
#else
#define CQ_GLOBAL
#endif

struct JobDev {
    const uint8_t CQ_GLOBAL* img;
    int64_t stride;
    int32_t H, W;
    int32_t K, scheme, max_iters, prune;
    uint64_t seed;
    double tol;
    uint8_t CQ_GLOBAL* palette;
    uint8_t CQ_GLOBAL* out_idx;
    uint8_t CQ_GLOBAL* out_rgb;
    uint16_t CQ_GLOBAL* hkeys;  // histogram: low key bits of the pixels, each tile's sorted by bucket
    uint16_t CQ_GLOBAL* hk2;    // histogram: compacted low key bits, bucket after bucket
    uint32_t CQ_GLOBAL* hcnt;   // histogram: compacted counts, bucket after bucket
    uint32_t CQ_GLOBAL* hmat;   // histogram: tile x bucket, pixel count | start inside the tile << 16
    uint32_t CQ_GLOBAL* hnu;    // histogram: unique colours per bucket
    uint32_t CQ_GLOBAL* hbs;    // histogram: first compacted entry of each bucket
    uint8_t CQ_GLOBAL* lut;
    Meta CQ_GLOBAL* meta;
    double CQ_GLOBAL* trace;
    Rec CQ_GLOBAL* rec;   // sorted table rows (kMaxK x kRow)
    uint32_t CQ_GLOBAL* prow; // colour table: the palette's distance rows, sorted (kMaxK x kRow)
    uint8_t CQ_GLOBAL* ord; // every row's whole centre order (kMaxK x kRow bytes), the next sort's start
    unsigned long long CQ_GLOBAL* sums;
    unsigned long long CQ_GLOBAL* part;  // per assignment block: distance count, near-tie count
    uint64_t CQ_GLOBAL* vals;  // init: tagged block values, then the run sums
    uint32_t CQ_GLOBAL* d2;
    uint64_t CQ_GLOBAL* grp;  // k-means colour records, two buffers of n (shares d2's region)
    uint32_t CQ_GLOBAL* keys;
    uint32_t CQ_GLOBAL* counts;
    uint8_t CQ_GLOBAL* assign;
    double CQ_GLOBAL* centers;
    double CQ_GLOBAL* cprev;  // pruned runs: the centres the current iteration assigns to
    int64_t capacity;    // entries of keys / counts
    int64_t n;           // unique colours, set once the histogram is known
    int64_t chunk;       // colours per assignment / LUT block
    int64_t init_C;      // colours per block of the initialization team
    int32_t init_first;  // first block of the initialization team
    int32_t init_blocks; // blocks of the team (0: no cooperative initialization)
    int32_t packed;      // image rows are contiguous and 4-byte aligned
    int32_t map_k;       // palette entries the pixel map searches
    int32_t regroup_period;  // pruned runs: regroup the colours at iterations 1-4 and every this many
    int32_t lut_rec;     // the colour table starts each colour's search at its cluster's entry
                         // (a pruned run's final records) instead of searching every entry
    // the pixels the histogram counts: the whole image, or after 2:1
    // subsampling its pixels at even row and column
    int64_t hstride;     // bytes between rows of the view
    int32_t hH, hW;      // rows and columns of the view
    int32_t hpitch;      // bytes between pixels of a view row (3 or 6)
    int32_t hpacked;     // the view is the whole image, its rows contiguous and 4-byte aligned
    int32_t map_direct;  // the map searches the palette per pixel: the colour table only
                         // covers the colours the histogram counted
    int32_t pad2_;
};

// Pixels the histogram of a job counts.
__host__ __device__ __forceinline__ int64_t hist_pixels(const JobDev& J) { return int64_t(J.hH) * J.hW; }

// Pruned runs regroup their colour records (a counting sort by cluster and
// distance bucket) in the update step of iterations 1-4 and of every
// multiple of `period` after that; between regroupings the records keep their
// order and only their cluster fields change.  Results never depend on the
// order, only the speed of the sort-means passes does.
__host__ __device__ __forceinline__ bool regroup_at(int it, int period)
{
    return it <= 4 || it % period == 0;
}

// Record buffer (0 or 1) that holds the colour records during iteration it:
// the number of regroupings before it, modulo 2.
__host__ __device__ __forceinline__ int record_buffer(int it, int period)
{
    const int before = it - 1;
    int c = before < 4 ? before : 4;
    if (before >= 5) c += before / period - 4 / period;
    return c & 1;
}

// Read-only view of global memory that a kernel does not write: loads with a
// wave-uniform address through it become scalar loads.
#if defined(__HIP_DEVICE_COMPILE__)
#define CQ_CONST __attribute__((address_space(4)))
#else
#define CQ_CONST
#endif
template <typename T>
__device__ __forceinline__ const T CQ_CONST* cp(T CQ_GLOBAL* p)
{
    return (const T CQ_CONST*)p;
}

// Host-side stores into a descriptor, and host-side reads of one.
template <typename T>
inline T CQ_GLOBAL* to_dev(T* p) { return (T CQ_GLOBAL*)p; }
template <typename T>
inline T* from_dev(T CQ_GLOBAL* p) { return (T*)p; }

// A descriptor pointer as a plain pointer; the compiler keeps treating every
// access derived from it as global memory.
template <typename T>
__device__ __forceinline__ T* gp(T CQ_GLOBAL* p)
{
    return (T*)p;
}

// Per-job results gathered for one device-to-host copy.
struct JobResult {
    int64_t n_unique;
    uint64_t ndc, near_ties, sq_err, total_w;
    double sse_last;
    int32_t done, iters, converged, bad_input, sync_error, pad_;
};

// LBG initialization: the splitting vector (eps, eps, eps), and the stopping
// threshold and iteration limit of the k-means refinement after each stage
// (the threshold is the paper's, Section 3.3).
constexpr double kLbgEps = 1.0;
constexpr double kLbgTol = 0.001;
constexpr int32_t kLbgMaxIters = 100;

// WU initialization: five uint64 statistics over a 33^3 grid (32 levels per
// channel plus a zero border).
constexpr size_t kWuTableBytes = sizeof(uint64_t) * 5 * 33 * 33 * 33;

enum MapId {
    kMapHist = 0,
    kMapHistCount,   // histogram counting blocks
    kMapAssign,      // every job with iterations (first iteration, final pass)
    kMapAssignFull,  // unpruned jobs (full searches after the first iteration)
    kMapAssignWalk,  // pruned jobs (sort-means passes)
    kMapUpdate,      // table blocks and regrouping blocks
    kMapUpdateTable, // table blocks only (iterations without regrouping)
    kMapLut,
    kMapPalRows,     // palette rows sorted by distance (colour tables searched from the clusters)
    kMapPix,
    kMapInit,
    kMapVarTiles,    // VAR: colour tiles
    kMapVarGroups,   // VAR: one block per centre
    kMapWu,          // WU: blocks of colours
    kMapDenTiles,    // DEN: colour tiles
    kMapDenCentres,  // DEN: one block per centre
    kNumMaps
};

__device__ __forceinline__ int find_job(const int* __restrict__ map, int B, int block)
{
    int lo = 0, hi = B;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (map[mid] <= block) lo = mid; else hi = mid;
    }
    return lo;
}

// Descriptor region: jobs, block maps, gathered results.
// Descriptor region of a batch: job descriptors, block maps, and two slots of
// control-block copies (read back alternately while iterations continue).
inline size_t desc_bytes(int B)
{
    return align256(sizeof(JobDev) * size_t(B)) + align256(sizeof(int) * size_t(kNumMaps) * size_t(B + 1)) +
           2 * align256(sizeof(JobResult) * size_t(B));
}
inline size_t desc_maps_off(int B) { return align256(sizeof(JobDev) * size_t(B)); }
inline size_t desc_results_off(int B)
{
    return desc_maps_off(B) + align256(sizeof(int) * size_t(kNumMaps) * size_t(B + 1));
}

// ---------------------------------------------------------------- layout

struct Layout {
    size_t lut, meta, trace, rec, prow, ord, sums, centers, cprev, palette, part, desc;
    size_t chunks, work, hkeys, hk2, hcnt, hmat, hnu, hbs, keys, counts, assign;
    size_t fixed_end;  // end of the regions every call may use
    size_t total;      // end including the per-pixel and per-colour regions
};

// npix: pixels the histogram regions must serve (0 = none); n_cap: colours
// the per-colour regions must hold (0 = none); with_colour_arrays: also
// reserve keys / counts / assign (used by cq_quantize).  The histogram's
// staging and the initialization / k-means buffers share one work region:
// the histogram is done before either starts.
inline Layout make_layout(int64_t npix, int64_t n_cap, bool with_colour_arrays)
{
    Layout L{};
    size_t o = 0;
    L.lut = o;      o = align256(o + kNumKeys);
    L.meta = o;     o = align256(o + 512);
    L.trace = o;    o = align256(o + sizeof(double) * kMaxIters);
    // the sorted table: kTablePad entries past the last row for the final round of a walk
    L.rec = o;      o = align256(o + sizeof(Rec) * (kMaxK * kRow + kTablePad));
    L.prow = o;     o = align256(o + sizeof(uint32_t) * kMaxK * kRow);
    L.ord = o;      o = align256(o + size_t(kMaxK) * kRow);  // the rows' centre order, one byte per entry
    L.sums = o;     o = align256(o + sizeof(uint64_t) * 2 * kSumStride);  // two iterations
    L.centers = o;  o = align256(o + sizeof(double) * 3 * kMaxK);
    L.cprev = o;    o = align256(o + sizeof(double) * 3 * kMaxK);
    L.palette = o;  o = align256(o + 3 * kMaxK);
    L.part = o;     o = align256(o + sizeof(uint64_t) * 2 * kMaxAssignBlocks);
    L.desc = o;     o = align256(o + desc_bytes(1));
    L.fixed_end = o;
    const size_t n = n_cap > 0 ? size_t(n_cap) : 0;
    const size_t np = npix > 0 ? size_t(npix) : 0;
    // init: tagged block values and picks, both for two round parities
    L.chunks = o;   o = align256(o + sizeof(uint64_t) * 2 * (kInitMaxBlocks + 1));
    // work region
    L.work = o;
    size_t hist = 0;
    if (np > 0) {
        L.hkeys = o + hist; hist = align256(hist + sizeof(uint16_t) * np);
        L.hk2 = o + hist;   hist = align256(hist + sizeof(uint16_t) * np);
        L.hcnt = o + hist;  hist = align256(hist + sizeof(uint32_t) * np);
        L.hmat = o + hist;  hist = align256(hist + sizeof(uint32_t) * size_t(kHistBuckets) * size_t(hist_tiles(npix)));
        L.hnu = o + hist;   hist = align256(hist + sizeof(uint32_t) * kHistBuckets);
        L.hbs = o + hist;   hist = align256(hist + sizeof(uint32_t) * kHistBuckets);
    }
    // init (colours beyond what LDS holds): D^2, kInitThreads R entries per
    // block (below n + kInitThreads per block); k-means: two uint64 records
    // per colour
    const size_t d2_init = n > 0 ? sizeof(uint32_t) * (n + size_t(kInitThreads + 1) * kInitMaxBlocks) : 0;
    const size_t d2_km = sizeof(uint64_t) * 2 * n;
    // init WU: the moment table
    const size_t wu = n > 0 ? kWuTableBytes : 0;
    size_t work = hist > d2_init ? hist : d2_init;
    work = work > d2_km ? work : d2_km;
    work = work > wu ? work : wu;
    o = align256(o + work);
    if (with_colour_arrays) {
        L.keys = o;   o = align256(o + sizeof(uint32_t) * n);
        L.counts = o; o = align256(o + sizeof(uint32_t) * n);
        L.assign = o; o = align256(o + n);
    } else {
        // memberships of the k-means refinement of an LBG initialization
        L.keys = L.counts = 0;
        L.assign = 0;
        if (n > 0) {
            L.assign = o;
            o = align256(o + n);
        }
    }
    L.total = o;
    return L;
}

template <typename T>
inline T* at(void* ws, size_t off) { return reinterpret_cast<T*>(static_cast<char*>(ws) + off); }

// ---------------------------------------------------------------- device helpers
__device__ __forceinline__ void key_rgb(uint32_t key, int& r, int& g, int& b)
{
    r = int((key >> 16) & 255u);
    g = int((key >> 8) & 255u);
    b = int(key & 255u);
}

// Exact integer squared distance between colours.
__device__ __forceinline__ uint32_t dist_u32(int r0, int g0, int b0, int r1, int g1, int b1)
{
    const int dr = r0 - r1, dg = g0 - g1, db = b0 - b1;
    return uint32_t(dr * dr + dg * dg + db * db);
}

// FP64 squared distance in the fixed order (d0*d0 + d1*d1) + d2*d2, each
// operation rounded separately (no fused multiply-add).
__device__ __forceinline__ double dist_f64(double x0, double x1, double x2,
                                           double c0, double c1, double c2)
{
#pragma clang fp contract(off)
    const double d0 = x0 - c0;
    const double d1 = x1 - c1;
    const double d2 = x2 - c2;
    return d0 * d0 + d1 * d1 + d2 * d2;
}

// splitmix64 (Steele, Lea & Flood 2014).
__device__ __forceinline__ uint64_t splitmix64(uint64_t& s)
{
    s += 0x9E3779B97F4A7C15ull;
    uint64_t z = s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// splitmix64 is counter-based: the i-th output (0-based) of the stream whose
// state starts at s0 is the finalizer applied to s0 + (i + 1) gamma.
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t s0, uint64_t i)
{
    uint64_t s = s0 + i * 0x9E3779B97F4A7C15ull;
    return splitmix64(s);
}

// r mod T (T >= 1), exactly.  The quotient is estimated in FP64 twice (the
// first estimate is within 2^12 / T + 1 of r / T, so the remainder left by it
// has magnitude below 2^12 + 2 T, which the second estimate resolves to within
// one step) and the integer remainder is corrected; anything outside [0, T)
// after that falls back to the integer division, so the result never depends
// on the estimates.
__host__ __device__ __forceinline__ uint64_t mod_u64(uint64_t r, uint64_t T)
{
    if (T == 1) return 0;
    const double dT = double(T);
    const double q1d = double(r) / dT;  // below 2^63 for T >= 2
    const uint64_t q1 = uint64_t(q1d);
    int64_t m = int64_t(r - q1 * T);
    const int64_t q2 = int64_t(__builtin_floor(double(m) / dT));
    m -= q2 * int64_t(T);
    if (m < 0) m += int64_t(T);
    if (m >= int64_t(T)) m -= int64_t(T);
    if (T >= (1ull << 52) || m < 0 || m >= int64_t(T)) return r % T;
    return uint64_t(m);
}

// r mod T as mod_u64, with the quotient estimates taken as products by
// inv ~ 1 / T instead of quotients (the exact remainder is checked the same
// way, so the result never depends on inv).
__device__ __forceinline__ uint64_t mod_u64_inv(uint64_t r, uint64_t T, double inv)
{
    if (T == 1) return 0;
    const uint64_t q1 = uint64_t(double(r) * inv);  // below 2^64 for T >= 2
    int64_t m = int64_t(r - q1 * T);
    const int64_t q2 = int64_t(__builtin_floor(double(m) * inv));
    m -= q2 * int64_t(T);
    if (m < 0) m += int64_t(T);
    if (m >= int64_t(T)) m -= int64_t(T);
    if (T >= (1ull << 52) || m < 0 || m >= int64_t(T)) return r % T;
    return uint64_t(m);
}

// Uniform integer in [0, T), T >= 1: outputs below 2^64 mod T are redrawn.
// The remainder of each draw is computed beside the threshold's (they do not
// depend on each other), with one reciprocal for both.
__device__ __forceinline__ uint64_t uniform_below(uint64_t& s, uint64_t T)
{
    const double inv = 1.0 / double(T);
    const uint64_t reject_below = mod_u64_inv(0ull - T, T, inv);
    uint64_t r = splitmix64(s);
    uint64_t m = mod_u64_inv(r, T, inv);
    while (r < reject_below) {
        r = splitmix64(s);
        m = mod_u64_inv(r, T, inv);
    }
    return m;
}

// ---------------------------------------------------------------- wave-wide
// Scans and reductions over the 64 lanes of a wave with DPP moves (register
// to register, no LDS round trip): an inclusive scan inside each row of 16
// lanes by shifts of 1, 2, 4 and 8 lanes, then the last lane of a row added to
// the rows after it (row_bcast:15, row_bcast:31).  Every lane of the wave must
// be active.  A lane with no source lane, or in a row that a move skips,
// receives `old`.
constexpr int kDppRowShr1 = 0x111, kDppRowShr2 = 0x112, kDppRowShr4 = 0x114, kDppRowShr8 = 0x118;
constexpr int kDppRowBcast15 = 0x142, kDppRowBcast31 = 0x143;

template <int kCtrl, int kRowMask, typename T>
__device__ __forceinline__ T dpp_move(T old, T v)
{
    static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit values");
    if constexpr (sizeof(T) == 4) {
        const int r = __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, old), __builtin_bit_cast(int, v), kCtrl,
                                                  kRowMask, 0xf, false);
        return __builtin_bit_cast(T, r);
    } else {
        const uint64_t o = __builtin_bit_cast(uint64_t, old), x = __builtin_bit_cast(uint64_t, v);
        const uint32_t lo = uint32_t(__builtin_amdgcn_update_dpp(int(uint32_t(o)), int(uint32_t(x)), kCtrl,
                                                                 kRowMask, 0xf, false));
        const uint32_t hi = uint32_t(__builtin_amdgcn_update_dpp(int(uint32_t(o >> 32)), int(uint32_t(x >> 32)),
                                                                 kCtrl, kRowMask, 0xf, false));
        return __builtin_bit_cast(T, (uint64_t(hi) << 32) | lo);
    }
}

template <typename T>
__device__ __forceinline__ T read_lane(T v, int lane)
{
    static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit values");
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
    } else {
        const uint64_t x = __builtin_bit_cast(uint64_t, v);
        const uint32_t lo = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(x)), lane));
        const uint32_t hi = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(x >> 32)), lane));
        return __builtin_bit_cast(T, (uint64_t(hi) << 32) | lo);
    }
}

// Inclusive prefix sum over the lanes.
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T x)
{
    const T z = T(0);
    x += dpp_move<kDppRowShr1, 0xf>(z, x);
    x += dpp_move<kDppRowShr2, 0xf>(z, x);
    x += dpp_move<kDppRowShr4, 0xf>(z, x);
    x += dpp_move<kDppRowShr8, 0xf>(z, x);
    x += dpp_move<kDppRowBcast15, 0xa>(z, x);
    x += dpp_move<kDppRowBcast31, 0xc>(z, x);
    return x;
}

// Inclusive prefix maximum over the lanes (a lane without a source keeps its
// own value, so any ordered type works).
template <typename T>
__device__ __forceinline__ T wave_incl_max(T x)
{
    auto mx = [](T a, T b) { return b > a ? b : a; };
    x = mx(x, dpp_move<kDppRowShr1, 0xf>(x, x));
    x = mx(x, dpp_move<kDppRowShr2, 0xf>(x, x));
    x = mx(x, dpp_move<kDppRowShr4, 0xf>(x, x));
    x = mx(x, dpp_move<kDppRowShr8, 0xf>(x, x));
    x = mx(x, dpp_move<kDppRowBcast15, 0xa>(x, x));
    x = mx(x, dpp_move<kDppRowBcast31, 0xc>(x, x));
    return x;
}

// Sum and maximum over the lanes, the same value in every lane.
template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
    return read_lane(wave_incl_scan(v), 63);
}

template <typename T>
__device__ __forceinline__ T wave_max(T v)
{
    return read_lane(wave_incl_max(v), 63);
}

// Block-wide exclusive scan of one value per thread (blockDim.x <= 1024,
// multiple of 64).  `tmp` must hold 64 entries.  Returns the
// exclusive prefix; *total receives the block sum.
template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T* tmp, T* total)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nwaves = blockDim.x >> 6;
    const T incl = wave_incl_scan(v);
    if (lane == 63) tmp[wave] = incl;
    __syncthreads();
    if (wave == 0) {
        const T w = lane < nwaves ? tmp[lane] : T(0);
        const T wi = wave_incl_scan(w);
        if (lane < nwaves) tmp[lane] = wi - w;  // exclusive wave offsets
        if (lane == nwaves - 1) tmp[63] = wi;   // block total (slot 63 is free)
    }
    __syncthreads();
    const T res = tmp[wave] + incl - v;
    if (total) *total = tmp[63];
    __syncthreads();
    return res;
}

// Barrier of a team of co-resident blocks (a cooperative launch).  `counter`
// only grows: the e-th barrier (1-based) of a team of G blocks completes when
// it reaches target = e * G.
// Arrival is a release add (earlier writes of the block become visible first);
// the wait polls with relaxed loads, which do not invalidate the L2 on every
// poll, and a single acquire fence follows.  A wait longer than the spin limit,
// or an error raised by another block, makes every block return false so that
// the kernel can end.
constexpr uint32_t kSpinLimit = 1u << 22;

__device__ __forceinline__ bool grid_barrier(uint32_t* counter, uint32_t target, int32_t* error)
{
    __shared__ int s_ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        uint32_t spins = 0;
        while (__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
                ++spins > kSpinLimit) {
                __hip_atomic_store(error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
}

// Wait (thread 0 of the block) until *flag >= target, published with a
// release store by another block; relaxed polling, one acquire fence, and the
// same spin limit and error convention as grid_barrier.
__device__ __forceinline__ bool wait_flag(uint32_t* flag, uint32_t target, int32_t* error)
{
    __shared__ int s_ok2;
    if (threadIdx.x == 0) {
        int ok = 1;
        uint32_t spins = 0;
        while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
                ++spins > kSpinLimit) {
                __hip_atomic_store(error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        s_ok2 = ok;
    }
    __syncthreads();
    return s_ok2 != 0;
}



}  // namespace cq

// ---------------------------------------------------------------- host side
namespace cq {
void set_error(const char* fmt, ...);
void clear_error();
cq_status check_launch(const char* what);
// Event bracketing of one kernel launch (active only for the timed kernel).
void timer_begin(const char* kernel, hipStream_t s);
void timer_end(const char* kernel, hipStream_t s);
}  // namespace cq

// Launch a kernel (the variadic part is the launch statement), bracketed by
// the kernel timer, then check the launch.
#define CQ_TIMED_LAUNCH(name, s, ...)                                                \
    do {                                                                             \
        ::cq::timer_begin(name, s);                                                  \
        __VA_ARGS__;                                                                 \
        ::cq::timer_end(name, s);                                                    \
        CQ_LAUNCH_CHECK(name);                                                       \
    } while (0)

#define CQ_HIP_TRY(expr)                                                             \
    do {                                                                             \
        hipError_t e_ = (expr);                                                      \
        if (e_ != hipSuccess) {                                                      \
            ::cq::set_error("%s failed: %s", #expr, hipGetErrorString(e_));          \
            return CQ_EDEVICE;                                                       \
        }                                                                            \
    } while (0)

#define CQ_LAUNCH_CHECK(what)                                                        \
    do {                                                                             \
        cq_status s_ = ::cq::check_launch(what);                                     \
        if (s_ != CQ_OK) return s_;                                                  \
    } while (0)
