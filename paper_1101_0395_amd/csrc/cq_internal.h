// Internal definitions shared by the HIP sources of libcq: workspace layout,
// the device-side control block, and small device helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/cq.h"

namespace cq {

constexpr uint32_t kNumKeys = 1u << 24;          // all 24-bit colours
constexpr uint32_t kBitmapWords = kNumKeys / 32;  // presence bitmap words
constexpr int kMaxK = 256;
constexpr int kMaxIters = 100000;
constexpr int64_t kMaxPixels = int64_t(1) << 28;

// Bitmap compaction: each block owns a contiguous run of bitmap words.
constexpr int kCompactThreads = 256;
constexpr int kCompactWordsPerThread = 8;
constexpr int kCompactWordsPerBlock = kCompactThreads * kCompactWordsPerThread;
constexpr int kCompactBlocks = kBitmapWords / kCompactWordsPerBlock;  // 256

// Initialization: one chunk of colours per block.
constexpr int kInitThreads = 256;
constexpr int kInitItemsPerThread = 4;
constexpr int kInitChunk = kInitThreads * kInitItemsPerThread;  // 1024
constexpr int kSelectThreads = 1024;

// Sorted centre table: row stride (entries) independent of K.
constexpr int kRow = kMaxK;

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
    uint32_t pad[46];
};
static_assert(sizeof(Meta) <= 512, "Meta must fit its slot");

// ---------------------------------------------------------------- layout
constexpr size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

struct Layout {
    size_t tbl, bitmap, lut, meta, trace, td, tm, sums, centers, palette, blk;
    size_t chunks, d2, keys, counts, assign;
    size_t fixed_end;  // end of the regions every call may use
    size_t total;      // end including the per-colour regions for n_cap colours
};

// n_cap: number of colours the per-colour regions must hold (0 = none).
// with_colour_arrays: also reserve keys/counts/assign (used by cq_quantize).
inline Layout make_layout(int64_t n_cap, bool with_colour_arrays)
{
    Layout L{};
    size_t o = 0;
    L.tbl = o;      o = align256(o + sizeof(uint32_t) * kNumKeys);
    L.bitmap = o;   o = align256(o + sizeof(uint32_t) * kBitmapWords);
    L.lut = o;      o = align256(o + kNumKeys);
    L.meta = o;     o = align256(o + 512);
    L.trace = o;    o = align256(o + sizeof(double) * kMaxIters);
    L.td = o;       o = align256(o + sizeof(double) * kMaxK * kRow);
    L.tm = o;       o = align256(o + kMaxK * kRow);
    L.sums = o;     o = align256(o + sizeof(uint64_t) * 5 * kMaxK);
    L.centers = o;  o = align256(o + sizeof(double) * 3 * kMaxK);
    L.palette = o;  o = align256(o + 3 * kMaxK);
    L.blk = o;      o = align256(o + sizeof(uint32_t) * 2 * kCompactBlocks);
    L.fixed_end = o;
    const size_t n = n_cap > 0 ? size_t(n_cap) : 0;
    const size_t nchunks = (n + kInitChunk - 1) / kInitChunk;
    L.chunks = o;   o = align256(o + sizeof(uint64_t) * (nchunks + 1));
    L.d2 = o;       o = align256(o + sizeof(uint32_t) * n);
    if (with_colour_arrays) {
        L.keys = o;   o = align256(o + sizeof(uint32_t) * n);
        L.counts = o; o = align256(o + sizeof(uint32_t) * n);
        L.assign = o; o = align256(o + n);
    } else {
        L.keys = L.counts = L.assign = 0;
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

// Uniform integer in [0, T), T >= 1: outputs below 2^64 mod T are redrawn.
__device__ __forceinline__ uint64_t uniform_below(uint64_t& s, uint64_t T)
{
    const uint64_t reject_below = (0ull - T) % T;
    for (;;) {
        const uint64_t r = splitmix64(s);
        if (r >= reject_below) return r % T;
    }
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
    T incl = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const T up = __shfl_up(incl, d, 64);
        if (lane >= d) incl += up;
    }
    if (lane == 63) tmp[wave] = incl;
    __syncthreads();
    if (wave == 0) {
        T w = lane < nwaves ? tmp[lane] : T(0);
        T wi = w;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const T up = __shfl_up(wi, d, 64);
            if (lane >= d) wi += up;
        }
        if (lane < nwaves) tmp[lane] = wi - w;  // exclusive wave offsets
        if (lane == nwaves - 1) tmp[63] = wi;   // block total (slot 63 is free)
    }
    __syncthreads();
    const T res = tmp[wave] + incl - v;
    if (total) *total = tmp[63];
    __syncthreads();
    return res;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const T o = __shfl_xor(v, d, 64);
        v = o > v ? o : v;
    }
    return v;
}

}  // namespace cq

// ---------------------------------------------------------------- host side
namespace cq {
void set_error(const char* fmt, ...);
void clear_error();
cq_status check_launch(const char* what);
}  // namespace cq

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
