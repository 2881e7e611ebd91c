// Data reduction of Section 2.2 (items 1 and 2): the unique colours of an image
// and their pixel counts, in ascending key order.
//
// The paper hashes colours into a chained table.  Here the 2^24 keys are split
// into kHistBuckets buckets of consecutive keys (the top 11 bits), and every
// tile of pixels is sorted by bucket in LDS before each bucket is counted in
// LDS, so no global counter is ever incremented by more than one block:
//   k_hist_part      per tile: pixels per bucket (LDS), their exclusive prefix
//                    over the buckets (the tile-local starts), the tile's low
//                    key bits sorted by bucket into the tile's own range, and
//                    the tile's row of counts and starts;
//   k_hist_count     per bucket (a fixed number of blocks per job): the
//                    bucket's segments of every tile counted in LDS, the
//                    non-zero counters compacted in ascending order at the
//                    bucket's place in the compacted arrays (the sum over the
//                    tiles of the bucket's tile-local starts);
//   k_hist_emit      per bucket (one wave each): the bucket's (key, count)
//                    pairs at its first output entry, and N'.
// The image is read from HBM once, into registers; every launch covers all
// jobs of a batch.
#include "cq_internal.h"

namespace cq {

constexpr int kHistThreads = 512;
static_assert(kHistTile <= 32768, "a tile's bucket counts and starts share one 32-bit word");

// Key of the pixel p (row-major index) of a job's histogram view.
__device__ __forceinline__ uint32_t load_key(const uint8_t* __restrict__ img, int64_t p, int32_t W,
                                             int64_t row_stride, int32_t pitch, bool packed)
{
    const uint8_t* q;
    if (packed) {
        q = img + 3 * p;
    } else {
        const uint32_t y = uint32_t(p) / uint32_t(W), x = uint32_t(p) - y * uint32_t(W);  // p < 2^28
        q = img + int64_t(y) * row_stride + pitch * x;
    }
    return (uint32_t(q[0]) << 16) | (uint32_t(q[1]) << 8) | uint32_t(q[2]);
}

// Keys of the four pixels held in three little-endian dwords:
// a = R0 G0 B0 R1, b = G1 B1 R2 G2, c = B2 R3 G3 B3.
__device__ __forceinline__ void unpack4(uint32_t a, uint32_t b, uint32_t c, uint32_t k[4])
{
    k[0] = ((a & 0xffu) << 16) | (a & 0xff00u) | ((a >> 16) & 0xffu);
    k[1] = ((a >> 24) << 16) | ((b & 0xffu) << 8) | ((b >> 8) & 0xffu);
    k[2] = (((b >> 16) & 0xffu) << 16) | ((b >> 24) << 8) | (c & 0xffu);
    k[3] = (((c >> 8) & 0xffu) << 16) | (((c >> 16) & 0xffu) << 8) | (c >> 24);
}

// The pixels of tile `lb` of a packed histogram view, held in registers:
// four pixels per thread per step in three dwords, plus one pixel of the
// tail of an image whose pixel count is not a multiple of 4.  visit(f) calls
// f(key, valid) for each of them.
struct PackedTile {
    static constexpr int kSteps = kHistTile / 4 / kHistThreads;
    uint32_t a[kSteps], b[kSteps], c[kSteps], tail;
    int64_t g0, g1, tp, p1;

    __device__ __forceinline__ void load(const JobDev& J, int64_t lb)
    {
        const uint8_t* __restrict__ img = gp(J.img);
        const uint32_t* __restrict__ w = reinterpret_cast<const uint32_t*>(img);
        const int64_t npix = hist_pixels(J);
        const int64_t p0 = lb * kHistTile;
        p1 = p0 + kHistTile < npix ? p0 + kHistTile : npix;
        g0 = p0 >> 2;
        g1 = p1 >> 2;  // whole groups of four pixels
#pragma unroll
        for (int s = 0; s < kSteps; ++s) {  // all loads first
            const int64_t g = g0 + s * kHistThreads + threadIdx.x;
            const bool in = g < g1;
            a[s] = in ? w[3 * g + 0] : 0u;
            b[s] = in ? w[3 * g + 1] : 0u;
            c[s] = in ? w[3 * g + 2] : 0u;
        }
        tp = g1 * 4 + threadIdx.x;
        tail = tp < p1 ? load_key(img, tp, J.hW, J.hstride, 3, true) : 0u;
    }

    template <typename F>
    __device__ __forceinline__ void visit(F f) const
    {
#pragma unroll
        for (int s = 0; s < kSteps; ++s) {
            const bool in = g0 + s * kHistThreads + threadIdx.x < g1;
            uint32_t k[4];
            unpack4(a[s], b[s], c[s], k);
#pragma unroll
            for (int q = 0; q < 4; ++q) f(k[q], in);
        }
        f(tail, tp < p1);
    }
};

// The pixels of tile `lb` of a strided view (every second pixel of every
// second row, or rows with padding), one pixel per thread per step, read
// again on every visit (the second time mostly from the L2).
struct StridedTile {
    const uint8_t* img;
    int64_t p0, p1, stride;
    int32_t W, pitch;

    __device__ __forceinline__ void load(const JobDev& J, int64_t lb)
    {
        img = gp(J.img);
        const int64_t npix = hist_pixels(J);
        p0 = lb * kHistTile;
        p1 = p0 + kHistTile < npix ? p0 + kHistTile : npix;
        stride = J.hstride;
        W = J.hW;
        pitch = J.hpitch;
    }

    template <typename F>
    __device__ __forceinline__ void visit(F f) const
    {
        for (int64_t p = p0; p < p1; p += kHistThreads) {
            const int64_t q = p + threadIdx.x;
            const bool in = q < p1;
            f(in ? load_key(img, q, W, stride, pitch, false) : 0u, in);
        }
    }
};

// Exclusive prefix of kHistBuckets values (one block of kHistThreads
// threads, kHistBuckets / kHistThreads consecutive values per thread);
// returns the total.
constexpr int kPerBucketThread = kHistBuckets / kHistThreads;  // 4
__device__ __forceinline__ uint32_t bucket_scan(const uint32_t* __restrict__ v, uint32_t* __restrict__ out,
                                                uint32_t* tmp)
{
    uint32_t vals[kPerBucketThread], sum = 0;
#pragma unroll
    for (int u = 0; u < kPerBucketThread; ++u) {
        vals[u] = v[threadIdx.x * kPerBucketThread + u];
        sum += vals[u];
    }
    uint32_t total = 0;
    uint32_t pre = block_exclusive_scan<uint32_t>(sum, tmp, &total);
#pragma unroll
    for (int u = 0; u < kPerBucketThread; ++u) {
        out[threadIdx.x * kPerBucketThread + u] = pre;
        pre += vals[u];
    }
    return total;
}

// ------------------------------------------------------------------ kernels
// One block per tile of kHistTile pixels, read from HBM once into registers.
// The tile's pixels are counted per bucket in LDS; the exclusive prefix of
// the counts over the buckets gives each bucket's start inside the tile; the
// pixels' low key bits are placed at those starts in LDS (the order inside a
// bucket is whatever the LDS atomics give) and stored to the tile's own
// range of hkeys in one coalesced pass.  The tile's counts and starts go to
// its row of hmat (tile-major), both in one word: count | start << 16 (each
// at most kHistTile = 2^15).
template <typename Tile>
__device__ __forceinline__ void part_tile(const JobDev& J, int lb, const Tile& tile, uint32_t* cnt,
                                          uint32_t* tmp, uint16_t* skey)
{
    // one LDS atomic per pixel: lanes with different buckets proceed together,
    // lanes that share one are serialized by the LDS unit
    tile.visit([&](uint32_t key, bool in) {
        if (in) atomicAdd(&cnt[key >> kHistLowBits], 1u);
    });
    __syncthreads();
    uint32_t* __restrict__ mrow = gp(J.hmat) + int64_t(lb) * kHistBuckets;
    {
        uint32_t v[kPerBucketThread], sum = 0;
#pragma unroll
        for (int u = 0; u < kPerBucketThread; ++u) {
            v[u] = cnt[threadIdx.x * kPerBucketThread + u];
            sum += v[u];
        }
        uint32_t pre = block_exclusive_scan<uint32_t>(sum, tmp, nullptr);
#pragma unroll
        for (int u = 0; u < kPerBucketThread; ++u) {
            const int b = threadIdx.x * kPerBucketThread + u;
            mrow[b] = v[u] | (pre << 16);
            cnt[b] = pre;  // becomes the bucket's cursor
            pre += v[u];
        }
    }
    __syncthreads();
    // each pixel's low bits to its bucket's cursor
    tile.visit([&](uint32_t key, bool in) {
        if (in) skey[atomicAdd(&cnt[key >> kHistLowBits], 1u)] = uint16_t(key & (kHistLow - 1));
    });
    __syncthreads();
    const int64_t npix = hist_pixels(J);
    const int64_t p0 = int64_t(lb) * kHistTile;
    const int n = int(p0 + kHistTile < npix ? kHistTile : npix - p0);
    // pairs of keys as one dword where the tile's range allows (it starts at
    // a multiple of kHistTile, so it is 4-byte aligned)
    uint32_t* __restrict__ out2 = reinterpret_cast<uint32_t*>(gp(J.hkeys) + p0);
    const uint32_t* s2 = reinterpret_cast<const uint32_t*>(skey);
    for (int i = threadIdx.x; i < n / 2; i += kHistThreads) out2[i] = s2[i];
    if ((n & 1) && threadIdx.x == 0) gp(J.hkeys)[p0 + n - 1] = skey[n - 1];
}

__global__ void __launch_bounds__(kHistThreads) k_hist_part(const JobDev* __restrict__ jobs,
                                                            const int* __restrict__ map, int B)
{
    __shared__ uint32_t cnt[kHistBuckets];
    __shared__ uint32_t tmp[64];
    __shared__ __align__(16) uint16_t skey[kHistTile];
    const int jb = find_job(map, B, blockIdx.x);
    const JobDev& J = jobs[jb];
    const int lb = blockIdx.x - map[jb];
    for (int t = threadIdx.x; t < kHistBuckets; t += kHistThreads) cnt[t] = 0u;
    if (J.hpacked) {
        PackedTile tile;
        tile.load(J, lb);
        __syncthreads();
        part_tile(J, lb, tile, cnt, tmp, skey);
    } else {
        StridedTile tile;
        tile.load(J, lb);
        __syncthreads();
        part_tile(J, lb, tile, cnt, tmp, skey);
    }
}

// Per job, hist_count_blocks(npix) blocks (a power of two from 64 or 256 up
// to one per bucket); block c of C takes the virtual buckets c, c + C, ....  Virtual
// bucket v = 8 j + x is bucket 256 (j / 32) + 32 x + j mod 32.  Workgroups
// are handed to the eight XCDs in turn, so x = v mod 8 is the block's XCD (C
// and every job's first block index are multiples of 8), and an XCD takes
// whole groups of 32 consecutive buckets, every eighth group: the 128-byte
// lines of hmat, and the neighbouring segments of hkeys, that a group's
// blocks share are fetched into one L2, while the work of any range of
// colours is spread over all XCDs.
//
// A bucket's pixels are its segment of every tile (tile t's row of hmat gives
// the segment's length and start inside the tile).  The non-empty segments
// are listed in tile order with their first position in the bucket's
// concatenation and the offset that turns a position into an hkeys index;
// the bucket's place in the compacted arrays hk2 / hcnt is the sum over the
// tiles of its tile-local starts (the number of pixels of all lower buckets).
// A bucket of at most one key per thread is ranked through a bitmap of the
// keys present.  A larger bucket is read in windows of kHistWindow positions:
// a bitmap marks the positions where a segment starts, and each wave reads 64
// consecutive positions per load, a lane's segment being the one before it
// plus the marks up to the lane (a population count), so no lane searches.
// Its keys are counted in LDS with adds that return nothing, so a wave's adds
// pipeline; all 8192 counters are read back (32 KiB of LDS, a fraction of a
// microsecond) and the non-zero ones cleared again.  The distinct keys go, in ascending order with their counts, to the bucket's
// place.  Dynamic LDS: the segment starts (tiles + 1 entries) and offsets
// (tiles entries).
constexpr int kHistWindow = 16384;       // positions per bitmap window
static_assert(kHistWindow % (64 * (kHistThreads / 64)) == 0, "whole 64-position words per wave");

__global__ void __launch_bounds__(kHistThreads, 4) k_hist_count(const JobDev* __restrict__ jobs,
                                                             const int* __restrict__ map, int B)
{
    __shared__ uint32_t c[kHistLow];
    __shared__ uint64_t tmp[64];
    // small buckets: keys present and their ranks; large ones: segment starts of a window
    __shared__ __align__(8) uint32_t s_bits[kHistWindow / 32];
    __shared__ uint32_t s_total, s_start, s_nseg;
    __shared__ int s_def[kHistBuckets / 64], s_ndef;  // buckets the wave pass leaves to the block (C >= 64)
    extern __shared__ uint32_t seg[];  // [ntiles + 1] starts, then [ntiles] offsets
    uint32_t* s_wpre = s_bits + kHistLow / 32;
    static_assert(kHistWindow / 32 >= 2 * (kHistLow / 32), "the small-bucket arrays fit the window bitmap");
    const int jb = find_job(map, B, blockIdx.x);
    const JobDev& J = jobs[jb];
    const int cb0 = blockIdx.x - map[jb];
    const int kCountBlocks = map[jb + 1] - map[jb];
    const int ntiles = int(hist_tiles(hist_pixels(J)));
    uint32_t* cstart = seg;
    int32_t* coff = reinterpret_cast<int32_t*>(seg + ntiles + 1);
    for (int t = threadIdx.x; t < kHistLow; t += kHistThreads) c[t] = 0u;
    for (int t = threadIdx.x; t < kHistLow / 32; t += kHistThreads) s_bits[t] = 0u;
    const uint32_t* __restrict__ mat = gp(J.hmat);
    const uint16_t* __restrict__ hkeys = gp(J.hkeys);
    constexpr int R = kHistLow / kHistThreads;  // 16 counters per thread in the compaction
    constexpr int kUnroll = 16;                 // loads in flight per lane
    static_assert(kHistBuckets % 256 == 0, "groups of 32 buckets dealt to eight XCDs");
    const int wave = int(threadIdx.x >> 6), lane = int(threadIdx.x & 63);
    // the block's buckets: virtual buckets cb0 + i C
    const int nmine = (kHistBuckets - cb0 + kCountBlocks - 1) / kCountBlocks;
    auto bucket_of = [&](int i) {
        const int vb = cb0 + i * kCountBlocks;
        const int j = vb >> 3;
        return (j >> 5) * 256 + (vb & 7) * 32 + (j & 31);
    };
    // Wave pass (small images, whose tiles fit one wave): wave w takes the
    // block's buckets w, w + 8, ... on its own, with no block barrier.  Lane t scans tile t's segment; an empty
    // bucket, or one of at most 64 pixels, is finished here: each lane takes
    // one pixel (its tile is the last non-empty one starting at or before
    // it: a prefix maximum over positions marked in a 64-byte LDS row), the
    // wave sorts the keys (bitonic, across lanes), and the first lane of each
    // run of equal keys writes the key and the run's length at its rank.
    // Larger buckets are left to the block-wide code below.
    const bool wave_pass = ntiles <= 64 && nmine <= kHistBuckets / 64;
    if (wave_pass) {
        if (threadIdx.x == 0) s_ndef = 0;
        __syncthreads();
        for (int wi = wave; wi < nmine; wi += kHistThreads / 64) {
            const int b = bucket_of(wi);
            const uint32_t m = lane < ntiles ? mat[int64_t(lane) * kHistBuckets + b] : 0u;
            const uint32_t len = m & 0xffffu, sst = m >> 16;
            const uint64_t v = (uint64_t(len != 0u) << 32) | len;
            const uint64_t incl = wave_incl_scan(v);
            const uint32_t pos = uint32_t(incl - v);
            const uint32_t total = uint32_t(read_lane(incl, 63));
            const uint32_t place = wave_sum(sst);
            if (lane == 0) gp(J.hbs)[b] = place;
            if (total == 0) {
                if (lane == 0) gp(J.hnu)[b] = 0u;
            } else if (total > 64) {
                if (lane == 0) s_def[atomicAdd(&s_ndef, 1)] = b;
            } else {
                uint8_t* own = reinterpret_cast<uint8_t*>(s_bits) + 64 * wave;
                own[lane] = 0;
                __builtin_amdgcn_wave_barrier();
                if (len != 0u) own[pos] = uint8_t(lane);
                __builtin_amdgcn_wave_barrier();
                const int t = wave_incl_max(int(own[lane]));
                const int32_t off = int32_t(lane * kHistTile + int(sst) - int(pos));
                const int32_t toff = __shfl(off, t, 64);
                uint32_t key = uint32_t(lane) < total ? uint32_t(hkeys[int64_t(toff) + lane]) : 0xffffu;
                // bitonic sort of the 64 lanes' keys, ascending
                for (int k = 2; k <= 64; k <<= 1) {
                    for (int jj = k >> 1; jj > 0; jj >>= 1) {
                        const uint32_t o = uint32_t(__shfl_xor(int(key), jj, 64));
                        const bool up = (lane & k) == 0, lower = (lane & jj) == 0;
                        key = (lower == up) ? (o < key ? o : key) : (o > key ? o : key);
                    }
                }
                const uint32_t prev = uint32_t(__shfl_up(int(key), 1, 64));
                const bool valid = key != 0xffffu;
                const bool head = valid && (lane == 0 || prev != key);
                const unsigned long long heads = __ballot(head);
                if (head) {
                    const unsigned long long below = (1ull << lane) - 1ull;
                    const unsigned long long after = heads & ~(below | (1ull << lane));
                    const uint32_t next = after ? uint32_t(__ffsll(after) - 1) : total;
                    const uint32_t rank = uint32_t(__popcll(heads & below));
                    gp(J.hk2)[place + rank] = uint16_t(key);
                    gp(J.hcnt)[place + rank] = next - uint32_t(lane);
                }
                if (lane == 0) gp(J.hnu)[b] = uint32_t(__popcll(heads));
            }
        }
        __syncthreads();
        // the LDS rows the waves used start the small-bucket bitmap, which
        // must be empty
        for (int t = threadIdx.x; t < kHistThreads / 4; t += kHistThreads) s_bits[t] = 0u;
        __syncthreads();
    }
    const int nlist = wave_pass ? s_ndef : nmine;
    for (int li = 0; li < nlist; ++li) {
        const int b = wave_pass ? s_def[li] : bucket_of(li);
        // the non-empty segments: one scan of (count of them, their lengths)
        uint64_t carry = 0;
        uint32_t place = 0;
        for (int t0 = 0; t0 < ntiles; t0 += kHistThreads) {
            const int t = t0 + threadIdx.x;
            const uint32_t m = t < ntiles ? mat[int64_t(t) * kHistBuckets + b] : 0u;
            const uint32_t len = m & 0xffffu, sst = m >> 16;
            uint64_t tot = 0;
            const uint64_t ex = carry + block_exclusive_scan<uint64_t>((uint64_t(len != 0u) << 32) | len, tmp, &tot);
            if (len != 0u) {
                const uint32_t js = uint32_t(ex >> 32), pos = uint32_t(ex);
                cstart[js] = pos;
                coff[js] = int32_t(t * kHistTile + int(sst) - int(pos));
            }
            carry += tot;
            place += sst;
        }
        place = wave_sum(place);
        if (lane == 0) reinterpret_cast<uint32_t*>(tmp)[wave] = place;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t p = 0;
            for (int w = 0; w < kHistThreads / 64; ++w) p += reinterpret_cast<uint32_t*>(tmp)[w];
            const uint32_t nseg = uint32_t(carry >> 32), total = uint32_t(carry);
            s_start = p;
            s_total = total;
            s_nseg = nseg;
            cstart[nseg] = total;
            gp(J.hbs)[b] = p;
        }
        __syncthreads();
        const uint32_t total = s_total, nseg = s_nseg;
        if (total == 0) {
            if (threadIdx.x == 0) gp(J.hnu)[b] = 0u;
            continue;
        }
        const uint32_t start = s_start;
        uint16_t* __restrict__ hk = gp(J.hk2) + start;
        uint32_t* __restrict__ hc = gp(J.hcnt) + start;
        // number of segments starting before position i (cstart ascending)
        auto starts_below = [&](uint32_t i) -> uint32_t {
            uint32_t lo = 0, hi = nseg;
            while (lo < hi) {
                const uint32_t mid = (lo + hi) >> 1;
                if (cstart[mid] < i) lo = mid + 1; else hi = mid;
            }
            return lo;
        };
        if (total <= kHistThreads) {
            // at most one key per thread: the first thread of each key marks
            // it in a bitmap, and a key's rank among the distinct keys is the
            // count of marks below it (an exclusive scan of the 256 words'
            // population counts, then the word's own lower bits)
            const uint32_t i = threadIdx.x;
            uint32_t key = 0xffffffffu;
            if (i < total) {
                const uint32_t js = starts_below(i + 1) - 1;  // the last segment starting at or before i
                key = uint32_t(hkeys[int64_t(coff[js]) + i]);
            }
            const bool first = key != 0xffffffffu && atomicAdd(&c[key], 1u) == 0u;
            if (first) atomicOr(&s_bits[key >> 5], 1u << (key & 31u));
            __syncthreads();
            const uint32_t word = threadIdx.x < kHistLow / 32 ? s_bits[threadIdx.x] : 0u;
            uint32_t nuniq = 0;
            const uint32_t wpre =
                block_exclusive_scan<uint32_t>(__popc(word), reinterpret_cast<uint32_t*>(tmp), &nuniq);
            if (threadIdx.x < kHistLow / 32) s_wpre[threadIdx.x] = wpre;
            __syncthreads();
            if (first) {
                const uint32_t w = key >> 5;
                const uint32_t rank = s_wpre[w] + __popc(s_bits[w] & ((1u << (key & 31u)) - 1u));
                hk[rank] = uint16_t(key);
                hc[rank] = c[key];
            }
            if (threadIdx.x == 0) gp(J.hnu)[b] = nuniq;
            __syncthreads();  // the counters and the bitmap are read
            if (first) c[key] = 0u;
            if (threadIdx.x < kHistLow / 32) s_bits[threadIdx.x] = 0u;
            __syncthreads();
            continue;
        }
        const uint64_t* bits64 = reinterpret_cast<const uint64_t*>(s_bits);
        const uint64_t below = lane == 63 ? ~uint64_t(0) : (uint64_t(2) << lane) - 1u;  // marks at or before the lane
        for (uint32_t w0 = 0; w0 < total; w0 += kHistWindow) {
            const uint32_t w1 = w0 + kHistWindow < total ? w0 + kHistWindow : total;
            // the window's segment starts, as marks
            for (int t = threadIdx.x; t < kHistWindow / 32; t += kHistThreads) s_bits[t] = 0u;
            const uint32_t jlo = starts_below(w0), jhi = starts_below(w1);
            __syncthreads();
            for (uint32_t js = jlo + threadIdx.x; js < jhi; js += kHistThreads) {
                const uint32_t r = cstart[js] - w0;
                atomicOr(&s_bits[r >> 5], 1u << (r & 31u));
            }
            __syncthreads();
            // wave w takes positions [a, e) of the window, whole words of 64
            const uint32_t pw = (w1 - w0 + kHistThreads - 1) / kHistThreads * 64;
            const uint32_t a = w0 + uint32_t(wave) * pw;
            const uint32_t e = a + pw < w1 ? a + pw : w1;
            uint32_t jbase = a < e ? starts_below(a) : 0u;  // segments starting before a
            for (uint32_t base = a; base < e; base += 64 * kUnroll) {
                uint32_t kq[kUnroll];
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) {
                    const uint32_t wb = base + 64 * u;
                    const uint64_t marks = wb < e ? bits64[(wb - w0) >> 6] : 0u;
                    // the lane's segment: the last one starting at or before it
                    const uint32_t js = jbase + uint32_t(__popcll(marks & below)) - 1u;
                    jbase += uint32_t(__popcll(marks));
                    const uint32_t i = wb + uint32_t(lane);
                    kq[u] = i < e ? uint32_t(hkeys[int64_t(coff[js]) + i]) : 0xffffffffu;
                }
#pragma unroll
                for (int u = 0; u < kUnroll; ++u)
                    if (kq[u] != 0xffffffffu) atomicAdd(&c[kq[u]], 1u);  // no return value: the adds pipeline
            }
            __syncthreads();  // the window's marks are read
        }
        // thread t owns counters [t R, (t + 1) R)
        uint32_t v[R];
        uint32_t nz = 0;
#pragma unroll
        for (int u = 0; u < R; ++u) {
            v[u] = c[threadIdx.x * R + u];
            nz += v[u] != 0u;
        }
        uint32_t nuniq = 0;
        uint32_t o = block_exclusive_scan<uint32_t>(nz, reinterpret_cast<uint32_t*>(tmp), &nuniq);
#pragma unroll
        for (int u = 0; u < R; ++u) {
            if (v[u] != 0u) {
                hk[o] = uint16_t(threadIdx.x * R + u);
                hc[o] = v[u];
                ++o;
                c[threadIdx.x * R + u] = 0u;
            }
        }
        if (threadIdx.x == 0) gp(J.hnu)[b] = nuniq;
        // the small-bucket bitmap must start empty
        for (int t = threadIdx.x; t < kHistLow / 32; t += kHistThreads) s_bits[t] = 0u;
        __syncthreads();
    }
}

// The (key, count) pairs of every bucket, at the bucket's first output entry
// (the exclusive prefix of the unique counts of the buckets, which each block
// computes for itself from the 2048 counts); entries past `capacity` are not
// written.  Wave w of a block takes the buckets w, w + 8, ... of the block's
// kEmitPerBlock * per_wave (per_wave 1, or 4 in a batch of many small images,
// where the prefix would otherwise cost more than the pairs); the first
// block of a job also stores N'.
constexpr int kEmitPerBlock = kHistThreads / 64;

__global__ void __launch_bounds__(kHistThreads) k_hist_emit(const JobDev* __restrict__ jobs, int per_wave)
{
    __shared__ uint32_t us[kHistBuckets];
    __shared__ uint32_t tmp[64];
    const int blocks_per_job = kHistBuckets / (kEmitPerBlock * per_wave);
    const JobDev& J = jobs[blockIdx.x / blocks_per_job];
    const int blk = blockIdx.x % blocks_per_job;
    const uint32_t n_unique = bucket_scan(gp(J.hnu), us, tmp);
    if (blk == 0 && threadIdx.x == 0) gp(J.meta)->n_unique = int64_t(n_unique);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    for (int i = 0; i < per_wave; ++i) {
        const int b = (blk * per_wave + i) * kEmitPerBlock + int(threadIdx.x >> 6);
        const uint32_t nb = gp(J.hnu)[b];
        if (nb == 0) continue;
        const uint32_t start = gp(J.hbs)[b];
        const uint16_t* __restrict__ hk = gp(J.hk2) + start;
        const uint32_t* __restrict__ hc = gp(J.hcnt) + start;
        const int64_t out = us[b];
        uint32_t* __restrict__ keys = gp(J.keys);
        uint32_t* __restrict__ counts = gp(J.counts);
        const int64_t capacity = J.capacity;
        constexpr int kUnroll = 16;  // loads in flight per lane (a bucket of a large image holds thousands)
        for (uint32_t j0 = 0; j0 < nb; j0 += kUnroll * 64) {
            uint32_t kq[kUnroll], cq[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const uint32_t j = j0 + u * 64 + lane;
                kq[u] = j < nb ? uint32_t(hk[j]) : 0u;
                cq[u] = j < nb ? hc[j] : 0u;
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const uint32_t j = j0 + u * 64 + lane;
                const int64_t o = out + j;
                if (j < nb && o < capacity) {
                    keys[o] = (uint32_t(b) << kHistLowBits) | kq[u];
                    counts[o] = cq[u];
                }
            }
        }
    }
}

// ------------------------------------------------------------------ host
int hist_blocks(int64_t npix) { return int(hist_tiles(npix)); }

// Counting blocks of a job: about one per 4096 pixels, a power of two
// between min_blocks (64 or 256) and one per bucket.
int hist_count_blocks(int64_t npix, int min_blocks)
{
    int c = min_blocks;
    while (c < kHistBuckets && int64_t(c) * 4096 < npix) c <<= 1;
    return c;
}

// Histogram of every job; N' is left in each job's meta.
// The unreduced data set of Algo. 1: one (key, count 1) record per pixel, in
// row-major order.
constexpr int kPixelKeyThreads = 256;
__global__ void __launch_bounds__(kPixelKeyThreads) k_pixel_keys(const uint8_t* __restrict__ img, int32_t W,
                                                                 int64_t row_stride, int64_t npix,
                                                                 uint32_t* __restrict__ keys,
                                                                 uint32_t* __restrict__ counts)
{
    const int64_t p = int64_t(blockIdx.x) * kPixelKeyThreads + threadIdx.x;
    if (p >= npix) return;
    keys[p] = load_key(img, p, W, row_stride, 3, false);
    counts[p] = 1u;
}

cq_status launch_pixel_keys(const uint8_t* img, int32_t H, int32_t W, int64_t row_stride, uint32_t* keys,
                            uint32_t* counts, hipStream_t s)
{
    const int64_t npix = int64_t(H) * W;  // at most 2^28
    const int blocks = int((npix + kPixelKeyThreads - 1) / kPixelKeyThreads);
    CQ_TIMED_LAUNCH("k_pixel_keys", s,
                    k_pixel_keys<<<blocks, kPixelKeyThreads, 0, s>>>(img, W, row_stride, npix, keys, counts));
    return CQ_OK;
}

cq_status launch_histogram(const JobDev* jobs, const int* maps, int B, int total_tiles, int total_count,
                           int max_tiles, int emit_per_wave, hipStream_t s)
{
    const int* tmap = maps + kMapHist * (B + 1);
    const int* cmap = maps + kMapHistCount * (B + 1);
    const size_t seg_lds = sizeof(uint32_t) * (2 * size_t(max_tiles) + 1);
    CQ_TIMED_LAUNCH("k_hist_part", s, k_hist_part<<<total_tiles, kHistThreads, 0, s>>>(jobs, tmap, B));
    CQ_TIMED_LAUNCH("k_hist_count", s, k_hist_count<<<total_count, kHistThreads, seg_lds, s>>>(jobs, cmap, B));
    CQ_TIMED_LAUNCH("k_hist_emit", s, k_hist_emit<<<kHistBuckets / (kEmitPerBlock * emit_per_wave) * B, kHistThreads, 0, s>>>(
                                           jobs, emit_per_wave));
    return CQ_OK;
}

}  // namespace cq
