// Data reduction of Section 2.2 (items 1 and 2): the unique colours of an image
// and their pixel counts, in ascending key order.
//
// The paper hashes colours into a chained table.  Here the 2^24 keys are split
// into kHistBuckets buckets of consecutive keys (the top 11 bits), and the
// pixels are partitioned by bucket before each bucket is counted in LDS, so no
// global counter is ever incremented by more than one block:
//   k_hist_buckets   per tile of pixels: pixels per bucket (LDS), one column
//                    of the bucket x tile count matrix;
//   k_hist_colscan   per bucket: exclusive prefix of its row over the tiles,
//                    and the bucket's pixel total;
//   k_hist_starts    per job: the first pixel slot of every bucket;
//   k_hist_scatter   per tile: every pixel's low 13 key bits into its bucket's
//                    range (bucket start + the tile's prefix + rank);
//   k_hist_count     per bucket (a fixed number of blocks per job): counts of
//                    its 8192 keys in LDS, then the non-zero ones compacted in
//                    ascending order in place;
//   k_hist_ustarts   per job: the first output entry of every bucket and N';
//   k_hist_emit      per bucket (one wave each): the bucket's (key, count)
//                    pairs from there.
// Every launch covers all jobs of a batch.
#include "cq_internal.h"

namespace cq {

constexpr int kHistThreads = 512;

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

// Calls f(key, valid) for the pixels of tile `lb` of the histogram view, four
// pixels per thread per step from three dword loads when the view is packed.
template <typename F>
__device__ __forceinline__ void for_tile_pixels(const JobDev& J, int64_t lb, F f)
{
    const uint8_t* __restrict__ img = gp(J.img);
    const int64_t npix = hist_pixels(J);
    const int64_t p0 = lb * kHistTile;
    const int64_t p1 = p0 + kHistTile < npix ? p0 + kHistTile : npix;
    if (J.hpacked) {
        const uint32_t* __restrict__ w = reinterpret_cast<const uint32_t*>(img);
        const int64_t g0 = p0 >> 2, g1 = p1 >> 2;  // whole groups of four pixels
        constexpr int kSteps = kHistTile / 4 / kHistThreads;
        uint32_t a[kSteps], b[kSteps], c[kSteps];
#pragma unroll
        for (int s = 0; s < kSteps; ++s) {  // all loads first
            const int64_t g = g0 + s * kHistThreads + threadIdx.x;
            const bool in = g < g1;
            a[s] = in ? w[3 * g + 0] : 0u;
            b[s] = in ? w[3 * g + 1] : 0u;
            c[s] = in ? w[3 * g + 2] : 0u;
        }
#pragma unroll
        for (int s = 0; s < kSteps; ++s) {
            const bool in = g0 + s * kHistThreads + threadIdx.x < g1;
            uint32_t k[4];
            unpack4(a[s], b[s], c[s], k);
#pragma unroll
            for (int q = 0; q < 4; ++q) f(k[q], in);
        }
        // the last tile of an image whose pixel count is not a multiple of 4
        const int64_t tail = g1 * 4 + threadIdx.x;
        const bool tin = tail < p1;
        f(tin ? load_key(img, tail, J.hW, J.hstride, 3, true) : 0u, tin);
    } else {
        for (int64_t p = p0; p < p1; p += kHistThreads) {
            const int64_t q = p + threadIdx.x;
            const bool in = q < p1;
            f(in ? load_key(img, q, J.hW, J.hstride, J.hpitch, false) : 0u, in);
        }
    }
}

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
__global__ void __launch_bounds__(kHistThreads) k_hist_buckets(const JobDev* __restrict__ jobs,
                                                               const int* __restrict__ map, int B)
{
    __shared__ uint32_t cnt[kHistBuckets];
    const int jb = find_job(map, B, blockIdx.x);
    const JobDev& J = jobs[jb];
    const int lb = blockIdx.x - map[jb];
    for (int t = threadIdx.x; t < kHistBuckets; t += kHistThreads) cnt[t] = 0u;
    __syncthreads();
    // one LDS atomic per pixel: lanes with different buckets proceed together,
    // lanes that share one are serialized by the LDS unit
    for_tile_pixels(J, lb, [&](uint32_t key, bool in) {
        if (in) atomicAdd(&cnt[key >> kHistLowBits], 1u);
    });
    __syncthreads();
    const int64_t ntiles = hist_tiles(hist_pixels(J));
    uint32_t* __restrict__ mat = gp(J.hmat);
    for (int t = threadIdx.x; t < kHistBuckets; t += kHistThreads) mat[t * ntiles + lb] = cnt[t];
}

// One block per (job, bucket): exclusive prefix over the tiles, in place.
__global__ void __launch_bounds__(256) k_hist_colscan(const JobDev* __restrict__ jobs)
{
    __shared__ uint32_t tmp[64];
    const JobDev& J = jobs[blockIdx.x / kHistBuckets];
    const int b = blockIdx.x % kHistBuckets;
    const int64_t ntiles = hist_tiles(hist_pixels(J));
    uint32_t* __restrict__ row = gp(J.hmat) + b * ntiles;
    uint32_t carry = 0;
    for (int64_t t0 = 0; t0 < ntiles; t0 += blockDim.x) {
        const int64_t t = t0 + threadIdx.x;
        const uint32_t v = t < ntiles ? row[t] : 0u;
        uint32_t tot = 0;
        const uint32_t ex = block_exclusive_scan<uint32_t>(v, tmp, &tot);
        if (t < ntiles) row[t] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) gp(J.hbt)[b] = carry;
}

// One block per job: first pixel slot of every bucket.
__global__ void __launch_bounds__(kHistThreads) k_hist_starts(const JobDev* __restrict__ jobs)
{
    __shared__ uint32_t tmp[64];
    const JobDev& J = jobs[blockIdx.x];
    bucket_scan(gp(J.hbt), gp(J.hbs), tmp);
}

// One block per job: first output entry of every bucket, and N'.
__global__ void __launch_bounds__(kHistThreads) k_hist_ustarts(const JobDev* __restrict__ jobs)
{
    __shared__ uint32_t tmp[64];
    const JobDev& J = jobs[blockIdx.x];
    const uint32_t total = bucket_scan(gp(J.hnu), gp(J.hus), tmp);
    if (threadIdx.x == 0) gp(J.meta)->n_unique = int64_t(total);
}

__global__ void __launch_bounds__(kHistThreads) k_hist_scatter(const JobDev* __restrict__ jobs,
                                                               const int* __restrict__ map, int B)
{
    __shared__ uint32_t pos[kHistBuckets];
    const int jb = find_job(map, B, blockIdx.x);
    const JobDev& J = jobs[jb];
    const int lb = blockIdx.x - map[jb];
    const int64_t ntiles = hist_tiles(hist_pixels(J));
    const uint32_t* __restrict__ mat = gp(J.hmat);
    const uint32_t* __restrict__ bs = gp(J.hbs);
    for (int b = threadIdx.x; b < kHistBuckets; b += kHistThreads)
        pos[b] = bs[b] + mat[b * ntiles + lb];  // bucket start + this tile's prefix
    __syncthreads();
    uint16_t* __restrict__ hk = gp(J.hkeys);
    for_tile_pixels(J, lb, [&](uint32_t key, bool in) {
        if (in) hk[atomicAdd(&pos[key >> kHistLowBits], 1u)] = uint16_t(key & (kHistLow - 1));
    });
}

// Per job, hist_count_blocks(npix) blocks (a power of two up to one per
// bucket), block c of C taking the buckets c, c + C, ...: a bucket of at most
// one key per thread is ranked through a bitmap of the keys present; a larger
// bucket's keys are counted in LDS, then the non-zero
// counters are compacted in ascending key order over the front of the
// bucket's own range (its keys are all read before anything is written).  The
// 8192 counters are cleared once; a bucket marks the groups of 64 counters it
// touches, and only those are read back and cleared again, so a bucket costs
// in proportion to its contents.
constexpr int kGroups = kHistLow / 64;  // 128 groups of 64 counters

__global__ void __launch_bounds__(kHistThreads) k_hist_count(const JobDev* __restrict__ jobs,
                                                             const int* __restrict__ map, int B)
{
    __shared__ uint32_t c[kHistLow];
    __shared__ uint32_t touched[kGroups / 32];
    __shared__ uint32_t tmp[64];
    __shared__ uint32_t s_total[kHistBuckets / 256], s_start[kHistBuckets / 256];  // this block's buckets
    __shared__ uint32_t s_bits[kHistLow / 32], s_wpre[kHistLow / 32];  // small buckets: keys present, ranks
    const int jb = find_job(map, B, blockIdx.x);
    const JobDev& J = jobs[jb];
    const int cb0 = blockIdx.x - map[jb];
    const int kCountBlocks = map[jb + 1] - map[jb];  // at least 256
    for (int t = threadIdx.x; t < kHistLow; t += kHistThreads) c[t] = 0u;
    if (threadIdx.x < kGroups / 32) touched[threadIdx.x] = 0u;
    if (threadIdx.x < kHistLow / 32) s_bits[threadIdx.x] = 0u;
    // every bucket's pixel count and first slot at once, not one bucket after another
    if (threadIdx.x < kHistBuckets / 256) {
        const int b = cb0 + threadIdx.x * kCountBlocks;
        s_total[threadIdx.x] = b < kHistBuckets ? gp(J.hbt)[b] : 0u;
        s_start[threadIdx.x] = b < kHistBuckets ? gp(J.hbs)[b] : 0u;
    }
    __syncthreads();
    constexpr int R = kHistLow / kHistThreads;  // 16 counters per thread in the compaction
    constexpr int kUnroll = 8;
    for (int b = cb0, q = 0; b < kHistBuckets; b += kCountBlocks, ++q) {
        const uint32_t total = s_total[q];
        if (total == 0) {
            if (threadIdx.x == 0) gp(J.hnu)[b] = 0u;
            continue;
        }
        const uint32_t start = s_start[q];
        uint16_t* __restrict__ hk = gp(J.hkeys) + start;
        uint32_t* __restrict__ hc = gp(J.hcnt) + start;
        if (total <= kHistThreads) {
            // at most one key per thread: the first thread of each key marks
            // it in a bitmap, and a key's rank among the distinct keys is the
            // count of marks below it (an exclusive scan of the 256 words'
            // population counts, then the word's own lower bits)
            const uint32_t key = threadIdx.x < total ? uint32_t(hk[threadIdx.x]) : 0xffffffffu;
            const bool first = key != 0xffffffffu && atomicAdd(&c[key], 1u) == 0u;
            if (first) atomicOr(&s_bits[key >> 5], 1u << (key & 31u));
            __syncthreads();
            const uint32_t word = threadIdx.x < kHistLow / 32 ? s_bits[threadIdx.x] : 0u;
            uint32_t nuniq = 0;
            const uint32_t wpre = block_exclusive_scan<uint32_t>(__popc(word), tmp, &nuniq);
            if (threadIdx.x < kHistLow / 32) s_wpre[threadIdx.x] = wpre;
            __syncthreads();
            if (first) {
                const uint32_t w = key >> 5;
                const uint32_t rank = s_wpre[w] + __popc(s_bits[w] & ((1u << (key & 31u)) - 1u));
                hk[rank] = uint16_t(key);  // every key was read before the first barrier
                hc[rank] = c[key];
            }
            if (threadIdx.x == 0) gp(J.hnu)[b] = nuniq;
            __syncthreads();  // the counters and the bitmap are read
            if (first) c[key] = 0u;
            if (threadIdx.x < kHistLow / 32) s_bits[threadIdx.x] = 0u;
            __syncthreads();
            continue;
        }
        // eight keys in flight per thread before their LDS atomics
        for (uint32_t i0 = 0; i0 < total; i0 += kUnroll * kHistThreads) {
            uint32_t kq[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const uint32_t i = i0 + u * kHistThreads + threadIdx.x;
                kq[u] = i < total ? uint32_t(hk[i]) : 0xffffffffu;
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                if (kq[u] == 0xffffffffu) continue;
                if (atomicAdd(&c[kq[u]], 1u) == 0u) atomicOr(&touched[kq[u] >> 11], 1u << ((kq[u] >> 6) & 31u));
            }
        }
        __syncthreads();
        // thread t owns counters [t R, (t + 1) R), inside group t R / 64
        const int g = threadIdx.x * R / 64;
        const bool hit = (touched[g >> 5] >> (g & 31)) & 1u;
        uint32_t v[R];
        uint32_t nz = 0;
#pragma unroll
        for (int u = 0; u < R; ++u) {
            v[u] = hit ? c[threadIdx.x * R + u] : 0u;
            nz += v[u] != 0u;
        }
        uint32_t nuniq = 0;
        uint32_t o = block_exclusive_scan<uint32_t>(nz, tmp, &nuniq);
        if (hit) {
#pragma unroll
            for (int u = 0; u < R; ++u) {
                if (v[u] != 0u) {
                    hk[o] = uint16_t(threadIdx.x * R + u);
                    hc[o] = v[u];
                    ++o;
                    c[threadIdx.x * R + u] = 0u;
                }
            }
        }
        if (threadIdx.x == 0) gp(J.hnu)[b] = nuniq;
        __syncthreads();  // every touched counter is cleared and the mask was read
        if (threadIdx.x < kGroups / 32) touched[threadIdx.x] = 0u;
        __syncthreads();
    }
}

// One block per (job, bucket): the bucket's pairs into keys / counts at the
// prefix of the unique counts; entries past `capacity` are not written.
// One wave per bucket, kHistThreads / 64 buckets per block.
constexpr int kEmitPerBlock = kHistThreads / 64;

__global__ void __launch_bounds__(kHistThreads) k_hist_emit(const JobDev* __restrict__ jobs)
{
    constexpr int kBlocksPerJob = kHistBuckets / kEmitPerBlock;
    const JobDev& J = jobs[blockIdx.x / kBlocksPerJob];
    const int b = (blockIdx.x % kBlocksPerJob) * kEmitPerBlock + int(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const uint32_t nb = gp(J.hnu)[b];
    if (nb == 0) return;
    const uint32_t start = gp(J.hbs)[b];
    const uint16_t* __restrict__ hk = gp(J.hkeys) + start;
    const uint32_t* __restrict__ hc = gp(J.hcnt) + start;
    const int64_t out = gp(J.hus)[b];
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

// ------------------------------------------------------------------ host
int hist_blocks(int64_t npix) { return int(hist_tiles(npix)); }

// Counting blocks of a job: about one per 4096 pixels, a power of two
// between 256 and one per bucket.
int hist_count_blocks(int64_t npix)
{
    int c = 256;
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
                           hipStream_t s)
{
    const int* tmap = maps + kMapHist * (B + 1);
    const int* cmap = maps + kMapHistCount * (B + 1);
    CQ_TIMED_LAUNCH("k_hist_buckets", s, k_hist_buckets<<<total_tiles, kHistThreads, 0, s>>>(jobs, tmap, B));
    CQ_TIMED_LAUNCH("k_hist_colscan", s, k_hist_colscan<<<kHistBuckets * B, 256, 0, s>>>(jobs));
    CQ_TIMED_LAUNCH("k_hist_starts", s, k_hist_starts<<<B, kHistThreads, 0, s>>>(jobs));
    CQ_TIMED_LAUNCH("k_hist_scatter", s, k_hist_scatter<<<total_tiles, kHistThreads, 0, s>>>(jobs, tmap, B));
    CQ_TIMED_LAUNCH("k_hist_count", s, k_hist_count<<<total_count, kHistThreads, 0, s>>>(jobs, cmap, B));
    CQ_TIMED_LAUNCH("k_hist_ustarts", s, k_hist_ustarts<<<B, kHistThreads, 0, s>>>(jobs));
    CQ_TIMED_LAUNCH("k_hist_emit", s, k_hist_emit<<<kHistBuckets / kEmitPerBlock * B, kHistThreads, 0, s>>>(jobs));
    return CQ_OK;
}

}  // namespace cq
