// Data reduction of Section 2.2 (items 1 and 2): the unique colours of an image
// and their pixel counts.
//
// The paper hashes colours into a chained table.  Here each block first folds
// a tile of pixels into a small open-addressing table in LDS, then the 2^24
// possible colours index a dense uint32 count table directly, and a 2^24-bit
// presence bitmap records which entries were touched.  Compaction walks the 2 MiB bitmap
// (not the 64 MiB table), so the unique colours come out in ascending key order
// with a prefix sum over word popcounts, and only the touched table entries are
// read and reset.  Both regions are left all-zero for the next call.
#include "cq_internal.h"

namespace cq {

// Tile aggregation in LDS: each block folds the pixels of a tile into an
// open-addressing table of (key + 1, count) pairs, then adds every distinct key
// of the tile to the global table with one atomic (and sets its bitmap bit).
// Keys that find no free slot within kHashProbes probes go straight to the
// global table.
constexpr int kHistThreads = 256;
constexpr int kHashBits = 12;
constexpr int kHashSlots = 1 << kHashBits;     // 4096 slots, 32 KiB of LDS
constexpr int kHistTile = kHashSlots / 2;      // pixels per tile (load <= 1/2)
constexpr int kHashProbes = 16;

__device__ __forceinline__ void tile_insert(uint32_t key, uint32_t* hkey, uint32_t* hcnt,
                                            uint32_t* __restrict__ tbl, uint32_t* __restrict__ bitmap)
{
    uint32_t slot = (key * 0x9E3779B1u) >> (32 - kHashBits);
    const uint32_t tag = key + 1u;
    for (int probe = 0; probe < kHashProbes; ++probe) {
        const uint32_t old = atomicCAS(hkey + slot, 0u, tag);
        if (old == 0u || old == tag) {
            atomicAdd(hcnt + slot, 1u);
            return;
        }
        slot = (slot + 1u) & (kHashSlots - 1);
    }
    atomicAdd(tbl + key, 1u);
    atomicOr(bitmap + (key >> 5), 1u << (key & 31u));
}

__device__ __forceinline__ void tile_flush(uint32_t* hkey, uint32_t* hcnt, uint32_t* __restrict__ tbl,
                                           uint32_t* __restrict__ bitmap)
{
    __syncthreads();
    for (int slot = threadIdx.x; slot < kHashSlots; slot += kHistThreads) {
        const uint32_t tag = hkey[slot];
        if (tag == 0u) continue;
        const uint32_t key = tag - 1u;
        atomicAdd(tbl + key, hcnt[slot]);
        atomicOr(bitmap + (key >> 5), 1u << (key & 31u));
        hkey[slot] = 0u;
        hcnt[slot] = 0u;
    }
    __syncthreads();
}

__device__ __forceinline__ uint32_t load_key(const uint8_t* __restrict__ img, int64_t p, int32_t W,
                                             int64_t row_stride, bool packed)
{
    const uint8_t* q;
    if (packed) {
        q = img + 3 * p;
    } else {
        const int64_t y = p / W, x = p - y * W;
        q = img + y * row_stride + 3 * x;
    }
    return (uint32_t(q[0]) << 16) | (uint32_t(q[1]) << 8) | uint32_t(q[2]);
}

// Each block folds up to kTilesPerBlock consecutive tiles of its job.
// Packed images (row stride 3W, 4-byte aligned) are read four pixels (three
// dwords) per thread.
constexpr int kTilesPerBlock = 4;

__global__ void __launch_bounds__(kHistThreads) k_hist_tiles(const JobDev* __restrict__ jobs,
                                                             const int* __restrict__ map, int B)
{
    __shared__ uint32_t hkey[kHashSlots];
    __shared__ uint32_t hcnt[kHashSlots];
    const int jb = find_job(map, B, blockIdx.x);
    const JobDev& J = jobs[jb];
    const int lb = blockIdx.x - map[jb];
    const uint8_t* __restrict__ img = gp(J.img);
    uint32_t* __restrict__ tbl = gp(J.tbl);
    uint32_t* __restrict__ bitmap = gp(J.bitmap);
    const int32_t W = J.W;
    const int64_t row_stride = J.stride;
    const bool packed = J.packed != 0;
    for (int t = threadIdx.x; t < kHashSlots; t += kHistThreads) {
        hkey[t] = 0u;
        hcnt[t] = 0u;
    }
    __syncthreads();
    const int64_t npix = int64_t(J.H) * W;
    const int64_t ntiles = (npix + kHistTile - 1) / kHistTile;
    const uint32_t* w = reinterpret_cast<const uint32_t*>(img);
    for (int64_t tile = int64_t(lb) * kTilesPerBlock; tile < ntiles && tile < int64_t(lb + 1) * kTilesPerBlock; ++tile) {
        const int64_t p0 = tile * kHistTile;
        const int64_t p1 = p0 + kHistTile < npix ? p0 + kHistTile : npix;
        if (packed && p1 - p0 == kHistTile) {
            // full tile: 4 pixels per thread per step, 12 bytes as three dwords
            for (int64_t g = (p0 >> 2) + threadIdx.x; g < (p1 >> 2); g += kHistThreads) {
                const uint32_t a = w[3 * g + 0];
                const uint32_t b = w[3 * g + 1];
                const uint32_t c = w[3 * g + 2];
                // little-endian bytes: a = R0 G0 B0 R1, b = G1 B1 R2 G2, c = B2 R3 G3 B3
                tile_insert(((a & 0xffu) << 16) | (a & 0xff00u) | ((a >> 16) & 0xffu), hkey, hcnt, tbl, bitmap);
                tile_insert(((a >> 24) << 16) | ((b & 0xffu) << 8) | ((b >> 8) & 0xffu), hkey, hcnt, tbl, bitmap);
                tile_insert((((b >> 16) & 0xffu) << 16) | ((b >> 24) << 8) | (c & 0xffu), hkey, hcnt, tbl, bitmap);
                tile_insert((((c >> 8) & 0xffu) << 16) | (((c >> 16) & 0xffu) << 8) | (c >> 24), hkey, hcnt, tbl, bitmap);
            }
        } else {
            for (int64_t p = p0 + threadIdx.x; p < p1; p += kHistThreads)
                tile_insert(load_key(img, p, W, row_stride, packed), hkey, hcnt, tbl, bitmap);
        }
        tile_flush(hkey, hcnt, tbl, bitmap);
    }
}

// Pass 1 of the compaction: popcount of each block's bitmap words.
__global__ void __launch_bounds__(kCompactThreads) k_bitmap_count(const JobDev* __restrict__ jobs)
{
    __shared__ uint32_t tmp[64];
    const JobDev& J = jobs[blockIdx.x / kCompactBlocks];
    const uint32_t blk_id = blockIdx.x % kCompactBlocks;
    const uint32_t* __restrict__ bitmap = gp(J.bitmap);
    const uint32_t base = blk_id * kCompactWordsPerBlock + threadIdx.x * kCompactWordsPerThread;
    const uint4* p = reinterpret_cast<const uint4*>(bitmap + base);
    const uint4 u = p[0], v = p[1];
    uint32_t c = __popc(u.x) + __popc(u.y) + __popc(u.z) + __popc(u.w) + __popc(v.x) + __popc(v.y) +
                 __popc(v.z) + __popc(v.w);
    c = wave_sum(c);
    if ((threadIdx.x & 63) == 0) tmp[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (int w = 0; w < kCompactThreads / 64; ++w) s += tmp[w];
        gp(J.blk)[blk_id] = s;
    }
}

// Pass 2: exclusive scan of the per-block counts (one block of 256 threads).
__global__ void __launch_bounds__(kCompactBlocks) k_bitmap_scan(const JobDev* __restrict__ jobs)
{
    __shared__ uint32_t tmp[64];
    const JobDev& J = jobs[blockIdx.x];
    uint32_t total = 0;
    const uint32_t off = block_exclusive_scan<uint32_t>(J.blk[threadIdx.x], tmp, &total);
    gp(J.blk)[kCompactBlocks + threadIdx.x] = off;
    if (threadIdx.x == 0) gp(J.meta)->n_unique = int64_t(total);
}

// Pass 3: emit the keys in ascending order and clear the bitmap words.  Keys
// past `capacity` are not written; their table entries are reset here.
__global__ void __launch_bounds__(kCompactThreads) k_bitmap_emit(const JobDev* __restrict__ jobs)
{
    __shared__ uint32_t tmp[64];
    const JobDev& J = jobs[blockIdx.x / kCompactBlocks];
    const uint32_t blk_id = blockIdx.x % kCompactBlocks;
    uint32_t* __restrict__ bitmap = gp(J.bitmap);
    uint32_t* __restrict__ tbl = gp(J.tbl);
    uint32_t* __restrict__ keys = gp(J.keys);
    const int64_t capacity = J.capacity;
    const uint32_t base = blk_id * kCompactWordsPerBlock + threadIdx.x * kCompactWordsPerThread;
    uint4* p = reinterpret_cast<uint4*>(bitmap + base);
    const uint4 u = p[0], v = p[1];
    const uint32_t words[8] = {u.x, u.y, u.z, u.w, v.x, v.y, v.z, v.w};
    uint32_t c = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) c += __popc(words[j]);
    const uint32_t local = block_exclusive_scan<uint32_t>(c, tmp, nullptr);
    int64_t o = int64_t(J.blk[kCompactBlocks + blk_id]) + local;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        uint32_t wbits = words[j];
        while (wbits) {
            const uint32_t bit = __ffs(wbits) - 1;
            wbits &= wbits - 1;
            const uint32_t key = (base + j) * 32u + bit;
            if (o < capacity)
                keys[o] = key;
            else
                tbl[key] = 0u;
            ++o;
        }
    }
    if (c) {
        p[0] = make_uint4(0, 0, 0, 0);
        p[1] = make_uint4(0, 0, 0, 0);
    }
}

// Pass 4: counts[o] = table[keys[o]], and the entry is reset.
constexpr int kGatherBlocks = 64;  // per job

__global__ void __launch_bounds__(256) k_gather_counts(const JobDev* __restrict__ jobs)
{
    const JobDev& J = jobs[blockIdx.x / kGatherBlocks];
    const int lb = blockIdx.x % kGatherBlocks;
    const uint32_t* __restrict__ keys = gp(J.keys);
    uint32_t* __restrict__ counts = gp(J.counts);
    uint32_t* __restrict__ tbl = gp(J.tbl);
    const int64_t n = gp(J.meta)->n_unique < J.capacity ? gp(J.meta)->n_unique : J.capacity;
    const int64_t stride = int64_t(kGatherBlocks) * blockDim.x;
    for (int64_t o = int64_t(lb) * blockDim.x + threadIdx.x; o < n; o += stride) {
        const uint32_t key = keys[o];
        counts[o] = tbl[key];
        tbl[key] = 0u;
    }
}

// Workspace preparation: zero the count table and the bitmap with a plain
// fill kernel.
__global__ void __launch_bounds__(256) k_fill_zero(uint4* __restrict__ p, int64_t n16)
{
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n16; i += stride)
        p[i] = make_uint4(0, 0, 0, 0);
}

// ------------------------------------------------------------------ host
cq_status launch_fill_zero(void* p, size_t bytes, hipStream_t s)
{
    const int64_t n16 = int64_t(bytes / 16);
    CQ_TIMED_LAUNCH("k_fill_zero", s, k_fill_zero<<<2048, 256, 0, s>>>(reinterpret_cast<uint4*>(p), n16));
    return CQ_OK;
}

int hist_blocks(int64_t npix)
{
    const int64_t tiles = (npix + kHistTile - 1) / kHistTile;
    return int((tiles + kTilesPerBlock - 1) / kTilesPerBlock);
}

// Histogram and compaction of every job; N' is left in each job's meta.
cq_status launch_histogram(const JobDev* jobs, const int* maps, int B, int total_hist_blocks, hipStream_t s)
{
    CQ_TIMED_LAUNCH("k_hist_tiles", s, k_hist_tiles<<<total_hist_blocks, kHistThreads, 0, s>>>(jobs, maps + kMapHist * (B + 1), B));
    CQ_TIMED_LAUNCH("k_bitmap_count", s, k_bitmap_count<<<kCompactBlocks * B, kCompactThreads, 0, s>>>(jobs));
    CQ_TIMED_LAUNCH("k_bitmap_scan", s, k_bitmap_scan<<<B, kCompactBlocks, 0, s>>>(jobs));
    CQ_TIMED_LAUNCH("k_bitmap_emit", s, k_bitmap_emit<<<kCompactBlocks * B, kCompactThreads, 0, s>>>(jobs));
    CQ_TIMED_LAUNCH("k_gather_counts", s, k_gather_counts<<<kGatherBlocks * B, 256, 0, s>>>(jobs));
    return CQ_OK;
}

}  // namespace cq
