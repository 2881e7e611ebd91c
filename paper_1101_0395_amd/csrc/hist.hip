// Data reduction of Section 2.2 (items 1 and 2): the unique colours of an image
// and their pixel counts.
//
// The paper hashes colours into a chained table.  Here the 2^24 possible
// colours index a dense uint32 count table directly, and a 2^24-bit presence
// bitmap records which entries were touched.  Compaction walks the 2 MiB bitmap
// (not the 64 MiB table), so the unique colours come out in ascending key order
// with a prefix sum over word popcounts, and only the touched table entries are
// read and reset.  Both regions are left all-zero for the next call.
#include "cq_internal.h"

namespace cq {

__device__ __forceinline__ void count_key(uint32_t key, uint32_t* __restrict__ tbl,
                                          uint32_t* __restrict__ bitmap)
{
    const uint32_t old = atomicAdd(tbl + key, 1u);
    if (old == 0u) atomicOr(bitmap + (key >> 5), 1u << (key & 31u));
}

// Contiguous image (row stride 3W), base 4-byte aligned: each thread takes 4
// pixels = 12 bytes as three dword loads.
__global__ void __launch_bounds__(256) k_hist_packed(const uint8_t* __restrict__ img, int64_t npix,
                                                     uint32_t* __restrict__ tbl,
                                                     uint32_t* __restrict__ bitmap)
{
    const int64_t ngroups = npix >> 2;
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const uint32_t* w = reinterpret_cast<const uint32_t*>(img);
    for (int64_t g = tid; g < ngroups; g += stride) {
        const uint32_t a = w[3 * g + 0];
        const uint32_t b = w[3 * g + 1];
        const uint32_t c = w[3 * g + 2];
        // little-endian bytes: a = R0 G0 B0 R1, b = G1 B1 R2 G2, c = B2 R3 G3 B3
        const uint32_t k0 = ((a & 0xffu) << 16) | (a & 0xff00u) | ((a >> 16) & 0xffu);
        const uint32_t k1 = ((a >> 24) << 16) | ((b & 0xffu) << 8) | ((b >> 8) & 0xffu);
        const uint32_t k2 = (((b >> 16) & 0xffu) << 16) | ((b >> 24) << 8) | (c & 0xffu);
        const uint32_t k3 = (((c >> 8) & 0xffu) << 16) | (((c >> 16) & 0xffu) << 8) | (c >> 24);
        count_key(k0, tbl, bitmap);
        count_key(k1, tbl, bitmap);
        count_key(k2, tbl, bitmap);
        count_key(k3, tbl, bitmap);
    }
    // the last npix % 4 pixels
    const int64_t rem = npix - (ngroups << 2);
    if (tid < rem) {
        const uint8_t* p = img + 3 * ((ngroups << 2) + tid);
        count_key((uint32_t(p[0]) << 16) | (uint32_t(p[1]) << 8) | uint32_t(p[2]), tbl, bitmap);
    }
}

// General row stride: one pixel per thread iteration.
__global__ void __launch_bounds__(256) k_hist_rows(const uint8_t* __restrict__ img, int32_t H,
                                                   int32_t W, int64_t row_stride,
                                                   uint32_t* __restrict__ tbl,
                                                   uint32_t* __restrict__ bitmap)
{
    const int64_t npix = int64_t(H) * W;
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < npix; p += stride) {
        const int64_t y = p / W, x = p - y * W;
        const uint8_t* q = img + y * row_stride + 3 * x;
        count_key((uint32_t(q[0]) << 16) | (uint32_t(q[1]) << 8) | uint32_t(q[2]), tbl, bitmap);
    }
}

// Pass 1 of the compaction: popcount of each block's bitmap words.
__global__ void __launch_bounds__(kCompactThreads) k_bitmap_count(const uint32_t* __restrict__ bitmap,
                                                                  uint32_t* __restrict__ blk_count)
{
    __shared__ uint32_t tmp[64];
    const uint32_t base = blockIdx.x * kCompactWordsPerBlock + threadIdx.x * kCompactWordsPerThread;
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
        blk_count[blockIdx.x] = s;
    }
}

// Pass 2: exclusive scan of the per-block counts (one block of 256 threads).
__global__ void __launch_bounds__(kCompactBlocks) k_bitmap_scan(const uint32_t* __restrict__ blk_count,
                                                                uint32_t* __restrict__ blk_offset,
                                                                Meta* __restrict__ meta)
{
    __shared__ uint32_t tmp[64];
    uint32_t total = 0;
    const uint32_t off = block_exclusive_scan<uint32_t>(blk_count[threadIdx.x], tmp, &total);
    blk_offset[threadIdx.x] = off;
    if (threadIdx.x == 0) meta->n_unique = int64_t(total);
}

// Pass 3: emit (key, count) in ascending key order, reset the touched table
// entries and bitmap words.  Entries past `capacity` are counted but not
// written.
__global__ void __launch_bounds__(kCompactThreads) k_bitmap_emit(uint32_t* __restrict__ bitmap,
                                                                 uint32_t* __restrict__ tbl,
                                                                 const uint32_t* __restrict__ blk_offset,
                                                                 uint32_t* __restrict__ keys,
                                                                 uint32_t* __restrict__ counts,
                                                                 int64_t capacity)
{
    __shared__ uint32_t tmp[64];
    const uint32_t base = blockIdx.x * kCompactWordsPerBlock + threadIdx.x * kCompactWordsPerThread;
    uint4* p = reinterpret_cast<uint4*>(bitmap + base);
    const uint4 u = p[0], v = p[1];
    const uint32_t words[8] = {u.x, u.y, u.z, u.w, v.x, v.y, v.z, v.w};
    uint32_t c = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) c += __popc(words[j]);
    const uint32_t local = block_exclusive_scan<uint32_t>(c, tmp, nullptr);
    int64_t o = int64_t(blk_offset[blockIdx.x]) + local;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        uint32_t wbits = words[j];
        while (wbits) {
            const uint32_t bit = __ffs(wbits) - 1;
            wbits &= wbits - 1;
            const uint32_t key = (base + j) * 32u + bit;
            const uint32_t cnt = tbl[key];
            tbl[key] = 0u;
            if (o < capacity) {
                keys[o] = key;
                counts[o] = cnt;
            }
            ++o;
        }
    }
    if (c) {
        p[0] = make_uint4(0, 0, 0, 0);
        p[1] = make_uint4(0, 0, 0, 0);
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
    k_fill_zero<<<2048, 256, 0, s>>>(reinterpret_cast<uint4*>(p), n16);
    CQ_LAUNCH_CHECK("k_fill_zero");
    return CQ_OK;
}

int hist_grid(int64_t work_items)
{
    int64_t blocks = (work_items + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    return int(blocks);
}

// Enqueues the histogram and compaction; n_unique is left in meta->n_unique.
cq_status launch_histogram(const uint8_t* img, int32_t H, int32_t W, int64_t row_stride,
                           uint32_t* keys, uint32_t* counts, int64_t capacity, void* ws,
                           const Layout& L, hipStream_t s)
{
    uint32_t* tbl = at<uint32_t>(ws, L.tbl);
    uint32_t* bitmap = at<uint32_t>(ws, L.bitmap);
    uint32_t* blk = at<uint32_t>(ws, L.blk);
    Meta* meta = at<Meta>(ws, L.meta);
    const int64_t npix = int64_t(H) * W;
    const bool packed = row_stride == 3 * int64_t(W) && (reinterpret_cast<uintptr_t>(img) & 3u) == 0;
    if (packed) {
        k_hist_packed<<<hist_grid((npix + 3) / 4), 256, 0, s>>>(img, npix, tbl, bitmap);
        CQ_LAUNCH_CHECK("k_hist_packed");
    } else {
        k_hist_rows<<<hist_grid(npix), 256, 0, s>>>(img, H, W, row_stride, tbl, bitmap);
        CQ_LAUNCH_CHECK("k_hist_rows");
    }
    k_bitmap_count<<<kCompactBlocks, kCompactThreads, 0, s>>>(bitmap, blk);
    CQ_LAUNCH_CHECK("k_bitmap_count");
    k_bitmap_scan<<<1, kCompactBlocks, 0, s>>>(blk, blk + kCompactBlocks, meta);
    CQ_LAUNCH_CHECK("k_bitmap_scan");
    k_bitmap_emit<<<kCompactBlocks, kCompactThreads, 0, s>>>(bitmap, tbl, blk + kCompactBlocks, keys,
                                                             counts, capacity);
    CQ_LAUNCH_CHECK("k_bitmap_emit");
    return CQ_OK;
}

}  // namespace cq
