// Pixel-mapping phase (Section 1) and the MSE of Section 3.1.
//
// The nearest palette entry depends only on the colour, so it is found once
// per unique colour (exact integer distances, lowest index on ties) and stored
// in a 2^24-entry byte table indexed by the colour key.  Only the N' entries of
// the image's colours are written; the per-pixel map then reads each pixel,
// looks its key up and writes the index and/or the palette colour.  The squared
// error of every pixel is n_i |x_i - P_lut|^2 summed over the unique colours,
// an exact uint64.
#include "cq_internal.h"

namespace cq {

constexpr int kLutThreads = 256;

__global__ void __launch_bounds__(kLutThreads) k_lut(const uint32_t* __restrict__ keys,
                                                     const uint32_t* __restrict__ counts, int64_t n,
                                                     const uint8_t* __restrict__ palette, int K,
                                                     uint8_t* __restrict__ lut, Meta* __restrict__ meta)
{
    __shared__ int pal[3 * kMaxK];
    __shared__ unsigned long long red[kLutThreads / 64];
    for (int t = threadIdx.x; t < 3 * K; t += blockDim.x) pal[t] = palette[t];
    __syncthreads();
    unsigned long long err = 0;
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint32_t key = keys[i];
        int r, g, b;
        key_rgb(key, r, g, b);
        uint32_t bd = dist_u32(r, g, b, pal[0], pal[1], pal[2]);
        int best = 0;
        for (int k = 1; k < K; ++k) {
            const uint32_t d = dist_u32(r, g, b, pal[3 * k], pal[3 * k + 1], pal[3 * k + 2]);
            if (d < bd) {
                bd = d;
                best = k;
            }
        }
        lut[key] = uint8_t(best);
        if (counts) err += (unsigned long long)counts[i] * bd;
    }
    if (!counts) return;
    err = wave_sum(err);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = err;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long s = 0;
        for (int w = 0; w < kLutThreads / 64; ++w) s += red[w];
        atomicAdd(reinterpret_cast<unsigned long long*>(&meta->sq_err), s);
    }
}

// Contiguous image, 4-byte aligned image and outputs: 4 pixels per thread.
__global__ void __launch_bounds__(256) k_map_packed(const uint8_t* __restrict__ img, int64_t npix,
                                                    const uint8_t* __restrict__ lut,
                                                    const uint8_t* __restrict__ palette, int K,
                                                    uint8_t* __restrict__ out_idx,
                                                    uint8_t* __restrict__ out_rgb)
{
    // all 256 entries, zero past K, so that any table byte indexes in bounds
    __shared__ uint8_t pal[3 * kMaxK];
    for (int t = threadIdx.x; t < 3 * kMaxK; t += blockDim.x) pal[t] = t < 3 * K ? palette[t] : 0;
    __syncthreads();
    const int64_t ngroups = npix >> 2;
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const uint32_t* w = reinterpret_cast<const uint32_t*>(img);
    for (int64_t g = tid; g < ngroups; g += stride) {
        const uint32_t a = w[3 * g + 0];
        const uint32_t b = w[3 * g + 1];
        const uint32_t c = w[3 * g + 2];
        const uint32_t k0 = ((a & 0xffu) << 16) | (a & 0xff00u) | ((a >> 16) & 0xffu);
        const uint32_t k1 = ((a >> 24) << 16) | ((b & 0xffu) << 8) | ((b >> 8) & 0xffu);
        const uint32_t k2 = (((b >> 16) & 0xffu) << 16) | ((b >> 24) << 8) | (c & 0xffu);
        const uint32_t k3 = (((c >> 8) & 0xffu) << 16) | (((c >> 16) & 0xffu) << 8) | (c >> 24);
        const uint32_t i0 = lut[k0], i1 = lut[k1], i2 = lut[k2], i3 = lut[k3];
        if (out_idx)
            reinterpret_cast<uint32_t*>(out_idx)[g] = i0 | (i1 << 8) | (i2 << 16) | (i3 << 24);
        if (out_rgb) {
            const uint8_t* p0 = pal + 3 * i0;
            const uint8_t* p1 = pal + 3 * i1;
            const uint8_t* p2 = pal + 3 * i2;
            const uint8_t* p3 = pal + 3 * i3;
            uint32_t* o = reinterpret_cast<uint32_t*>(out_rgb) + 3 * g;
            o[0] = uint32_t(p0[0]) | (uint32_t(p0[1]) << 8) | (uint32_t(p0[2]) << 16) | (uint32_t(p1[0]) << 24);
            o[1] = uint32_t(p1[1]) | (uint32_t(p1[2]) << 8) | (uint32_t(p2[0]) << 16) | (uint32_t(p2[1]) << 24);
            o[2] = uint32_t(p2[2]) | (uint32_t(p3[0]) << 8) | (uint32_t(p3[1]) << 16) | (uint32_t(p3[2]) << 24);
        }
    }
    const int64_t rem = npix - (ngroups << 2);
    if (tid < rem) {
        const int64_t px = (ngroups << 2) + tid;
        const uint8_t* p = img + 3 * px;
        const uint32_t idx = lut[(uint32_t(p[0]) << 16) | (uint32_t(p[1]) << 8) | uint32_t(p[2])];
        if (out_idx) out_idx[px] = uint8_t(idx);
        if (out_rgb) {
            out_rgb[3 * px + 0] = pal[3 * idx + 0];
            out_rgb[3 * px + 1] = pal[3 * idx + 1];
            out_rgb[3 * px + 2] = pal[3 * idx + 2];
        }
    }
}

// General row stride or alignment: one pixel per thread iteration.  Outputs
// are dense (W bytes and 3 W bytes per row).
__global__ void __launch_bounds__(256) k_map_rows(const uint8_t* __restrict__ img, int32_t H, int32_t W,
                                                  int64_t row_stride, const uint8_t* __restrict__ lut,
                                                  const uint8_t* __restrict__ palette, int K,
                                                  uint8_t* __restrict__ out_idx,
                                                  uint8_t* __restrict__ out_rgb)
{
    __shared__ uint8_t pal[3 * kMaxK];
    for (int t = threadIdx.x; t < 3 * kMaxK; t += blockDim.x) pal[t] = t < 3 * K ? palette[t] : 0;
    __syncthreads();
    const int64_t npix = int64_t(H) * W;
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < npix; p += stride) {
        const int64_t y = p / W, x = p - y * W;
        const uint8_t* q = img + y * row_stride + 3 * x;
        const uint32_t idx = lut[(uint32_t(q[0]) << 16) | (uint32_t(q[1]) << 8) | uint32_t(q[2])];
        if (out_idx) out_idx[p] = uint8_t(idx);
        if (out_rgb) {
            out_rgb[3 * p + 0] = pal[3 * idx + 0];
            out_rgb[3 * p + 1] = pal[3 * idx + 1];
            out_rgb[3 * p + 2] = pal[3 * idx + 2];
        }
    }
}

__global__ void k_zero_sq_err(Meta* meta) { meta->sq_err = 0; }

// ------------------------------------------------------------------ host
int map_grid(int64_t items)
{
    int64_t blocks = (items + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    return int(blocks);
}

cq_status launch_lut(const uint32_t* keys, const uint32_t* counts, int64_t n, const uint8_t* palette,
                     int K, void* ws, const Layout& L, hipStream_t s)
{
    Meta* meta = at<Meta>(ws, L.meta);
    if (counts) {
        k_zero_sq_err<<<1, 1, 0, s>>>(meta);
        CQ_LAUNCH_CHECK("k_zero_sq_err");
    }
    int64_t blocks = (n + kLutThreads - 1) / kLutThreads;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    k_lut<<<int(blocks), kLutThreads, 0, s>>>(keys, counts, n, palette, K, at<uint8_t>(ws, L.lut), meta);
    CQ_LAUNCH_CHECK("k_lut");
    return CQ_OK;
}

cq_status launch_map(const uint8_t* img, int32_t H, int32_t W, int64_t row_stride,
                     const uint8_t* palette, int K, uint8_t* out_idx, uint8_t* out_rgb, void* ws,
                     const Layout& L, hipStream_t s)
{
    if (!out_idx && !out_rgb) return CQ_OK;
    const uint8_t* lut = at<uint8_t>(ws, L.lut);
    const int64_t npix = int64_t(H) * W;
    const bool aligned = (reinterpret_cast<uintptr_t>(img) & 3u) == 0 &&
                         (reinterpret_cast<uintptr_t>(out_idx) & 3u) == 0 &&
                         (reinterpret_cast<uintptr_t>(out_rgb) & 3u) == 0;
    if (row_stride == 3 * int64_t(W) && aligned) {
        k_map_packed<<<map_grid((npix + 3) / 4), 256, 0, s>>>(img, npix, lut, palette, K, out_idx, out_rgb);
        CQ_LAUNCH_CHECK("k_map_packed");
    } else {
        k_map_rows<<<map_grid(npix), 256, 0, s>>>(img, H, W, row_stride, lut, palette, K, out_idx, out_rgb);
        CQ_LAUNCH_CHECK("k_map_rows");
    }
    return CQ_OK;
}

}  // namespace cq
