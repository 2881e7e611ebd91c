// Pixel-mapping phase (Section 1) and the MSE of Section 3.1.
//
// The nearest palette entry depends only on the colour, so it is found once
// per unique colour (exact integer distances, lowest index on ties) and stored
// in a 2^24-entry byte table indexed by the colour (channel bits interleaved).  Only the N' entries of
// the image's colours are written; the per-pixel map then reads each pixel,
// looks its key up and writes the index and/or the palette colour.  The squared
// error of every pixel is n_i |x_i - P_lut|^2 summed over the unique colours,
// an exact uint64.
//
// With 2:1 subsampling the unique colours are those of a quarter of the
// pixels, so the table does not cover the others: such a job searches the
// palette for every pixel instead and sums the squared error over the pixels.
#include "cq_internal.h"

namespace cq {

constexpr int kLutThreads = 256;
constexpr int kMapThreads = 256;

// Position of colour (r, g, b) in the byte table: the bits of the three
// channels interleaved (Morton order, b in bits 0, 3, 6, ..., g one above, r
// two above).  Colours close in all three channels then share cache lines of
// the table, so the pixels of an image region, whose colours differ a little
// in every channel, look up few distinct lines and mostly hit the L2.  (In
// key order a line holds 128 values of b at one (r, g): neighbouring pixels
// whose r or g differ land on different lines.)
__device__ __forceinline__ uint32_t spread_bits(uint32_t x)
{
    x = (x | (x << 8)) & 0x0000F00Fu;
    x = (x | (x << 4)) & 0x000C30C3u;
    x = (x | (x << 2)) & 0x00249249u;
    return x;
}

__device__ __forceinline__ uint32_t lut_slot(uint32_t r, uint32_t g, uint32_t b)
{
    return (spread_bits(r) << 2) | (spread_bits(g) << 1) | spread_bits(b);
}

__device__ __forceinline__ uint32_t lut_slot_key(uint32_t key)
{
    return lut_slot(key >> 16, (key >> 8) & 0xffu, key & 0xffu);
}
constexpr int kMapGroupsPerBlock = 1024;  // 4-pixel groups per map block

// Nearest-entry search.  Since |x - p|^2 = |x|^2 - (2 x.p - |p|^2), the
// nearest entry has the largest 2 x.p - |p|^2, an exact integer (x.p is one
// four-byte dot product of the colours packed in key order, R << 16 | G << 8
// | B).  Entry t is stored with (255 - t) - (|p|^2 << 8), so a colour's value
// for it, (x.p << 9) plus that, is ((2 x.p - |p|^2) << 8) | (255 - t): the
// largest value belongs to the nearest entry and, among equal distances, to
// the lowest index.
//
// The palette table in LDS holds (packed entry, stored value) per entry; the
// entries from K up to kMaxK have a value too small ever to be the largest,
// so a search may run to an even count and read two entries at a time.
__device__ __forceinline__ void load_search_palette(const uint8_t* __restrict__ palette, int K, uint2* ent)
{
    for (int t = threadIdx.x; t < kMaxK; t += blockDim.x) {
        const uint8_t* q = palette + 3 * t;
        const int r = t < K ? q[0] : 0, g = t < K ? q[1] : 0, b = t < K ? q[2] : 0;
        const uint32_t packed = (uint32_t(r) << 16) | (uint32_t(g) << 8) | uint32_t(b);
        const int pp = t < K ? r * r + g * g + b * b : 0x3fffff;
        ent[t] = make_uint2(packed, uint32_t((255 - t) - (pp << 8)));
    }
}

// Index of the entry nearest to colour x (key order) among the first K2 (even)
// of `ent`, lowest index on ties; *d receives the squared distance.
__device__ __forceinline__ int nearest_entry(uint32_t x, const uint2* ent, int K2, uint32_t* d)
{
    int best = -0x7fffffff - 1;
#pragma unroll 4
    for (int k = 0; k < K2; k += 2) {
        const uint4 e = *reinterpret_cast<const uint4*>(ent + k);  // entries k and k + 1
        const int v0 = int((__builtin_amdgcn_udot4(x, e.x, 0u, false) << 9) + e.y);
        const int v1 = int((__builtin_amdgcn_udot4(x, e.z, 0u, false) << 9) + e.w);
        best = max(best, max(v0, v1));
    }
    *d = uint32_t(int(__builtin_amdgcn_udot4(x, x, 0u, false)) - (best >> 8));
    return 255 - (best & 255);
}

// Squared distance between two colours packed in key order.
__device__ __forceinline__ uint32_t packed_dist(uint32_t x, uint32_t p)
{
    return __builtin_amdgcn_udot4(x, x, 0u, false) + __builtin_amdgcn_udot4(p, p, 0u, false) -
           2u * __builtin_amdgcn_udot4(x, p, 0u, false);
}

// Rows of the palette's distance table: row p lists every entry q by
// (|P_p - P_q|^2, q) ascending, as one word (|P_p - P_q|^2 << 8) | q (a
// squared distance is below 2^18).  One wave per row, four entries per lane,
// sorted by a bitonic network (partners four or more entries apart are in
// other lanes, in the same register).  Only jobs with lut_rec get blocks.
constexpr int kPalRowsPerBlock = 4;
constexpr int kPalPerLane = kMaxK / 64;
static_assert(kRow % 4 == 0, "palette rows are read four entries at a time");

__global__ void __launch_bounds__(64 * kPalRowsPerBlock) k_pal_rows(const JobDev* __restrict__ jobs,
                                                                   const int* __restrict__ map, int B)
{
    const int jb = find_job(map, B, blockIdx.x);
    const JobDev& J = jobs[jb];
    const int K = J.map_k;
    const int p = (blockIdx.x - map[jb]) * kPalRowsPerBlock + int(threadIdx.x >> 6);
    if (p >= K) return;  // whole waves; no block barrier follows
    const int lane = threadIdx.x & 63;
    const uint8_t* __restrict__ pal = gp(J.palette);
    const int pr = pal[3 * p], pg = pal[3 * p + 1], pb = pal[3 * p + 2];
    uint32_t v[kPalPerLane];
#pragma unroll
    for (int i = 0; i < kPalPerLane; ++i) {
        const int q = kPalPerLane * lane + i;
        if (q < K) {
            const int dr = int(pal[3 * q]) - pr, dg = int(pal[3 * q + 1]) - pg, db = int(pal[3 * q + 2]) - pb;
            v[i] = (uint32_t(dr * dr + dg * dg + db * db) << 8) | uint32_t(q);
        } else {
            v[i] = 0xffffffffu;
        }
    }
    for (int size = 2; size <= kMaxK; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            if (stride >= kPalPerLane) {
#pragma unroll
                for (int i = 0; i < kPalPerLane; ++i) {
                    const uint32_t o = __shfl_xor(v[i], stride / kPalPerLane, 64);
                    const int e = kPalPerLane * lane + i;
                    const bool ascending = (e & size) == 0;
                    const bool lower = (e & stride) == 0;
                    v[i] = (lower == ascending) ? (o < v[i] ? o : v[i]) : (o > v[i] ? o : v[i]);
                }
            } else {
#pragma unroll
                for (int i = 0; i < kPalPerLane; ++i) {
                    if (i & stride) continue;
                    const int j = i | stride;
                    const bool ascending = ((kPalPerLane * lane + i) & size) == 0;
                    const uint32_t lo = v[i] < v[j] ? v[i] : v[j], hi = v[i] < v[j] ? v[j] : v[i];
                    v[i] = ascending ? lo : hi;
                    v[j] = ascending ? hi : lo;
                }
            }
        }
    }
    uint32_t* __restrict__ row = gp(J.prow) + int64_t(p) * kRow;
#pragma unroll
    for (int i = 0; i < kPalPerLane; ++i)
        if (kPalPerLane * lane + i < K) row[kPalPerLane * lane + i] = v[i];
}

// Nearest rounded palette entry of every unique colour (exact integer
// distances, lowest index on ties) into the job's byte table; adds
// n_i |x_i - P|^2 to the job's squared-error sum.  Block b of job j takes the
// colours [b chunk, (b + 1) chunk).
//
// A job with lut_rec reads its colours from the final records of its pruned
// run, each with the cluster c it was last assigned to, and scans row c of
// the palette's distance table: an entry q with |P_c - P_q| > 2 |x - P_c|
// is farther from x than P_c (|x - P_q| >= |P_c - P_q| - |x - P_c|), so the
// scan stops at the first entry with |P_c - P_q|^2 > 4 |x - P_c|^2, having
// seen every entry at least as near as P_c: the same nearest entry, and the
// same lowest index among equals, as a search of all entries.  Any other job
// searches all entries.
__global__ void __launch_bounds__(kLutThreads) k_lut(const JobDev* __restrict__ jobs,
                                                     const int* __restrict__ map, int B, int with_err)
{
    __shared__ __align__(16) uint2 ent[kMaxK];
    __shared__ unsigned long long red[kLutThreads / 64];
    const int jb = find_job(map, B, blockIdx.x);
    const JobDev& J = jobs[jb];
    const int lb = blockIdx.x - map[jb];
    const int K2 = (J.map_k + 1) & ~1;
    const uint32_t* __restrict__ keys = gp(J.keys);
    const uint32_t* __restrict__ counts = gp(J.counts);
    uint8_t* __restrict__ lut = gp(J.lut);
    load_search_palette(gp(J.palette), J.map_k, ent);
    __syncthreads();
    const int64_t lo = int64_t(lb) * J.chunk;
    const int64_t hi = lo + J.chunk < J.n ? lo + J.chunk : J.n;
    unsigned long long err = 0;
    const int iters = gp(J.meta)->iters;
    if (J.lut_rec && iters >= 1) {
        const uint64_t* __restrict__ g = gp(J.grp) + record_buffer(iters, J.regroup_period) * J.n;
        const uint32_t* __restrict__ rows = gp(J.prow);
        for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
            const uint64_t rec = g[i];
            const uint32_t key = uint32_t(rec) & 0xffffffu;
            const int c = int(uint32_t(rec) >> 24);
            const uint32_t w = uint32_t(rec >> 32) & 0x0fffffffu;
            uint32_t bd = packed_dist(key, ent[c].x);
            int bq = c;
            const uint32_t lim = 4u * bd;
            const uint32_t* __restrict__ row = rows + int64_t(c) * kRow;
            // four entries per load round trip (a row has kRow entries, a
            // multiple of four; those past K are never compared)
            const int K = J.map_k;
            bool more = true;
            for (int e0 = 0; more && e0 < K; e0 += 4) {
                const uint4 v4 = *reinterpret_cast<const uint4*>(row + e0);
                const uint32_t vs[4] = {v4.x, v4.y, v4.z, v4.w};
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const uint32_t v = vs[u];
                    if (!more || e0 + u >= K || (v >> 8) > lim) {
                        more = false;
                        continue;
                    }
                    const int q = int(v & 255u);
                    const uint32_t d = packed_dist(key, ent[q].x);
                    if (d < bd || (d == bd && q < bq)) {
                        bd = d;
                        bq = q;
                    }
                }
            }
            lut[lut_slot_key(key)] = uint8_t(bq);
            if (with_err) err += (unsigned long long)w * bd;
        }
    } else {
        for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
            const uint32_t key = keys[i];
            uint32_t d;
            lut[lut_slot_key(key)] = uint8_t(nearest_entry(key, ent, K2, &d));
            if (with_err) err += (unsigned long long)counts[i] * d;
        }
    }
    if (!with_err) return;
    err = wave_sum(err);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = err;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long s = 0;
        for (int w = 0; w < kLutThreads / 64; ++w) s += red[w];
        atomicAdd(reinterpret_cast<unsigned long long*>(&gp(J.meta)->sq_err), s);
    }
}

// Pixel map: index and/or palette colour of every pixel through the table.
// Block b of job j takes kMapGroupsPerBlock groups of 4 pixels.  Packed jobs
// (contiguous rows, 4-byte aligned image and outputs) read 12 bytes and write
// one dword of indices and three of colours per group, a thread issuing the
// loads of all its groups before any table lookup; other jobs go pixel by
// pixel.  The palette sits in LDS as one dword per entry (R | G << 8 | B << 16)
// with all 256 entries (zero past K), so any table byte indexes in bounds.
constexpr int kMapGroupsPerThread = kMapGroupsPerBlock / kMapThreads;

// The blocks of a launch go to the 8 XCDs in turn (block i to XCD i mod 8);
// this gives XCD x the consecutive logical blocks [start_x, start_x + count_x),
// so that each XCD's L2 serves one contiguous part of the data.
__device__ __forceinline__ int xcd_block(int i, int n)
{
    const int x = i & 7, q = n >> 3, r = n & 7;
    const int start = x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q;
    return start + (i >> 3);
}

// Per-pixel search of a job with map_direct: block b takes the pixels
// [4 b G, 4 (b + 1) G) (G = kMapGroupsPerBlock), one per thread per step.
// Adds the pixels' squared errors to the job's sum if with_err.
__device__ __forceinline__ void map_direct_pixels(const JobDev& J, int64_t g0, int64_t g1, const uint32_t* pal,
                                                  const uint2* ent, int with_err)
{
    const int K2 = (J.map_k + 1) & ~1;
    const uint8_t* __restrict__ img = gp(J.img);
    uint8_t* __restrict__ out_idx = gp(J.out_idx);
    uint8_t* __restrict__ out_rgb = gp(J.out_rgb);
    const int64_t npix = int64_t(J.H) * J.W;
    const int64_t p0 = g0 * 4, p1 = g1 * 4 < npix ? g1 * 4 : npix;
    const int32_t W = J.W;
    unsigned long long err = 0;
    for (int64_t p = p0 + threadIdx.x; p < p1; p += kMapThreads) {
        const uint32_t y = uint32_t(p) / uint32_t(W), x = uint32_t(p) - y * uint32_t(W);  // p < 2^28
        const uint8_t* q = img + int64_t(y) * J.stride + 3 * x;
        const uint32_t key = (uint32_t(q[0]) << 16) | (uint32_t(q[1]) << 8) | uint32_t(q[2]);
        uint32_t d;
        const int best = nearest_entry(key, ent, K2, &d);
        if (with_err) err += d;
        if (out_idx) out_idx[p] = uint8_t(best);
        if (out_rgb) {
            out_rgb[3 * p + 0] = uint8_t(pal[best]);
            out_rgb[3 * p + 1] = uint8_t(pal[best] >> 8);
            out_rgb[3 * p + 2] = uint8_t(pal[best] >> 16);
        }
    }
    if (!with_err) return;
    __shared__ unsigned long long red[kMapThreads / 64];
    err = wave_sum(err);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = err;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < kMapThreads / 64; ++w) t += red[w];
        atomicAdd(reinterpret_cast<unsigned long long*>(&gp(J.meta)->sq_err), t);
    }
}

__global__ void __launch_bounds__(kMapThreads) k_map(const JobDev* __restrict__ jobs,
                                                     const int* __restrict__ map, int B, int with_err)
{
    __shared__ uint32_t pal[kMaxK];
    __shared__ __align__(16) uint2 ent[kMaxK];  // read two entries at a time
    const int blk = xcd_block(int(blockIdx.x), int(gridDim.x));
    const int jb = find_job(map, B, blk);
    const JobDev& J = jobs[jb];
    const int lb = blk - map[jb];
    const int K = J.map_k;
    for (int t = threadIdx.x; t < kMaxK; t += blockDim.x) {
        const uint8_t* q = gp(J.palette) + 3 * t;
        pal[t] = t < K ? (uint32_t(q[0]) | (uint32_t(q[1]) << 8) | (uint32_t(q[2]) << 16)) : 0u;
    }
    const int64_t g0 = int64_t(lb) * kMapGroupsPerBlock;
    const int64_t g1 = g0 + kMapGroupsPerBlock;
    if (J.map_direct) {  // uniform over the block
        load_search_palette(gp(J.palette), K, ent);
        __syncthreads();
        map_direct_pixels(J, g0, g1, pal, ent, with_err);
        return;
    }
    __syncthreads();
    const uint8_t* __restrict__ img = gp(J.img);
    const uint8_t* __restrict__ lut = gp(J.lut);
    uint8_t* __restrict__ out_idx = gp(J.out_idx);
    uint8_t* __restrict__ out_rgb = gp(J.out_rgb);
    const int64_t npix = int64_t(J.H) * J.W;
    if (J.packed) {
        const int64_t ngroups = npix >> 2;
        const uint32_t* w = reinterpret_cast<const uint32_t*>(img);
        uint32_t a[kMapGroupsPerThread], b[kMapGroupsPerThread], c[kMapGroupsPerThread];
#pragma unroll
        for (int s = 0; s < kMapGroupsPerThread; ++s) {
            const int64_t g = g0 + s * kMapThreads + threadIdx.x;
            const bool in = g < ngroups;
            a[s] = in ? w[3 * g + 0] : 0u;
            b[s] = in ? w[3 * g + 1] : 0u;
            c[s] = in ? w[3 * g + 2] : 0u;
        }
        uint32_t ix[kMapGroupsPerThread][4];
#pragma unroll
        for (int s = 0; s < kMapGroupsPerThread; ++s) {
            // a = R0 G0 B0 R1, b = G1 B1 R2 G2, c = B2 R3 G3 B3 (bytes, low first)
            ix[s][0] = lut[lut_slot(a[s] & 0xffu, (a[s] >> 8) & 0xffu, (a[s] >> 16) & 0xffu)];
            ix[s][1] = lut[lut_slot(a[s] >> 24, b[s] & 0xffu, (b[s] >> 8) & 0xffu)];
            ix[s][2] = lut[lut_slot((b[s] >> 16) & 0xffu, b[s] >> 24, c[s] & 0xffu)];
            ix[s][3] = lut[lut_slot((c[s] >> 8) & 0xffu, (c[s] >> 16) & 0xffu, c[s] >> 24)];
        }
#pragma unroll
        for (int s = 0; s < kMapGroupsPerThread; ++s) {
            const int64_t g = g0 + s * kMapThreads + threadIdx.x;
            if (g >= ngroups) continue;
            const uint32_t i0 = ix[s][0], i1 = ix[s][1], i2 = ix[s][2], i3 = ix[s][3];
            if (out_idx)
                reinterpret_cast<uint32_t*>(out_idx)[g] = i0 | (i1 << 8) | (i2 << 16) | (i3 << 24);
            if (out_rgb) {
                const uint32_t q0 = pal[i0], q1 = pal[i1], q2 = pal[i2], q3 = pal[i3];
                uint32_t* o = reinterpret_cast<uint32_t*>(out_rgb) + 3 * g;
                o[0] = q0 | (q1 << 24);
                o[1] = (q1 >> 8) | (q2 << 16);
                o[2] = (q2 >> 16) | (q3 << 8);
            }
        }
        // the last npix % 4 pixels belong to the block holding group ngroups
        const int64_t rem = npix - (ngroups << 2);
        if (rem > 0 && ngroups >= g0 && ngroups < g1 && threadIdx.x < rem) {
            const int64_t px = (ngroups << 2) + threadIdx.x;
            const uint8_t* p = img + 3 * px;
            const uint32_t idx = lut[lut_slot(p[0], p[1], p[2])];
            if (out_idx) out_idx[px] = uint8_t(idx);
            if (out_rgb) {
                out_rgb[3 * px + 0] = uint8_t(pal[idx]);
                out_rgb[3 * px + 1] = uint8_t(pal[idx] >> 8);
                out_rgb[3 * px + 2] = uint8_t(pal[idx] >> 16);
            }
        }
    } else {
        const int32_t W = J.W;
        const int64_t p0 = g0 * 4, p1 = g1 * 4 < npix ? g1 * 4 : npix;
        for (int64_t p = p0 + threadIdx.x; p < p1; p += kMapThreads) {
            const uint32_t y = uint32_t(p) / uint32_t(W), x = uint32_t(p) - y * uint32_t(W);  // p < 2^28
            const uint8_t* q = img + int64_t(y) * J.stride + 3 * x;
            const uint32_t idx = lut[lut_slot(q[0], q[1], q[2])];
            if (out_idx) out_idx[p] = uint8_t(idx);
            if (out_rgb) {
                out_rgb[3 * p + 0] = uint8_t(pal[idx]);
                out_rgb[3 * p + 1] = uint8_t(pal[idx] >> 8);
                out_rgb[3 * p + 2] = uint8_t(pal[idx] >> 16);
            }
        }
    }
}

// ------------------------------------------------------------------ host
// Map blocks for an image of npix pixels (one group of four pixels per lane step).
int map_blocks(int64_t npix)
{
    const int64_t groups = (npix + 3) / 4;
    const int64_t b = (groups + kMapGroupsPerBlock - 1) / kMapGroupsPerBlock;
    return int(b < 1 ? 1 : b);
}

cq_status launch_lut(const JobDev* jobs, const int* maps, int B, int total, int with_err, hipStream_t s)
{
    CQ_TIMED_LAUNCH("k_lut", s, k_lut<<<total, kLutThreads, 0, s>>>(jobs, maps + kMapLut * (B + 1), B, with_err));
    return CQ_OK;
}

cq_status launch_pal_rows(const JobDev* jobs, const int* maps, int B, int total, hipStream_t s)
{
    CQ_TIMED_LAUNCH("k_pal_rows", s, k_pal_rows<<<total, 64 * kPalRowsPerBlock, 0, s>>>(jobs, maps + kMapPalRows * (B + 1), B));
    return CQ_OK;
}

int pal_rows_blocks(int K) { return (K + kPalRowsPerBlock - 1) / kPalRowsPerBlock; }

cq_status launch_map(const JobDev* jobs, const int* maps, int B, int total, int with_err, hipStream_t s)
{
    CQ_TIMED_LAUNCH("k_map", s, k_map<<<total, kMapThreads, 0, s>>>(jobs, maps + kMapPix * (B + 1), B, with_err));
    return CQ_OK;
}

}  // namespace cq
