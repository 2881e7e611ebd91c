// Initialization schemes of Section 2.3 on the N' unique colours: Forgy (FGY),
// farthest-first / max-min (MMX) and k-means++ (KPP, weighted by pixel count).
//
// Every chosen centre is a colour, so D^2 (squared distance to the nearest
// chosen centre) is an exact integer and the sampling weights n_i D_i^2 are
// exact uint64 values.  Each round is two kernels:
//   update : D^2 <- min(D^2, |x - chosen|^2) over all colours, one reduction
//            value per chunk of 1024 colours (sum of n D^2, or the packed
//            arg-max of D^2);
//   select : one block scans the chunk values, draws from the splitmix64
//            stream kept in the control block, locates the chunk and then the
//            colour, and writes the new centre.
// The draw order is the one documented for cq_init in cq.h.
#include "cq_internal.h"

namespace cq {

__device__ __forceinline__ void write_center(double* centers, int j, uint32_t key)
{
    int r, g, b;
    key_rgb(key, r, g, b);
    centers[3 * j + 0] = double(r);
    centers[3 * j + 1] = double(g);
    centers[3 * j + 2] = double(b);
}

// mode 0: KPP first round, chunk value = sum of counts (d2 untouched)
// mode 1: KPP later rounds, chunk value = sum of counts * d2
// mode 2: MMX, chunk value = max over the chunk of (d2 << 32 | ~index)
// first != 0: d2 is set to the distance to the chosen colour (no min).
__global__ void __launch_bounds__(kInitThreads) k_init_update(const uint32_t* __restrict__ keys,
                                                              const uint32_t* __restrict__ counts,
                                                              int64_t n, uint32_t* __restrict__ d2,
                                                              const Meta* __restrict__ meta, int mode,
                                                              int first, uint64_t* __restrict__ chunk_val)
{
    __shared__ uint64_t tmp[kInitThreads / 64];
    int cr = 0, cg = 0, cb = 0;
    if (mode != 0) key_rgb(keys[meta->chosen], cr, cg, cb);
    const int64_t base = int64_t(blockIdx.x) * kInitChunk;
    uint64_t acc = 0;
#pragma unroll
    for (int j = 0; j < kInitItemsPerThread; ++j) {
        const int64_t i = base + j * kInitThreads + threadIdx.x;
        if (i >= n) break;
        if (mode == 0) {
            acc += counts[i];
            continue;
        }
        int r, g, b;
        key_rgb(keys[i], r, g, b);
        const uint32_t d = dist_u32(r, g, b, cr, cg, cb);
        uint32_t m = d;
        if (!first) {
            const uint32_t old = d2[i];
            m = old < d ? old : d;
        }
        d2[i] = m;
        if (mode == 1) {
            acc += uint64_t(counts[i]) * m;
        } else {
            const uint64_t packed = (uint64_t(m) << 32) | uint64_t(0xFFFFFFFFu - uint32_t(i));
            acc = packed > acc ? packed : acc;
        }
    }
    acc = (mode == 2) ? wave_max(acc) : wave_sum(acc);
    if ((threadIdx.x & 63) == 0) tmp[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t v = tmp[0];
        for (int w = 1; w < kInitThreads / 64; ++w) v = (mode == 2) ? (tmp[w] > v ? tmp[w] : v) : v + tmp[w];
        chunk_val[blockIdx.x] = v;
    }
}

// KPP draw for round j: pick the colour whose inclusive prefix of weights
// first exceeds r = U(sum of weights).  weights = counts (j == 0) or
// counts * d2.  One block of kSelectThreads threads.
__global__ void __launch_bounds__(kSelectThreads) k_kpp_select(const uint32_t* __restrict__ keys,
                                                               const uint32_t* __restrict__ counts,
                                                               const uint32_t* __restrict__ d2,
                                                               int64_t n, int64_t nchunks,
                                                               uint64_t* __restrict__ chunk_val,
                                                               Meta* __restrict__ meta, int j,
                                                               double* __restrict__ centers)
{
    __shared__ uint64_t tmp[64];
    __shared__ uint64_t s_r;
    __shared__ int64_t s_chunk;
    __shared__ uint64_t s_before;
    // 1) exclusive prefix of chunk values, in place, segment by segment
    static_assert(kSelectThreads == kInitChunk, "one select thread per colour of a chunk");
    uint64_t carry = 0;
    for (int64_t seg = 0; seg < nchunks; seg += kSelectThreads) {
        const int64_t c = seg + threadIdx.x;
        const uint64_t v = c < nchunks ? chunk_val[c] : 0;
        uint64_t tot = 0;
        const uint64_t ex = block_exclusive_scan<uint64_t>(v, tmp, &tot);
        if (c < nchunks) chunk_val[c] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) {
        uint64_t rng = meta->rng;
        s_r = carry ? uniform_below(rng, carry) : 0;
        meta->rng = rng;
        s_chunk = -1;
    }
    __syncthreads();
    // make the in-place prefixes of this block visible to itself
    __threadfence_block();
    const uint64_t r = s_r;
    // 2) the chunk holding r: excl <= r < incl (zero-weight chunks never match)
    for (int64_t c = threadIdx.x; c < nchunks; c += kSelectThreads) {
        const uint64_t ex = chunk_val[c];
        const uint64_t in = (c + 1 < nchunks) ? chunk_val[c + 1] : carry;
        if (ex <= r && r < in) {
            s_chunk = c;
            s_before = ex;
        }
    }
    __syncthreads();
    int64_t c = s_chunk;
    uint64_t rr = r - s_before;
    if (c < 0) {  // unreachable: the weights sum to carry > 0
        c = 0;
        rr = 0;
    }
    // 3) inside the chunk: first colour whose inclusive prefix exceeds rr
    const int64_t base = c * kInitChunk;
    __shared__ int64_t s_pick;
    if (threadIdx.x == 0) s_pick = -1;
    __syncthreads();
    uint64_t w = 0;
    const int64_t i = base + threadIdx.x;  // kSelectThreads == kInitChunk
    if (i < n) w = (j == 0) ? uint64_t(counts[i]) : uint64_t(counts[i]) * d2[i];
    const uint64_t ex = block_exclusive_scan<uint64_t>(w, tmp, nullptr);
    if (i < n && ex <= rr && rr < ex + w) s_pick = i;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t pick = s_pick;
        if (pick < 0) pick = 0;  // unreachable when the weights are consistent
        meta->chosen = pick;
        write_center(centers, j, keys[pick]);
    }
}

// MMX: round 0 draws the first colour uniformly; later rounds take the
// arg-max of D^2 (lowest index on ties) from the packed chunk values.
__global__ void __launch_bounds__(kSelectThreads) k_mmx_select(const uint32_t* __restrict__ keys,
                                                               int64_t n, int64_t nchunks,
                                                               const uint64_t* __restrict__ chunk_val,
                                                               Meta* __restrict__ meta, int j,
                                                               double* __restrict__ centers)
{
    __shared__ uint64_t tmp[kSelectThreads / 64];
    int64_t pick;
    if (j == 0) {
        if (threadIdx.x != 0) return;
        uint64_t rng = meta->rng;
        pick = int64_t(uniform_below(rng, uint64_t(n)));
        meta->rng = rng;
    } else {
        uint64_t best = 0;
        for (int64_t c = threadIdx.x; c < nchunks; c += kSelectThreads) {
            const uint64_t v = chunk_val[c];
            best = v > best ? v : best;
        }
        best = wave_max(best);
        if ((threadIdx.x & 63) == 0) tmp[threadIdx.x >> 6] = best;
        __syncthreads();
        if (threadIdx.x != 0) return;
        for (int w = 1; w < kSelectThreads / 64; ++w) best = tmp[w] > best ? tmp[w] : best;
        best = tmp[0] > best ? tmp[0] : best;
        pick = int64_t(0xFFFFFFFFu - uint32_t(best & 0xFFFFFFFFull));
        if (pick >= n) pick = 0;  // unreachable: every colour packs a non-zero value
    }
    meta->chosen = pick;
    write_center(centers, j, keys[pick]);
}

// FGY: partial Fisher-Yates over positions [0, N').  Position j swaps with
// r_j = j + U(N' - j); the values held by displaced positions are kept in a
// small map searched by one wave.
__global__ void __launch_bounds__(64) k_forgy(const uint32_t* __restrict__ keys, int64_t n, int K,
                                              Meta* __restrict__ meta, double* __restrict__ centers)
{
    __shared__ int64_t pos[2 * kMaxK];
    __shared__ int64_t val[2 * kMaxK];
    __shared__ int cnt;
    __shared__ int64_t s_r;
    const int lane = threadIdx.x;
    if (lane == 0) cnt = 0;
    __syncthreads();
    uint64_t rng = meta->rng;
    for (int j = 0; j < K; ++j) {
        if (lane == 0) s_r = j + int64_t(uniform_below(rng, uint64_t(n - j)));
        __syncthreads();
        const int64_t r = s_r;
        // value currently at position q (identity unless recorded)
        int64_t vj = j, vr = r;
        int sj = -1, sr = -1;
        for (int b = 0; b < cnt; b += 64) {
            const int e = b + lane;
            const bool hj = e < cnt && pos[e] == j;
            const bool hr = e < cnt && pos[e] == r;
            const uint64_t mj = __ballot(hj), mr = __ballot(hr);
            if (mj) { const int l = __ffsll((unsigned long long)mj) - 1; sj = b + l; }
            if (mr) { const int l = __ffsll((unsigned long long)mr) - 1; sr = b + l; }
        }
        if (sj >= 0) vj = val[sj];
        if (sr >= 0) vr = val[sr];
        __syncthreads();
        if (lane == 0) {
            // position j now holds vr, position r holds vj
            if (sj >= 0) val[sj] = vr; else { pos[cnt] = j; val[cnt] = vr; ++cnt; }
            if (r != j) {
                if (sr >= 0) val[sr] = vj; else { pos[cnt] = r; val[cnt] = vj; ++cnt; }
            }
            write_center(centers, j, keys[vr]);
        }
        __syncthreads();
    }
    if (lane == 0) meta->rng = rng;
}

// N' <= K: the centres are the colours followed by zeros.
__global__ void k_centers_from_colours(const uint32_t* __restrict__ keys, int64_t n, int K,
                                       double* __restrict__ centers)
{
    const int k = threadIdx.x;
    if (k >= K) return;
    if (k < n) {
        write_center(centers, k, keys[k]);
    } else {
        centers[3 * k] = centers[3 * k + 1] = centers[3 * k + 2] = 0.0;
    }
}

__global__ void k_set_rng(Meta* meta, uint64_t seed) { meta->rng = seed; }

// ------------------------------------------------------------------ host
cq_status launch_init(const uint32_t* keys, const uint32_t* counts, int64_t n, int K, int scheme,
                      uint64_t seed, double* centers, void* ws, const Layout& L, hipStream_t s)
{
    Meta* meta = at<Meta>(ws, L.meta);
    if (n <= K) {
        k_centers_from_colours<<<1, kMaxK, 0, s>>>(keys, n, K, centers);
        CQ_LAUNCH_CHECK("k_centers_from_colours");
        return CQ_OK;
    }
    if (scheme == CQ_INIT_USER) return CQ_OK;
    k_set_rng<<<1, 1, 0, s>>>(meta, seed);
    CQ_LAUNCH_CHECK("k_set_rng");
    if (scheme == CQ_INIT_FORGY) {
        k_forgy<<<1, 64, 0, s>>>(keys, n, K, meta, centers);
        CQ_LAUNCH_CHECK("k_forgy");
        return CQ_OK;
    }
    uint64_t* chunk = at<uint64_t>(ws, L.chunks);
    uint32_t* d2 = at<uint32_t>(ws, L.d2);
    const int64_t nchunks = (n + kInitChunk - 1) / kInitChunk;
    const int grid = int(nchunks);
    if (scheme == CQ_INIT_KMEANSPP) {
        k_init_update<<<grid, kInitThreads, 0, s>>>(keys, counts, n, d2, meta, 0, 1, chunk);
        CQ_LAUNCH_CHECK("k_init_update");
        k_kpp_select<<<1, kSelectThreads, 0, s>>>(keys, counts, d2, n, nchunks, chunk, meta, 0, centers);
        CQ_LAUNCH_CHECK("k_kpp_select");
        for (int j = 1; j < K; ++j) {
            k_init_update<<<grid, kInitThreads, 0, s>>>(keys, counts, n, d2, meta, 1, j == 1, chunk);
            CQ_LAUNCH_CHECK("k_init_update");
            k_kpp_select<<<1, kSelectThreads, 0, s>>>(keys, counts, d2, n, nchunks, chunk, meta, j,
                                                      centers);
            CQ_LAUNCH_CHECK("k_kpp_select");
        }
    } else {  // CQ_INIT_MAXMIN
        k_mmx_select<<<1, kSelectThreads, 0, s>>>(keys, n, nchunks, chunk, meta, 0, centers);
        CQ_LAUNCH_CHECK("k_mmx_select");
        for (int j = 1; j < K; ++j) {
            k_init_update<<<grid, kInitThreads, 0, s>>>(keys, counts, n, d2, meta, 2, j == 1, chunk);
            CQ_LAUNCH_CHECK("k_init_update");
            k_mmx_select<<<1, kSelectThreads, 0, s>>>(keys, n, nchunks, chunk, meta, j, centers);
            CQ_LAUNCH_CHECK("k_mmx_select");
        }
    }
    return CQ_OK;
}

}  // namespace cq
