// Weighted Lloyd / Weighted Sort-Means iterations (Algo. 1, Algo. 2) and the
// relative-SSE stopping rule of Section 3.3.
//
// One iteration is three kernels:
//   k_table    (pruned mode, from iteration 2): pairwise centre distances and,
//              for every centre a, the other centres in increasing (distance,
//              index) order, a first (the K x K matrices d and M of Algo. 2);
//   k_assign   nearest centre of every unique colour in FP64 (full search, or
//              the sort-means scan of row m[i] that stops once
//              d[p][t] > 4 d(x, c_p) (1 + 1e-12)), fused with the weighted
//              update: per-block uint64 cluster sums n_k, S_k, Q_k in LDS,
//              flushed with global atomics;
//   k_finalize FP64 means S_k / n_k, SSE from the exact 128-bit identity
//              sum_k (n_k Q_k - |S_k|^2) / n_k, and the stopping test.
// Every kernel returns at once when the control block says the run has
// stopped, so the host can enqueue several iterations ahead of the check.
#include "cq_internal.h"

// Every floating-point operation in this file is rounded on its own.
#pragma clang fp contract(off)

namespace cq {

constexpr int kAssignThreads = 256;

__global__ void __launch_bounds__(kMaxK) k_table(const double* __restrict__ centers, int K,
                                                 double* __restrict__ td, uint8_t* __restrict__ tm,
                                                 const Meta* __restrict__ meta)
{
    if (meta->done) return;
    __shared__ double dv[kMaxK];
    const int a = blockIdx.x;
    const int b = threadIdx.x;
    const double a0 = centers[3 * a], a1 = centers[3 * a + 1], a2 = centers[3 * a + 2];
    double d = 0.0;
    if (b < K) d = dist_f64(a0, a1, a2, centers[3 * b], centers[3 * b + 1], centers[3 * b + 2]);
    dv[b] = d;
    __syncthreads();
    if (b >= K) return;
    int rank = 0;
    if (b != a) {
        rank = 1;
        for (int o = 0; o < K; ++o) {
            if (o == a || o == b) continue;
            const double e = dv[o];
            rank += (e < d || (e == d && o < b)) ? 1 : 0;
        }
    }
    td[a * kRow + rank] = d;
    tm[a * kRow + rank] = uint8_t(b);
}

__global__ void __launch_bounds__(kAssignThreads) k_assign(const uint32_t* __restrict__ keys,
                                                           const uint32_t* __restrict__ counts,
                                                           int64_t n, int K,
                                                           const double* __restrict__ centers,
                                                           const double* __restrict__ td,
                                                           const uint8_t* __restrict__ tm,
                                                           uint8_t* __restrict__ assign, int pruned,
                                                           unsigned long long* __restrict__ sums,
                                                           Meta* __restrict__ meta)
{
    if (meta->done) return;
    __shared__ double c[3 * kMaxK];
    __shared__ unsigned long long bins[5 * kMaxK];  // n, S0, S1, S2, Q per cluster
    __shared__ unsigned long long red[2 * (kAssignThreads / 64)];
    for (int t = threadIdx.x; t < 3 * K; t += blockDim.x) c[t] = centers[t];
    for (int t = threadIdx.x; t < 5 * kMaxK; t += blockDim.x) bins[t] = 0ull;
    __syncthreads();

    unsigned long long ndc = 0, ties = 0;
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
        int r, g, b;
        key_rgb(keys[i], r, g, b);
        const double x0 = double(r), x1 = double(g), x2 = double(b);
        int best;
        double bd;
        double second = 0.0;
        bool have_second = false;
        if (!pruned) {
            best = 0;
            bd = dist_f64(x0, x1, x2, c[0], c[1], c[2]);
            for (int k = 1; k < K; ++k) {
                const double d = dist_f64(x0, x1, x2, c[3 * k], c[3 * k + 1], c[3 * k + 2]);
                if (d < bd) {
                    second = bd;
                    bd = d;
                    best = k;
                } else if (!have_second || d < second) {
                    second = d;
                }
                have_second = true;
            }
            ndc += unsigned(K);
        } else {
            const int p = assign[i];
            const double prev = dist_f64(x0, x1, x2, c[3 * p], c[3 * p + 1], c[3 * p + 2]);
            const double limit = 4.0 * prev * (1.0 + 1e-12);
            best = p;
            bd = prev;
            unsigned evals = 1;
            const double* row_d = td + p * kRow;
            const uint8_t* row_m = tm + p * kRow;
            for (int j = 1; j < K; ++j) {
                if (row_d[j] > limit) break;
                const int t = row_m[j];
                const double d = dist_f64(x0, x1, x2, c[3 * t], c[3 * t + 1], c[3 * t + 2]);
                ++evals;
                if (d < bd || (d == bd && t < best)) {
                    second = bd;
                    bd = d;
                    best = t;
                } else if (!have_second || d < second) {
                    second = d;
                }
                have_second = true;
            }
            ndc += evals;
        }
        if (have_second && (second - bd) <= 1e-5 * second) ++ties;
        assign[i] = uint8_t(best);
        const unsigned long long w = counts[i];
        atomicAdd(&bins[best], w);
        atomicAdd(&bins[kMaxK + 3 * best + 0], w * unsigned(r));
        atomicAdd(&bins[kMaxK + 3 * best + 1], w * unsigned(g));
        atomicAdd(&bins[kMaxK + 3 * best + 2], w * unsigned(b));
        atomicAdd(&bins[4 * kMaxK + best], w * unsigned(r * r + g * g + b * b));
    }
    ndc = wave_sum(ndc);
    ties = wave_sum(ties);
    if ((threadIdx.x & 63) == 0) {
        red[threadIdx.x >> 6] = ndc;
        red[(kAssignThreads / 64) + (threadIdx.x >> 6)] = ties;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long a = 0, t = 0;
        for (int w = 0; w < kAssignThreads / 64; ++w) {
            a += red[w];
            t += red[kAssignThreads / 64 + w];
        }
        atomicAdd(reinterpret_cast<unsigned long long*>(&meta->ndc), a);
        atomicAdd(reinterpret_cast<unsigned long long*>(&meta->near_ties), t);
    }
    // flush the non-empty clusters of this block
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        const unsigned long long nk = bins[k];
        if (nk == 0) continue;
        atomicAdd(&sums[k], nk);
        atomicAdd(&sums[kMaxK + 3 * k + 0], bins[kMaxK + 3 * k + 0]);
        atomicAdd(&sums[kMaxK + 3 * k + 1], bins[kMaxK + 3 * k + 1]);
        atomicAdd(&sums[kMaxK + 3 * k + 2], bins[kMaxK + 3 * k + 2]);
        atomicAdd(&sums[4 * kMaxK + k], bins[4 * kMaxK + k]);
    }
}

__device__ __forceinline__ double u128_to_f64(unsigned __int128 v)
{
    const uint64_t hi = uint64_t(v >> 64);
    const uint64_t lo = uint64_t(v);
    return double(hi) * 18446744073709551616.0 + double(lo);
}

// One block of kMaxK threads.  `it` is the 1-based iteration number.
__global__ void __launch_bounds__(kMaxK) k_finalize(unsigned long long* __restrict__ sums, int K,
                                                    double* __restrict__ centers,
                                                    double* __restrict__ trace, int it, int max_iters,
                                                    double tol, Meta* __restrict__ meta)
{
    if (meta->done) return;
    __shared__ double term[kMaxK];
    __shared__ unsigned long long wsum[kMaxK];
    const int k = threadIdx.x;
    double t = 0.0;
    unsigned long long nk = 0;
    if (k < K) {
        nk = sums[k];
        if (nk != 0) {
            const unsigned long long s0 = sums[kMaxK + 3 * k + 0];
            const unsigned long long s1 = sums[kMaxK + 3 * k + 1];
            const unsigned long long s2 = sums[kMaxK + 3 * k + 2];
            const unsigned long long q = sums[4 * kMaxK + k];
            const double dn = double(nk);
            centers[3 * k + 0] = double(s0) / dn;
            centers[3 * k + 1] = double(s1) / dn;
            centers[3 * k + 2] = double(s2) / dn;
            const unsigned __int128 nq = (unsigned __int128)nk * q;
            const unsigned __int128 ss = (unsigned __int128)s0 * s0 + (unsigned __int128)s1 * s1 +
                                         (unsigned __int128)s2 * s2;
            t = u128_to_f64(nq - ss) / dn;
        }
        // clear the sums for the next iteration
        sums[k] = 0;
        sums[kMaxK + 3 * k + 0] = 0;
        sums[kMaxK + 3 * k + 1] = 0;
        sums[kMaxK + 3 * k + 2] = 0;
        sums[4 * kMaxK + k] = 0;
    }
    term[k] = t;
    wsum[k] = nk;
    __syncthreads();
    if (k != 0) return;
    double sse = 0.0;
    unsigned long long total = 0;
    for (int j = 0; j < K; ++j) {
        sse += term[j];  // ascending cluster order
        total += wsum[j];
    }
    meta->total_w = total;
    trace[it - 1] = sse;
    meta->iters = it;
    meta->sse_last = sse;
    bool stop = false, conv = false;
    if (sse == 0.0) {
        stop = conv = true;
    } else if (it >= 2) {
        const double drop = meta->sse_prev - sse;
        if (drop <= tol * sse) stop = conv = true;
    }
    if (it >= max_iters) stop = true;
    meta->sse_prev = sse;
    if (stop) {
        meta->done = 1;
        meta->converged = conv ? 1 : 0;
    }
}

// Palette: floor(c + 0.5) clamped to [0, 255].
__global__ void k_palette(const double* __restrict__ centers, int K, uint8_t* __restrict__ palette)
{
    const int t = threadIdx.x;
    if (t >= 3 * K) return;
    const double v = centers[t] + 0.5;
    int q;
    if (!(v >= 1.0))
        q = 0;
    else if (v >= 256.0)
        q = 255;
    else
        q = int(v);
    palette[t] = uint8_t(q);
}

// N' <= K: assign[i] = i.
__global__ void k_identity_assign(uint8_t* __restrict__ assign, int64_t n)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) assign[i] = uint8_t(i);
}

// Reset of the per-run fields of the control block and the cluster sums;
// flags a non-finite starting centre.
__global__ void __launch_bounds__(kMaxK) k_kmeans_begin(const double* __restrict__ centers, int K,
                                                        unsigned long long* __restrict__ sums,
                                                        Meta* __restrict__ meta)
{
    const int k = threadIdx.x;
    __shared__ int bad;
    if (k == 0) bad = 0;
    __syncthreads();
    if (k < K) {
        for (int c = 0; c < 3; ++c)
            if (!__builtin_isfinite(centers[3 * k + c])) atomicOr(&bad, 1);
    }
    for (int j = k; j < 5 * kMaxK; j += blockDim.x) sums[j] = 0;
    __syncthreads();
    if (k == 0) {
        meta->ndc = 0;
        meta->near_ties = 0;
        meta->iters = 0;
        meta->converged = 0;
        meta->sse_prev = 0.0;
        meta->sse_last = 0.0;
        meta->bad_input = bad;
        meta->done = bad;  // a bad start runs no iteration
    }
}

// ------------------------------------------------------------------ host
int assign_grid(int64_t n)
{
    int64_t blocks = (n + kAssignThreads - 1) / kAssignThreads;
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    return int(blocks);
}

cq_status launch_kmeans_begin(const double* centers, int K, void* ws, const Layout& L, hipStream_t s)
{
    k_kmeans_begin<<<1, kMaxK, 0, s>>>(centers, K, at<unsigned long long>(ws, L.sums),
                                       at<Meta>(ws, L.meta));
    CQ_LAUNCH_CHECK("k_kmeans_begin");
    return CQ_OK;
}

// Enqueue iterations [it0, it1] (1-based).
cq_status launch_kmeans_iters(const uint32_t* keys, const uint32_t* counts, int64_t n, int K,
                              double* centers, uint8_t* assign, int prune, int it0, int it1,
                              int max_iters, double tol, void* ws, const Layout& L, hipStream_t s)
{
    Meta* meta = at<Meta>(ws, L.meta);
    double* td = at<double>(ws, L.td);
    uint8_t* tm = at<uint8_t>(ws, L.tm);
    unsigned long long* sums = at<unsigned long long>(ws, L.sums);
    double* trace = at<double>(ws, L.trace);
    const int grid = assign_grid(n);
    for (int it = it0; it <= it1; ++it) {
        const int pruned_pass = prune && it >= 2;
        if (pruned_pass) {
            k_table<<<K, kMaxK, 0, s>>>(centers, K, td, tm, meta);
            CQ_LAUNCH_CHECK("k_table");
        }
        k_assign<<<grid, kAssignThreads, 0, s>>>(keys, counts, n, K, centers, td, tm, assign,
                                                  pruned_pass, sums, meta);
        CQ_LAUNCH_CHECK("k_assign");
        k_finalize<<<1, kMaxK, 0, s>>>(sums, K, centers, trace, it, max_iters, tol, meta);
        CQ_LAUNCH_CHECK("k_finalize");
    }
    return CQ_OK;
}

cq_status launch_palette(const double* centers, int K, uint8_t* palette, hipStream_t s)
{
    k_palette<<<1, 3 * kMaxK, 0, s>>>(centers, K, palette);
    CQ_LAUNCH_CHECK("k_palette");
    return CQ_OK;
}

cq_status launch_identity_assign(uint8_t* assign, int64_t n, hipStream_t s)
{
    if (n <= 0) return CQ_OK;
    k_identity_assign<<<int((n + 255) / 256), 256, 0, s>>>(assign, n);
    CQ_LAUNCH_CHECK("k_identity_assign");
    return CQ_OK;
}

}  // namespace cq
