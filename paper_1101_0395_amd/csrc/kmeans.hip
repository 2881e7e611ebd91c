// Weighted Lloyd / Weighted Sort-Means iterations (Algo. 1, Algo. 2) and the
// relative-SSE stopping rule of Section 3.3, for a batch of jobs.
//
// One iteration is two launches over all jobs:
//   k_assign   nearest centre of every unique colour in FP64: a full search
//              (Algo. 1, and the first iteration of Algo. 2) or the sort-means
//              scan of row m[i] of the sorted table, which stops once
//              d[p][t] > 4 d(x, c_p) (1 + 1e-12); fused with the weighted
//              update, i.e. per-block uint64 cluster sums n_k, S_k, Q_k in LDS
//              flushed with global atomics;
//   k_update   FP64 means S_k / n_k, SSE from the exact 128-bit identity
//              sum_k (n_k Q_k - |S_k|^2) / n_k, the stopping test and, in
//              pruned runs, the pairwise centre distances with every row
//              sorted by (distance, index), own centre first (the K x K
//              matrices d and M of Algo. 2) for the next iteration.
// The iteration number lives in each job's control block, so the same two
// launches serve every iteration and a stopped job's blocks return at once.
#include "cq_internal.h"

// Every floating-point operation in this file is rounded on its own.
#pragma clang fp contract(off)

namespace cq {

constexpr int kAssignThreads = 256;
constexpr int kRowCache = 32;   // leading entries of a sorted row staged in LDS
constexpr int kRowSlots = 64;   // rows staged per block
constexpr int kFetch = 16;      // row entries per global round trip past the staged prefix

// Adds (n, S_r, S_g, S_b, Q) of the valid lanes to the LDS bins of their
// clusters.  Lanes of one wave that share a cluster are summed first (up to
// four distinct clusters per wave); the rest add their own values.
__device__ __forceinline__ void bin_add(unsigned long long* bins, bool valid, int best,
                                        unsigned long long w, int r, int g, int b)
{
    const unsigned long long v1 = w * unsigned(r), v2 = w * unsigned(g), v3 = w * unsigned(b);
    const unsigned long long v4 = w * unsigned(r * r + g * g + b * b);
    const int lane = threadIdx.x & 63;
    unsigned long long active = __ballot(valid);
#pragma unroll 1
    for (int round = 0; round < 4 && active; ++round) {
        const int leader = __ffsll(active) - 1;
        const int kb = __shfl(best, leader, 64);
        const bool mine = valid && best == kb;
        const unsigned long long mask = __ballot(mine);
        const unsigned long long s0 = wave_sum(mine ? w : 0ull);
        const unsigned long long s1 = wave_sum(mine ? v1 : 0ull);
        const unsigned long long s2 = wave_sum(mine ? v2 : 0ull);
        const unsigned long long s3 = wave_sum(mine ? v3 : 0ull);
        const unsigned long long s4 = wave_sum(mine ? v4 : 0ull);
        if (lane == leader) {
            atomicAdd(&bins[kb], s0);
            atomicAdd(&bins[kMaxK + 3 * kb + 0], s1);
            atomicAdd(&bins[kMaxK + 3 * kb + 1], s2);
            atomicAdd(&bins[kMaxK + 3 * kb + 2], s3);
            atomicAdd(&bins[4 * kMaxK + kb], s4);
        }
        if (mine) valid = false;
        active &= ~mask;
    }
    if (valid) {
        atomicAdd(&bins[best], w);
        atomicAdd(&bins[kMaxK + 3 * best + 0], v1);
        atomicAdd(&bins[kMaxK + 3 * best + 1], v2);
        atomicAdd(&bins[kMaxK + 3 * best + 2], v3);
        atomicAdd(&bins[4 * kMaxK + best], v4);
    }
}

// Candidate-set summary of one colour: smallest distance, its centre (lowest
// index on ties) and the second smallest distance of the multiset (+inf when
// only one distance was evaluated).
struct Best {
    double bd;
    double second;
    int best;
};

__device__ __forceinline__ void best_push(Best& v, double d, int t)
{
    if (d < v.bd || (d == v.bd && t < v.best)) {
        v.second = v.bd;
        v.bd = d;
        v.best = t;
    } else if (d < v.second) {
        v.second = d;
    }
}

// Block reduction of the distance and near-tie counters, then one atomic each.
__device__ __forceinline__ void flush_counters(unsigned long long ndc, unsigned long long ties,
                                               unsigned long long* red, Meta* meta)
{
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
}

__device__ __forceinline__ void flush_bins(const unsigned long long* bins, int K,
                                           unsigned long long* __restrict__ sums)
{
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

__device__ __forceinline__ bool near_tie(const Best& v)
{
    return v.second != __builtin_inf() && (v.second - v.bd) <= 1e-5 * v.second;
}

// Full search over the centres for one colour per lane.  All lanes walk the
// same centre index, so the centres come through scalar loads.
__device__ __forceinline__ Best full_search(double x0, double x1, double x2,
                                            const double* __restrict__ centers, int K)
{
    Best v{dist_f64(x0, x1, x2, centers[0], centers[1], centers[2]), __builtin_inf(), 0};
#pragma unroll 4
    for (int k = 1; k < K; ++k) {
        const double d = dist_f64(x0, x1, x2, centers[3 * k], centers[3 * k + 1], centers[3 * k + 2]);
        if (d < v.bd) {
            v.second = v.bd;
            v.bd = d;
            v.best = k;
        } else if (d < v.second) {
            v.second = d;
        }
    }
    return v;
}

// Assignment fused with the cluster sums.  Block b of job j takes the colours
// [b chunk, (b + 1) chunk) (keys ascending, so a run is compact in colour space
// and touches few clusters), one colour per lane.  In a sort-means pass the
// block first gathers the previous centres p of its colours and stages the
// first kRowCache entries of each of those rows (at most kRowSlots rows) in
// LDS; scans read global memory only past that prefix or for rows beyond the
// staged ones.
__global__ void __launch_bounds__(kAssignThreads) k_assign(const JobDev* __restrict__ jobs,
                                                           const int* __restrict__ map, int B)
{
    __shared__ double c[3 * kMaxK];
    __shared__ unsigned long long bins[5 * kMaxK];  // n, S0, S1, S2, Q per cluster
    __shared__ unsigned long long red[2 * (kAssignThreads / 64)];
    __shared__ double ltd[kRowSlots * kRowCache];
    __shared__ uint8_t ltm[kRowSlots * kRowCache];
    __shared__ int slot_of[kMaxK];
    __shared__ int row_of[kRowSlots];
    __shared__ int need[kMaxK];
    __shared__ int scan_tmp[64];
    static_assert(kAssignThreads == kMaxK, "one thread per table row");
    const int jb = find_job(map, B, blockIdx.x);
    const JobDev& J = jobs[jb];
    const int lb = blockIdx.x - map[jb];
    Meta* __restrict__ meta = gp(J.meta);
    const int K = J.K;
    const int64_t n = J.n;
    const double* __restrict__ centers = gp(J.centers);
    const uint32_t* __restrict__ keys = gp(J.keys);
    const uint32_t* __restrict__ counts = gp(J.counts);
    uint8_t* __restrict__ assign = gp(J.assign);
    const int64_t lo = int64_t(lb) * J.chunk;
    const int64_t hi = lo + J.chunk < n ? lo + J.chunk : n;
    // every load this block needs first is issued before anything waits on it:
    // the control block, the centres, and the colours of the first pass
    const int done = meta->done;
    const int it = meta->iters + 1;
    double cv[3];
#pragma unroll
    for (int u = 0; u < 3; ++u) {
        const int t = u * kAssignThreads + threadIdx.x;
        cv[u] = t < 3 * K ? centers[t] : 0.0;
    }
    const int64_t i0 = lo + threadIdx.x;
    const bool valid0 = i0 < hi;
    const uint32_t key0 = valid0 ? keys[i0] : 0u;
    const uint32_t cnt0 = valid0 ? counts[i0] : 0u;
    const int p0 = valid0 ? assign[i0] : 0;
    if (done) return;
    const bool pruned = J.prune && it >= 2;
    if (lb == 0 && threadIdx.x == 0) meta->cur_it = it;
    unsigned long long* __restrict__ sums = gp(J.sums) + (it & 1) * 5 * kMaxK;
#pragma unroll
    for (int u = 0; u < 3; ++u) {
        const int t = u * kAssignThreads + threadIdx.x;
        if (t < 3 * K) c[t] = cv[u];
    }
    for (int t = threadIdx.x; t < 5 * kMaxK; t += blockDim.x) bins[t] = 0ull;
    if (pruned) {
        need[threadIdx.x] = 0;
        __syncthreads();
        if (valid0) need[p0] = 1;
        for (int64_t i = i0 + blockDim.x; i < hi; i += blockDim.x) need[assign[i]] = 1;
        __syncthreads();
        int total = 0;
        const int f = need[threadIdx.x];
        const int pos = block_exclusive_scan<int>(f, scan_tmp, &total);
        const int slot = (f && pos < kRowSlots) ? pos : -1;
        slot_of[threadIdx.x] = slot;
        if (slot >= 0) row_of[slot] = threadIdx.x;
        __syncthreads();
        // stage the leading entries of the needed rows: loads first, then stores
        const int nslots = total < kRowSlots ? total : kRowSlots;
        constexpr int kPer = kRowSlots * kRowCache / kAssignThreads;
        double dv[kPer];
        uint32_t mv[kPer];
        const double* __restrict__ td = gp(J.td);
        const uint8_t* __restrict__ tm = gp(J.tm);
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int e = u * kAssignThreads + threadIdx.x;
            const bool in = e < nslots * kRowCache;
            const int r = in ? row_of[e / kRowCache] : 0;
            dv[u] = in ? td[r * kRow + e % kRowCache] : 0.0;
            mv[u] = in ? tm[r * kRow + e % kRowCache] : 0u;
        }
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int e = u * kAssignThreads + threadIdx.x;
            if (e < nslots * kRowCache) {
                ltd[e] = dv[u];
                ltm[e] = uint8_t(mv[u]);
            }
        }
    }
    __syncthreads();

    unsigned long long ndc = 0, ties = 0;
    for (int64_t base = lo; base < hi; base += blockDim.x) {
        const int64_t i = base + threadIdx.x;
        const bool valid = i < hi;
        const bool first = base == lo;
        const uint32_t key = first ? key0 : (valid ? keys[i] : 0u);
        const unsigned long long w = first ? cnt0 : (valid ? counts[i] : 0u);
        int r, g, b;
        key_rgb(key, r, g, b);
        const double x0 = double(r), x1 = double(g), x2 = double(b);
        Best v{0.0, __builtin_inf(), 0};
        if (!pruned) {
            v = full_search(x0, x1, x2, centers, K);
            if (valid) ndc += unsigned(K);
        } else if (valid) {
            const int p = first ? p0 : assign[i];
            const double prev = dist_f64(x0, x1, x2, c[3 * p], c[3 * p + 1], c[3 * p + 2]);
            const double limit = 4.0 * prev * (1.0 + 1e-12);
            v.bd = prev;
            v.best = p;
            unsigned evals = 1;
            const int slot = slot_of[p];
            int j = 1;
            bool stopped = false;
            if (slot >= 0) {
                // staged prefix of row p: LDS reads only
                const int jend = K < kRowCache ? K : kRowCache;
                for (; j < jend; ++j) {
                    const double dj = ltd[slot * kRowCache + j];
                    const int t = ltm[slot * kRowCache + j];
                    if (dj > limit) {
                        stopped = true;
                        break;
                    }
                    best_push(v, dist_f64(x0, x1, x2, c[3 * t], c[3 * t + 1], c[3 * t + 2]), t);
                    ++evals;
                }
            }
            if (!stopped) {
                // rest of the row (or a row that was not staged) from global
                // memory, kFetch entries per round trip
                const double* __restrict__ grow_d = gp(J.td) + p * kRow;
                const uint8_t* __restrict__ grow_m = gp(J.tm) + p * kRow;
                for (; j < K && !stopped; j += kFetch) {
                    double dq[kFetch];
                    int tq[kFetch];
#pragma unroll
                    for (int q = 0; q < kFetch; ++q) {
                        const int jj = j + q < kRow ? j + q : kRow - 1;  // stays inside the row
                        dq[q] = grow_d[jj];
                        tq[q] = grow_m[jj];
                    }
#pragma unroll
                    for (int q = 0; q < kFetch; ++q) {
                        if (stopped) break;
                        if (j + q >= K || dq[q] > limit) {
                            stopped = true;
                            break;
                        }
                        const int t = tq[q];
                        best_push(v, dist_f64(x0, x1, x2, c[3 * t], c[3 * t + 1], c[3 * t + 2]), t);
                        ++evals;
                    }
                }
            }
            ndc += evals;
        }
        if (valid) {
            ties += near_tie(v) ? 1 : 0;
            assign[i] = uint8_t(v.best);
        }
        bin_add(bins, valid, v.best, w, r, g, b);
    }
    flush_counters(ndc, ties, red, meta);
    flush_bins(bins, K, sums);
}

// Exact unsigned 128-bit value converted to double by the fixed rule
// hi * 2^64 + lo, each conversion and the sum rounded to nearest.
__device__ __forceinline__ double u128_to_f64(unsigned __int128 v)
{
    const uint64_t hi = uint64_t(v >> 64);
    const uint64_t lo = uint64_t(v);
    return double(hi) * 18446744073709551616.0 + double(lo);
}

// acc + v[lane 0] + v[lane 1] + ... + v[lane 63], added one lane at a time in
// lane order (every lane returns the same value).
__device__ __forceinline__ double ordered_wave_sum(double acc, double v)
{
    const long long bits = __double_as_longlong(v);
    const int lo = int(bits & 0xffffffffll), hi = int(bits >> 32);
#pragma unroll
    for (int l = 0; l < 64; ++l) {
        const long long b = (long long)(unsigned)__builtin_amdgcn_readlane(lo, l) |
                            ((long long)__builtin_amdgcn_readlane(hi, l) << 32);
        acc += __longlong_as_double(b);
    }
    return acc;
}

// Update step, SSE, stopping rule and (pruned runs) the sorted table of the
// next iteration.  Job j gets K_j blocks of kMaxK threads when pruned, else 1.
// Every block derives the new centres from the cluster sums of this iteration
// in LDS; the job's block 0 alone writes the centres, the SSE trace and the
// control block and clears the sums of the next iteration.  An empty cluster
// keeps its centre: its global entry is neither rewritten nor changed, so the
// other blocks may read it.
__global__ void __launch_bounds__(kMaxK) k_update(const JobDev* __restrict__ jobs,
                                                  const int* __restrict__ map, int B)
{
    __shared__ double c[3 * kMaxK];
    __shared__ double term[kMaxK];
    __shared__ unsigned long long wsum[kMaxK];
    __shared__ double key[kMaxK];
    __shared__ double sdist[kMaxK];
    __shared__ int sidx[kMaxK];
    const int jb = find_job(map, B, blockIdx.x);
    const JobDev& J = jobs[jb];
    const int a = blockIdx.x - map[jb];
    Meta* __restrict__ meta = gp(J.meta);
    if (meta->done) return;
    const int it = meta->cur_it;
    const int K = J.K;
    double* __restrict__ centers = gp(J.centers);
    const unsigned long long* __restrict__ cur = gp(J.sums) + (it & 1) * 5 * kMaxK;
    unsigned long long* __restrict__ nxt = gp(J.sums) + ((it + 1) & 1) * 5 * kMaxK;
    const int k = threadIdx.x;
    double t = 0.0;
    unsigned long long nk = 0;
    if (k < K) {
        nk = cur[k];
        if (nk != 0) {
            const unsigned long long s0 = cur[kMaxK + 3 * k + 0];
            const unsigned long long s1 = cur[kMaxK + 3 * k + 1];
            const unsigned long long s2 = cur[kMaxK + 3 * k + 2];
            const unsigned long long q = cur[4 * kMaxK + k];
            const double dn = double(nk);
            c[3 * k + 0] = double(s0) / dn;
            c[3 * k + 1] = double(s1) / dn;
            c[3 * k + 2] = double(s2) / dn;
            const unsigned __int128 nq = (unsigned __int128)nk * q;
            const unsigned __int128 ss = (unsigned __int128)s0 * s0 + (unsigned __int128)s1 * s1 +
                                         (unsigned __int128)s2 * s2;
            t = u128_to_f64(nq - ss) / dn;
            if (a == 0) {
                centers[3 * k + 0] = c[3 * k + 0];
                centers[3 * k + 1] = c[3 * k + 1];
                centers[3 * k + 2] = c[3 * k + 2];
            }
        } else {
            c[3 * k + 0] = centers[3 * k + 0];
            c[3 * k + 1] = centers[3 * k + 1];
            c[3 * k + 2] = centers[3 * k + 2];
        }
    }
    term[k] = t;  // zero for k >= K and for empty clusters
    wsum[k] = nk;
    if (a == 0) {
        for (int j = k; j < 5 * kMaxK; j += blockDim.x) nxt[j] = 0ull;
    }
    __syncthreads();
    if (a == 0 && k < 64) {
        // SSE in ascending cluster order, walked through the registers of one
        // wave (lane l holds the terms of clusters l, l+64, l+128, l+192)
        const double t0 = term[k], t1 = term[k + 64], t2 = term[k + 128], t3 = term[k + 192];
        const unsigned long long total = wave_sum(wsum[k] + wsum[k + 64] + wsum[k + 128] + wsum[k + 192]);
        double sse = 0.0;
        sse = ordered_wave_sum(sse, t0);
        sse = ordered_wave_sum(sse, t1);
        sse = ordered_wave_sum(sse, t2);
        sse = ordered_wave_sum(sse, t3);
        if (k == 0) {
            meta->total_w = total;
            gp(J.trace)[it - 1] = sse;
            meta->iters = it;
            meta->sse_last = sse;
            bool stop = false, conv = false;
            if (sse == 0.0) {
                stop = conv = true;
            } else if (it >= 2) {
                const double drop = meta->sse_prev - sse;
                if (drop <= J.tol * sse) stop = conv = true;
            }
            if (it >= J.max_iters) stop = true;
            meta->sse_prev = sse;
            if (stop) {
                meta->done = 1;
                meta->converged = conv ? 1 : 0;
            }
        }
    }
    if (!J.prune) return;
    // row a of the table for the next iteration: the centres ordered by
    // (distance from c_a, index), a itself first (key -1); a bitonic sort of
    // kMaxK (key, index) pairs in LDS, slots past K keyed +inf
    const int b = k;
    double d = 0.0;
    if (b < K)
        d = dist_f64(c[3 * a], c[3 * a + 1], c[3 * a + 2], c[3 * b], c[3 * b + 1], c[3 * b + 2]);
    key[b] = b >= K ? __builtin_inf() : (b == a ? -1.0 : d);
    sidx[b] = b;
    sdist[b] = d;
    __syncthreads();
    for (int size = 2; size <= kMaxK; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            const int partner = b ^ stride;
            const double mk = key[b], pk = key[partner];
            const int mi = sidx[b], pi = sidx[partner];
            const bool partner_less = pk < mk || (pk == mk && pi < mi);
            const bool ascending = (b & size) == 0;
            const bool lower = b < partner;
            const bool take = (lower == ascending) ? partner_less : !partner_less;
            __syncthreads();
            if (take) {
                key[b] = pk;
                sidx[b] = pi;
            }
            __syncthreads();
        }
    }
    if (b >= K) return;
    const int src = sidx[b];
    gp(J.td)[a * kRow + b] = sdist[src];
    gp(J.tm)[a * kRow + b] = uint8_t(src);
}

// Palette: floor(c + 0.5) clamped to [0, 255]; also clears the squared-error
// accumulator of the pixel map.  One block per job.
__global__ void __launch_bounds__(3 * kMaxK) k_palette(const JobDev* __restrict__ jobs)
{
    const JobDev& J = jobs[blockIdx.x];
    const int t = threadIdx.x;
    if (t == 0) gp(J.meta)->sq_err = 0;
    if (t >= 3 * J.K) return;
    const double v = gp(J.centers)[t] + 0.5;
    int q;
    if (!(v >= 1.0))
        q = 0;
    else if (v >= 256.0)
        q = 255;
    else
        q = int(v);
    gp(J.palette)[t] = uint8_t(q);
}

// Per job: reset the run fields and both cluster-sum buffers; flag a
// non-finite starting centre; for N' <= K finish at once (centres = colours,
// assign[i] = i, SSE 0, no iteration).
__global__ void __launch_bounds__(kMaxK) k_kmeans_begin(const JobDev* __restrict__ jobs)
{
    const JobDev& J = jobs[blockIdx.x];
    Meta* __restrict__ meta = gp(J.meta);
    const int k = threadIdx.x;
    const int K = J.K;
    __shared__ int bad;
    if (k == 0) bad = 0;
    __syncthreads();
    const bool few = J.n <= K;
    if (few) {
        if (k < K) {
            if (k < J.n) {
                int r, g, b;
                key_rgb(J.keys[k], r, g, b);
                gp(J.centers)[3 * k + 0] = double(r);
                gp(J.centers)[3 * k + 1] = double(g);
                gp(J.centers)[3 * k + 2] = double(b);
                gp(J.assign)[k] = uint8_t(k);
            } else {
                gp(J.centers)[3 * k] = gp(J.centers)[3 * k + 1] = gp(J.centers)[3 * k + 2] = 0.0;
            }
        }
    } else if (k < K) {
        for (int c = 0; c < 3; ++c)
            if (!__builtin_isfinite(J.centers[3 * k + c])) atomicOr(&bad, 1);
    }
    for (int j = k; j < 10 * kMaxK; j += blockDim.x) gp(J.sums)[j] = 0;
    __syncthreads();
    if (k == 0) {
        meta->ndc = 0;
        meta->near_ties = 0;
        meta->iters = 0;
        meta->cur_it = 0;
        meta->converged = few ? 1 : 0;
        meta->sse_prev = 0.0;
        meta->sse_last = 0.0;
        meta->total_w = 0;
        meta->bad_input = bad;
        meta->done = (few || bad) ? 1 : 0;  // a bad start runs no iteration
    }
}

// ------------------------------------------------------------------ host
cq_status launch_kmeans_begin(const JobDev* jobs, int B, hipStream_t s)
{
    CQ_TIMED_LAUNCH("k_kmeans_begin", s, k_kmeans_begin<<<B, kMaxK, 0, s>>>(jobs));
    return CQ_OK;
}

// One iteration of every job that has not stopped.
cq_status launch_kmeans_iter(const JobDev* jobs, const int* maps, int B, int assign_blocks,
                             int update_blocks, hipStream_t s)
{
    CQ_TIMED_LAUNCH("k_assign", s, k_assign<<<assign_blocks, kAssignThreads, 0, s>>>(jobs, maps + kMapAssign * (B + 1), B));
    CQ_TIMED_LAUNCH("k_update", s, k_update<<<update_blocks, kMaxK, 0, s>>>(jobs, maps + kMapUpdate * (B + 1), B));
    return CQ_OK;
}

cq_status launch_palette(const JobDev* jobs, int B, hipStream_t s)
{
    CQ_TIMED_LAUNCH("k_palette", s, k_palette<<<B, 3 * kMaxK, 0, s>>>(jobs));
    return CQ_OK;
}

// Colours per assignment block.
int64_t assign_chunk(int64_t n)
{
    int64_t blocks = (n + kAssignThreads - 1) / kAssignThreads;
    if (blocks <= 4096) return kAssignThreads;
    const int64_t chunk = (n + 4095) / 4096;
    return (chunk + kAssignThreads - 1) / kAssignThreads * kAssignThreads;
}

}  // namespace cq
