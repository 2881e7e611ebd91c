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
#include <stdlib.h>

#include <mutex>

#include "batch.h"

// Every floating-point operation in this file is rounded on its own.
#pragma clang fp contract(off)

namespace cq {

constexpr int kAssignThreads = 256;
constexpr int kMaxAssignChunk = 32768;  // colours per block: the (cluster, bucket) counters are 16 bits
constexpr int kScatterChunk = 2048;  // colours per regrouping block

// Adds the five cluster statistics (n, S_r, S_g, S_b, Q) of the valid lanes
// to the LDS bins of their clusters, one LDS atomic per value and lane (lanes
// that share a cluster are serialized by the LDS unit, which costs the VALU
// nothing; summing them across the wave first costs five 64-bit reductions
// per distinct cluster).
__device__ __forceinline__ void bin_add_vals(unsigned long long* bins, bool valid, int k,
                                             unsigned long long v0, unsigned long long v1,
                                             unsigned long long v2, unsigned long long v3,
                                             unsigned long long v4)
{
    if (valid) {
        atomicAdd(&bins[kSumN + k], v0);
        atomicAdd(&bins[kSumS + 3 * k + 0], v1);
        atomicAdd(&bins[kSumS + 3 * k + 1], v2);
        atomicAdd(&bins[kSumS + 3 * k + 2], v3);
        atomicAdd(&bins[kSumQ + k], v4);
    }
}

// One colour (weight w, channels r, g, b) per valid lane into its cluster's bins.
__device__ __forceinline__ void bin_add(unsigned long long* bins, bool valid, int best,
                                        unsigned long long w, int r, int g, int b)
{
    bin_add_vals(bins, valid, best, w, w * unsigned(r), w * unsigned(g), w * unsigned(b),
                 w * unsigned(r * r + g * g + b * b));
}

// Running statistics of the colours a lane has put into one cluster, and
// the largest squared distance among them (bit pattern of the double).
struct Acc {
    int k;  // -1: empty
    unsigned long long n, s0, s1, s2, q, dmax;
};

__device__ __forceinline__ void acc_flush(const Acc& a, unsigned long long* bins, unsigned long long* maxd)
{
    atomicAdd(&bins[kSumN + a.k], a.n);
    atomicAdd(&bins[kSumS + 3 * a.k + 0], a.s0);
    atomicAdd(&bins[kSumS + 3 * a.k + 1], a.s1);
    atomicAdd(&bins[kSumS + 3 * a.k + 2], a.s2);
    atomicAdd(&bins[kSumQ + a.k], a.q);
    atomicMax(&maxd[a.k], a.dmax);
}

__device__ __forceinline__ void acc_add(Acc& a, unsigned long long* bins, unsigned long long* maxd, int k,
                                        unsigned long long w, int r, int g, int b, double d)
{
    if (k != a.k) {
        if (a.k >= 0) acc_flush(a, bins, maxd);
        a = Acc{k, 0ull, 0ull, 0ull, 0ull, 0ull, 0ull};
    }
    a.n += w;
    a.s0 += w * unsigned(r);
    a.s1 += w * unsigned(g);
    a.s2 += w * unsigned(b);
    a.q += w * unsigned(r * r + g * g + b * b);
    const unsigned long long db = (unsigned long long)__double_as_longlong(d);
    a.dmax = db > a.dmax ? db : a.dmax;
}

// Distance bucket of a colour: two per octave of d + 1, from 4 up (bucket 0
// also takes d + 1 < 4, bucket 15 everything from 1024 on).  Colours of a
// cluster that are about as far from its centre scan about as far along its
// table row, so the regrouping orders them by bucket within the cluster.
__device__ __forceinline__ int dist_bucket(double d)
{
    const unsigned long long bits = (unsigned long long)__double_as_longlong(d + 1.0);
    const int e = int((bits >> 52) & 0x7ffu) - 1023;
    const int b = 2 * e + int((bits >> 51) & 1u) - 4;
    return b < 0 ? 0 : (b > kBuckets - 1 ? kBuckets - 1 : b);
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

// Block reduction of the distance and near-tie counters into the block's own
// slot of the job's partial counts (plain stores: many blocks adding to one
// address would serialize); the update step adds the slots up.
__device__ __forceinline__ void flush_counters(unsigned long long ndc, unsigned long long ties,
                                               unsigned long long* red,
                                               unsigned long long* __restrict__ slot)
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
        slot[0] = a;
        slot[1] = t;
    }
}

// Adds the block's non-empty cluster bins and (cluster, bucket) colour
// counts to the job's statistics; in pruned runs (ccount and maxd non-null)
// also the largest squared distance of each cluster's colours.
__device__ __forceinline__ void flush_bins(const unsigned long long* bins, const uint32_t* ccount,
                                           const unsigned long long* maxd, int K,
                                           unsigned long long* __restrict__ sums)
{
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        const unsigned long long nk = bins[kSumN + k];
        if (nk == 0) continue;
        atomicAdd(&sums[kSumN + k], nk);
        atomicAdd(&sums[kSumS + 3 * k + 0], bins[kSumS + 3 * k + 0]);
        atomicAdd(&sums[kSumS + 3 * k + 1], bins[kSumS + 3 * k + 1]);
        atomicAdd(&sums[kSumS + 3 * k + 2], bins[kSumS + 3 * k + 2]);
        atomicAdd(&sums[kSumQ + k], bins[kSumQ + k]);
        if (maxd) atomicMax(&sums[kSumMaxD + k], maxd[k]);
    }
    if (!ccount) return;
    for (int w = threadIdx.x; w < K * kBuckets / 2; w += blockDim.x) {
        const uint32_t c = ccount[w];
        uint32_t* colours = reinterpret_cast<uint32_t*>(sums + kSumColours);
        if (c & 0xffffu) atomicAdd(&colours[2 * w], c & 0xffffu);
        if (c >> 16) atomicAdd(&colours[2 * w + 1], c >> 16);
    }
}

// One more colour of (cluster, bucket) pair cb in the block's packed counters.
__device__ __forceinline__ void count_pair(uint32_t* ccount, int cb)
{
    atomicAdd(&ccount[cb >> 1], 1u << ((cb & 1) << 4));
}

// FP64 minimum and maximum of two numbers (never NaN here), as single
// instructions: the compiler's fmin and fmax first quiet their operands when
// it cannot tell that they are results of arithmetic (values carried across
// a loop), one more instruction each.
__device__ __forceinline__ double min_f64(double a, double b)
{
    double r;
    asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

__device__ __forceinline__ double max_f64(double a, double b)
{
    double r;
    asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

__device__ __forceinline__ bool near_tie(const Best& v)
{
    return v.second != __builtin_inf() && (v.second - v.bd) <= 1e-5 * v.second;
}

// Full search over the centres for one colour per lane.  All lanes walk the
// same centre index, so every centre load has one address per wave.
// The same search when every centre is an integer colour (after an
// initialization that picks colours, before the first update): then each
// FP64 distance above is an exact integer, and so is
// |x - c|^2 = |x|^2 - (2 x.c - |c|^2).  Centre k is stored with
// (255 - k) - (|c|^2 << 8), so a colour's value for it, (x.c << 9) plus that,
// is ((2 x.c - |c|^2) << 8) | (255 - k) (x.c one four-byte dot product of the
// colours packed in key order): the largest value is the nearest centre,
// lowest index on ties, and the second largest gives the second smallest
// distance, as the FP64 search counts it (an equal distance included).  `ent`
// holds (packed centre, stored value) for the K centres, padded to an even
// count with values too small to matter for K >= 2.
__device__ __forceinline__ Best full_search_int(uint32_t x, const uint2* __restrict__ ent, int K)
{
    int b1 = -0x7fffffff - 1, b2 = -0x7fffffff - 1;
    const int K2 = (K + 1) & ~1;
#pragma unroll 4
    for (int k = 0; k < K2; k += 2) {
        const uint4 e = *reinterpret_cast<const uint4*>(ent + k);
        const int v0 = int((__builtin_amdgcn_udot4(x, e.x, 0u, false) << 9) + e.y);
        const int v1 = int((__builtin_amdgcn_udot4(x, e.z, 0u, false) << 9) + e.w);
        // the second largest of (b1, b2, v) is their median (one v_med3)
        b2 = max(min(b1, b2), min(max(b1, b2), v0));
        b1 = max(b1, v0);
        b2 = max(min(b1, b2), min(max(b1, b2), v1));
        b1 = max(b1, v1);
    }
    const int xx = int(__builtin_amdgcn_udot4(x, x, 0u, false));
    Best v;
    v.bd = double(xx - (b1 >> 8));
    v.second = K >= 2 ? double(xx - (b2 >> 8)) : __builtin_inf();
    v.best = 255 - (b1 & 255);
    return v;
}

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

// Packed colour record of the sort-means passes: bits 0-23 the colour key,
// bits 24-31 its cluster, bits 32-59 its pixel count (below 2^28 whenever
// there are two colours or more), bits 60-63 its distance bucket.
__device__ __forceinline__ uint64_t pack_colour(uint32_t key, int cluster, uint32_t count, int bucket)
{
    return uint64_t(key | (uint32_t(cluster) << 24)) | (uint64_t(count) << 32) | (uint64_t(bucket) << 60);
}

// Assignment fused with the cluster sums; block b of job j takes the colours
// [b chunk, (b + 1) chunk), one colour per lane.
//
// A full search (Algo. 1, the first iteration of Algo. 2) reads the colours in
// key order.  In a pruned run it also writes each colour as a packed record
// with its new cluster; the update step then regroups those records by
// cluster, so the sort-means passes that follow read colours that share their
// previous centre p.  A wave takes the distinct p of its lanes one at a time
// (nearly always one) and walks row p of the sorted table with one address per
// wave: entry j is evaluated by the lanes whose bound 4 d(x, c_p) (1 + 1e-12)
// it does not exceed, and the walk ends at the first entry beyond every
// lane's bound.  Rows are sorted, so each lane evaluates exactly the prefix of
// its row that the sequential scan of Algo. 2 evaluates.
//
// The two kinds of pass are separate kernels (kSortMeans false / true) so that each
// gets its own register allocation; a block whose job needs the other kind in
// this iteration returns at once.
template <bool kSortMeans>
__global__ void __launch_bounds__(kAssignThreads) k_assign(const JobDev* __restrict__ jobs,
                                                           const int* __restrict__ map, int B)
{
    __shared__ unsigned long long bins[5 * kMaxK];     // n, S0, S1, S2, Q per cluster
    // colours per (cluster, bucket) in pruned runs, two 16-bit counters per
    // word (a block holds at most 32768 colours)
    __shared__ uint32_t ccount[kMaxK * kBuckets / 2];
    __shared__ unsigned long long red[2 * (kAssignThreads / 64)];
    __shared__ unsigned long long s_maxd[kMaxK];  // pruned runs: per cluster, the largest squared distance
    __shared__ int s_slice;  // sort-means passes: the block's next slice of 64 colours
    // full searches with integer centres: (packed centre, stored value)
    __shared__ __align__(16) uint2 s_ent[kSortMeans ? 2 : kMaxK];
    const int jb = find_job(map, B, blockIdx.x);
    const JobDev& J = jobs[jb];
    const int lb = blockIdx.x - map[jb];
    Meta* __restrict__ meta = gp(J.meta);
    const int K = J.K;
    const int64_t n = J.n;
    const int64_t lo = int64_t(lb) * J.chunk;
    const int64_t hi = lo + J.chunk < n ? lo + J.chunk : n;
    const int done = meta->done;
    const int it = meta->iters + 1;
    if (done) return;
    const bool grouped = J.prune && it >= 2;
    if (grouped != kSortMeans) return;
    if (lb == 0 && threadIdx.x == 0) meta->cur_it = it;
    unsigned long long* __restrict__ sums = gp(J.sums) + (it & 1) * kSumStride;
    uint64_t* __restrict__ grp = gp(J.grp) + record_buffer(it, J.regroup_period) * n;
    for (int t = threadIdx.x; t < 5 * kMaxK; t += blockDim.x) bins[t] = 0ull;
    if (J.prune) {
        for (int t = threadIdx.x; t < K * kBuckets / 2; t += blockDim.x) ccount[t] = 0u;
        for (int t = threadIdx.x; t < K; t += blockDim.x) s_maxd[t] = 0ull;
        // the centres of this assignment, kept for the update (which
        // replaces them): the distance a centre moves bounds how far the
        // next scans of its cluster's colours can reach
        if (lb == 0)
            for (int t = threadIdx.x; t < 3 * K; t += blockDim.x) gp(J.cprev)[t] = gp(J.centers)[t];
    }
    if (threadIdx.x == 0) s_slice = 0;
    __syncthreads();

    unsigned long long ndc = 0, ties = 0;
    if constexpr (!kSortMeans) {
        const double* __restrict__ centers = gp(J.centers);
        const uint32_t* __restrict__ keys = gp(J.keys);
        const uint32_t* __restrict__ counts = gp(J.counts);
        uint8_t* __restrict__ assign = gp(J.assign);
        // integer centres: the integer search (same results, fewer instructions)
        bool whole = true;
        for (int t = threadIdx.x; t < 3 * K; t += blockDim.x) {
            const double c = centers[t];
            whole = whole && c >= 0.0 && c <= 255.0 && c == __builtin_trunc(c);
        }
        const bool integral = __syncthreads_and(whole ? 1 : 0) != 0;
        if (integral) {
            for (int t = threadIdx.x; t < kMaxK; t += blockDim.x) {
                uint32_t packed = 0;
                int pp = 0x3fffff;
                if (t < K) {
                    const int r = int(centers[3 * t]), g = int(centers[3 * t + 1]), b = int(centers[3 * t + 2]);
                    packed = (uint32_t(r) << 16) | (uint32_t(g) << 8) | uint32_t(b);
                    pp = r * r + g * g + b * b;
                }
                s_ent[t] = make_uint2(packed, uint32_t((255 - t) - (pp << 8)));
            }
            __syncthreads();
        }
        for (int64_t base = lo; base < hi; base += blockDim.x) {
            const int64_t i = base + threadIdx.x;
            const bool valid = i < hi;
            const uint32_t key = valid ? keys[i] : 0u;
            const uint32_t w = valid ? counts[i] : 0u;
            int r, g, b;
            key_rgb(key, r, g, b);
            const Best v = integral ? full_search_int(key, s_ent, K)
                                    : full_search(double(r), double(g), double(b), centers, K);
            if (valid) {
                ndc += unsigned(K);
                ties += near_tie(v) ? 1 : 0;
                assign[i] = uint8_t(v.best);
                if (J.prune) {
                    const int bk = dist_bucket(v.bd);
                    grp[i] = pack_colour(key, v.best, w, bk);
                    count_pair(ccount, v.best * kBuckets + bk);
                    atomicMax(&s_maxd[v.best], (unsigned long long)__double_as_longlong(v.bd));
                }
            }
            bin_add(bins, valid, v.best, w, r, g, b);
        }
    } else {
        const Rec CQ_CONST* rec = cp(J.rec);
        const uint8_t CQ_CONST* ord = cp(J.ord);
        Acc acc{-1, 0ull, 0ull, 0ull, 0ull, 0ull, 0ull};
        unsigned long long wave_evals = 0;  // the same in every lane
        // the waves take the block's slices of 64 colours in order from an LDS
        // counter, so a wave that finishes early takes more of them; each wave
        // takes its next slice, and starts loading it, before working on the
        // current one
        const int lane = threadIdx.x & 63;
        const int nslices = int((hi - lo + 63) / 64);
        auto take = [&]() { return __builtin_amdgcn_readfirstlane(lane == 0 ? atomicAdd(&s_slice, 1) : 0); };
        int sl = take();
        uint64_t g_next = sl < nslices && lo + sl * 64 + lane < hi ? grp[lo + sl * 64 + lane] : 0ull;
        while (sl < nslices) {
            const int64_t i = lo + int64_t(sl) * 64 + lane;
            const bool valid = i < hi;
            const uint64_t g0 = g_next;
            sl = take();
            g_next = sl < nslices && lo + sl * 64 + lane < hi ? grp[lo + sl * 64 + lane] : 0ull;  // in flight
            const uint32_t key = uint32_t(g0) & 0xffffffu;
            const int p = int((uint32_t(g0) >> 24) & 255u);
            const uint32_t w = uint32_t(g0 >> 32) & 0x0fffffffu;
            int r, g, b;
            key_rgb(key, r, g, b);
            const double x0 = double(r), x1 = double(g), x2 = double(b);
            Best vf{0.0, __builtin_inf(), 0};  // the lane's result, kept when its own row is walked
            unsigned long long pending = __ballot(valid);
            while (pending) {
                const int leader = __ffsll(pending) - 1;
                const int ps = __builtin_amdgcn_readlane(p, leader);
                const bool mine = valid && p == ps;
                // row ps of the table: entry 0 is centre ps itself, then the
                // other centres by distance from it; their indices are the
                // row's centre order, one byte each (four to a word)
                const Rec CQ_CONST* row = rec + ps * kRow;
                const uint32_t CQ_CONST* orow = reinterpret_cast<const uint32_t CQ_CONST*>(ord + ps * kRow);
                // the first round (the own entry and three more) in one round
                // trip; each round's evaluation overlaps the loads of the next
                Rec q[kWalk];
#pragma unroll
                for (int u = 0; u < kWalk; ++u) q[u] = row[u];
                uint32_t t4 = orow[0];
                // an empty statement that needs them all: the loads are
                // issued here, and waited for together, not one after the other
                static_assert(kWalk == 4, "a round's centre indices are one word; the statement below names every entry");
                asm volatile("" ::"s"(q[0].c0), "s"(q[0].c1), "s"(q[0].c2), "s"(q[1].c0), "s"(q[1].c1), "s"(q[1].c2),
                             "s"(q[1].d), "s"(q[2].c0), "s"(q[2].c1), "s"(q[2].c2), "s"(q[2].d), "s"(q[3].c0),
                             "s"(q[3].c1), "s"(q[3].c2), "s"(q[3].d), "s"(t4));
                const double prev = dist_f64(x0, x1, x2, q[0].c0, q[0].c1, q[0].c2);
                const double limit = 4.0 * prev * (1.0 + 1e-12);
                // Every lane of the wave follows the row; the lanes of other
                // rows keep their own results in vf.  The nearest distance is
                // taken over every entry walked, also those beyond a lane's
                // bound: such an entry is farther than the own centre (the
                // bound's relative margin of 1e-12 exceeds the rounding of
                // the three distances involved by far), so it is never nearer
                // than the best so far, nor equal to it.  The centre is the
                // first one met at that distance, which is the right one
                // unless another entry lies at exactly the same distance.
                // The second smallest distance over the entries walked is at
                // most the one over the entries the lane evaluates, and equal
                // to the nearest distance if there is such a tie; both are
                // made exact below where they matter.
                Best v{prev, __builtin_inf(), ps};
                // the distance count is a block total: the wave adds its
                // evaluations in scalar registers (lane masks), and lane 0
                // reports them
                const unsigned long long mine_mask = __builtin_amdgcn_ballot_w64(mine);
                wave_evals += (unsigned long long)__popcll(mine_mask);
                auto visit = [&](const Rec& e, int te) {
                    // lanes of this row whose bound takes the entry (compare
                    // predicate 5: ordered less or equal), for the count only
                    wave_evals += (unsigned long long)__popcll(__builtin_amdgcn_fcmp(e.d, limit, 5) & mine_mask);
                    const double d = dist_f64(x0, x1, x2, e.c0, e.c1, e.c2);
                    const bool better = d < v.bd;
                    v.second = min_f64(v.second, max_f64(v.bd, d));
                    v.bd = min_f64(v.bd, d);
                    v.best = better ? te : v.best;
                };
                // entries j .. j + kWalk - 1 per round; the table is padded so
                // that the last round of a row, and the round loaded ahead of
                // it, stay inside the allocation
                for (int j = 0; j < K; j += kWalk) {
                    Rec qn[kWalk];
                    uint32_t t4n = 0;
                    // the next round is needed if the bound of some lane of
                    // the row takes this round's last entry
                    const bool ahead =
                        j + kWalk < K && (__builtin_amdgcn_fcmp(q[kWalk - 1].d, limit, 5) & mine_mask) != 0ull;
                    if (ahead) {
#pragma unroll
                        for (int u = 0; u < kWalk; ++u) qn[u] = row[j + kWalk + u];
                        t4n = orow[(j + kWalk) / kWalk];
                    }
                    if (j > 0 && j + kWalk <= K) {
#pragma unroll
                        for (int u = 0; u < kWalk; ++u) {
                            visit(q[u], int((t4 >> (8 * u)) & 255u));
                            // one entry at a time: fewer registers, more waves per SIMD
                            __builtin_amdgcn_sched_barrier(0);
                        }
                    } else {
                        // the row's first round (its entry 0, the own centre,
                        // is taken above) or its last (entries from K on are
                        // no centres)
#pragma unroll
                        for (int u = 0; u < kWalk; ++u)
                            if (j + u > 0 && j + u < K) visit(q[u], int((t4 >> (8 * u)) & 255u));
                    }
                    if (!ahead) break;
#pragma unroll
                    for (int u = 0; u < kWalk; ++u) q[u] = qn[u];
                    t4 = t4n;
                }
                // The near-tie test, (second - bd) <= 1e-5 second, depends on
                // the exact second smallest distance s only where the lower
                // bound s' above is within twice that tolerance: from
                // s' - bd > 2e-5 s' and s >= s' follows s - bd > 1e-5 s with a
                // margin of about 1e-5 s, far above the rounding of the test.
                // The same lanes include every lane with an exact tie at the
                // nearest distance (s' = bd).  They (a few in ten thousand)
                // read the entries their bound takes again: the nearest
                // centre is the lowest index at distance bd, and the second
                // smallest distance is bd if two entries lie there, else the
                // smallest distance above bd.
                const bool recheck =
                    mine && v.second != __builtin_inf() && (v.second - v.bd) <= 2e-5 * v.second;
                if (__ballot(recheck) != 0ull) {
                    int at_bd = prev == v.bd ? 1 : 0;
                    int low = prev == v.bd ? ps : kMaxK;
                    double above = prev > v.bd ? prev : __builtin_inf();
                    for (int j = 1; j < K; ++j) {
                        const Rec e = row[j];
                        // no lane of the row evaluates this entry, or any later one
                        if ((__builtin_amdgcn_fcmp(e.d, limit, 5) & mine_mask) == 0ull) break;
                        const int te = int((orow[j / kWalk] >> (8 * (j % kWalk))) & 255u);
                        const double d = dist_f64(x0, x1, x2, e.c0, e.c1, e.c2);
                        if (e.d <= limit) {
                            if (d == v.bd) {
                                ++at_bd;
                                low = te < low ? te : low;
                            } else {
                                above = __builtin_fmin(above, d);
                            }
                        }
                    }
                    if (recheck) {
                        v.best = low;
                        v.second = at_bd >= 2 ? v.bd : above;
                    }
                }
                if (mine) vf = v;
                pending &= ~mine_mask;
            }
            if (valid) {
                ties += near_tie(vf) ? 1 : 0;
                const int bk = dist_bucket(vf.bd);
                const uint64_t rec_new = pack_colour(key, vf.best, w, bk);
                if (rec_new != g0) grp[i] = rec_new;  // most records stay as they are
                count_pair(ccount, vf.best * kBuckets + bk);
                acc_add(acc, bins, s_maxd, vf.best, w, r, g, b, vf.bd);
            }
        }
        if (lane == 0) ndc += wave_evals;
        // each lane's last cluster straight into LDS: lanes that share a
        // cluster are serialized by the LDS unit, cheaper than reducing
        // five 64-bit values across the wave
        if (acc.k >= 0) acc_flush(acc, bins, s_maxd);
    }
    __syncthreads();
    flush_counters(ndc, ties, red, gp(J.part) + 2 * lb);
    flush_bins(bins, J.prune ? ccount : nullptr, J.prune ? s_maxd : nullptr, K, sums);
}

// Exact unsigned 128-bit value converted to double by the fixed rule
// hi * 2^64 + lo, each conversion and the sum rounded to nearest.
__device__ __forceinline__ double u128_to_f64(unsigned __int128 v)
{
    const uint64_t hi = uint64_t(v >> 64);
    const uint64_t lo = uint64_t(v);
    return double(hi) * 18446744073709551616.0 + double(lo);
}

// Regrouping of a pruned run: this iteration's colour records (new cluster
// in bits 24-31, distance bucket in bits 60-63) are moved into the other
// record buffer ordered by (cluster, bucket), a counting sort whose offsets
// are the prefix sums of the (cluster, bucket) colour counts.  The order
// inside a pair is whatever the atomics give; no result depends on it.  Block
// s of the job's regrouping blocks takes the records [s chunk, (s + 1) chunk)
// (chunk: the job's assignment block size), kScatterChunk at a time.
constexpr int kPairs = kMaxK * kBuckets;
constexpr int kPairsPer = kPairs / kMaxK;  // pairs per thread in the regrouping scan
// LDS words of the regrouping offsets: pair cb lives at cb + cb / kPairsPer,
// so each thread's pairs are consecutive and the threads' runs start in
// different banks
constexpr int kStartWords = kPairs + kPairs / kPairsPer;

__device__ __forceinline__ void regroup(const JobDev& J, int s, int it, const uint32_t* __restrict__ colours,
                                        uint32_t* __restrict__ cursor, uint32_t* start, uint32_t* scan_tmp)
{
    constexpr int kPer = kPairsPer;
    const int k = threadIdx.x;
    const int lane = k & 63;
    const int npairs = J.K * kBuckets;
    const int64_t n = J.n;
    const int rb = record_buffer(it, J.regroup_period);
    const uint64_t* __restrict__ src = gp(J.grp) + rb * n;
    uint64_t* __restrict__ dst = gp(J.grp) + (rb ^ 1) * n;
    const unsigned long long below = (1ull << lane) - 1ull;
    constexpr int kPasses = kScatterChunk / kMaxK;
    // the block takes J.chunk records (the assignment blocks' size) in
    // sub-chunks of kScatterChunk: the offsets are computed once per block
    const int64_t lo = int64_t(s) * J.chunk;
    const int64_t hi = lo + J.chunk < n ? lo + J.chunk : n;
    // the first sub-chunk's records first, in flight while the offsets are computed
    uint64_t g[kPasses];
#pragma unroll
    for (int u = 0; u < kPasses; ++u) {
        const int64_t i = lo + u * kMaxK + k;
        g[u] = i < hi ? src[i] : 0ull;
    }
    // pair counts: coalesced loads into LDS, then each thread scans its run
    // of kPer consecutive pairs
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int cb = u * kMaxK + k;
        start[cb + cb / kPer] = cb < npairs ? colours[cb] : 0u;
    }
    __syncthreads();
    uint32_t c[kPer];
    uint32_t tsum = 0;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        c[u] = start[k * (kPer + 1) + u];
        tsum += c[u];
    }
    uint32_t run = block_exclusive_scan<uint32_t>(tsum, scan_tmp, nullptr);
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        start[k * (kPer + 1) + u] = run;
        run += c[u];
    }
    __syncthreads();
    for (int64_t sub = lo; sub < hi; sub += kScatterChunk) {
        if (sub > lo) {
#pragma unroll
            for (int u = 0; u < kPasses; ++u) {
                const int64_t i = sub + u * kMaxK + k;
                g[u] = i < hi ? src[i] : 0ull;
            }
        }
        // every record of the sub-chunk is ranked within its wave's group of
        // equal (cluster, bucket) first; the group leaders then reserve
        // their places with atomics that are all in flight together
        int cbv[kPasses], lead[kPasses], rank[kPasses];
        uint32_t pos[kPasses];
#pragma unroll
        for (int u = 0; u < kPasses; ++u) {
            const bool valid = sub + u * kMaxK + k < hi;
            cbv[u] = int((uint32_t(g[u]) >> 24) & 255u) * kBuckets + int(g[u] >> 60);
            lead[u] = -1;
            rank[u] = 0;
            int gsize = 0;
            unsigned long long pending = __ballot(valid);
            while (pending) {
                const int leader = __ffsll(pending) - 1;
                const int cs = __builtin_amdgcn_readlane(cbv[u], leader);
                const bool mine = valid && cbv[u] == cs;
                const unsigned long long mask = __ballot(mine);
                if (mine) {
                    lead[u] = leader;
                    rank[u] = __popcll(mask & below);
                }
                if (lane == leader) gsize = __popcll(mask);
                pending &= ~mask;
            }
            pos[u] = 0;
            if (gsize > 0) pos[u] = atomicAdd(&cursor[cbv[u]], uint32_t(gsize));
        }
#pragma unroll
        for (int u = 0; u < kPasses; ++u) {
            const uint32_t base = __shfl(pos[u], lead[u] < 0 ? 0 : lead[u], 64);
            if (lead[u] >= 0) dst[start[cbv[u] + cbv[u] / kPer] + base + rank[u]] = g[u];
        }
    }
}

// (key, index) order of table entries.
__device__ __forceinline__ bool entry_less(double k1, int i1, double k2, int i2)
{
    return k1 < k2 || (k1 == k2 && i1 < i2);
}

// Row `a` of the table for the next iteration, built by one wave: the
// centres ordered by (distance from c_a, index), a itself first (key -1),
// slots past K keyed +inf.  Lane l holds the four consecutive entries 4 l ..
// 4 l + 3 in registers.  The centres move little from one iteration to the
// next, so the row starts from its previous order (iteration 1: index
// order): if that is still sorted nothing moves, otherwise up to kFixPasses
// rounds of odd-even transposition repair it (the pairs inside a lane in
// registers, the pair across two lanes with one shuffle), and a bitonic sort
// of the whole row handles whatever is left.
constexpr int kFixPasses = 8;
constexpr int kRowsPerBlock = kMaxK / 64;  // one wave per row
constexpr int kPerLane = kRow / 64;        // entries per lane

__device__ __forceinline__ void cmp_swap(double& k0, int& i0, double& k1, int& i1)
{
    if (entry_less(k1, i1, k0, i0)) {
        const double tk = k0;
        const int ti = i0;
        k0 = k1;
        i0 = i1;
        k1 = tk;
        i1 = ti;
    }
}

// The row's previous order (iteration 1: index order), one entry per
// register: loaded before the centres are derived so the two overlap.
__device__ __forceinline__ void load_row_order(const JobDev& J, int a, int K, int it, int* prev)
{
    const int lane = threadIdx.x & 63;
    const uint8_t* __restrict__ orow = gp(J.ord) + a * kRow;
    // lane l's four order bytes in one load (rows are kRow bytes apart)
    const uint32_t four = (it > 1 && a < K) ? reinterpret_cast<const uint32_t*>(orow)[lane] : 0u;
#pragma unroll
    for (int i = 0; i < kPerLane; ++i) {
        const int e = kPerLane * lane + i;
        prev[i] = (it > 1 && e < K && a < K) ? int((four >> (8 * i)) & 255u) : e;
    }
}

__device__ __forceinline__ void build_row(const JobDev& J, int a, int K, const double* c, const int* prev,
                                          double reach)
{
    const int lane = threadIdx.x & 63;
    Rec* __restrict__ row = gp(J.rec) + a * kRow;
    const double a0 = c[3 * a], a1 = c[3 * a + 1], a2 = c[3 * a + 2];
    double k[kPerLane];
    int x[kPerLane];
#pragma unroll
    for (int i = 0; i < kPerLane; ++i) {
        const int f = prev[i];
        x[i] = f;
        k[i] = f >= K ? __builtin_inf()
                      : (f == a ? -1.0 : dist_f64(a0, a1, a2, c[3 * f], c[3 * f + 1], c[3 * f + 2]));
    }
    auto unsorted = [&]() {
        bool u = false;
#pragma unroll
        for (int i = 0; i + 1 < kPerLane; ++i) u = u || entry_less(k[i + 1], x[i + 1], k[i], x[i]);
        const double nk = __shfl_down(k[0], 1, 64);
        const int nx = __shfl_down(x[0], 1, 64);
        if (lane < 63) u = u || entry_less(nk, nx, k[kPerLane - 1], x[kPerLane - 1]);
        return __ballot(u) != 0ull;
    };
    bool uns = unsorted();
    for (int pass = 0; uns && pass < kFixPasses; ++pass) {
        // even pairs (2m, 2m+1): inside the lane
#pragma unroll
        for (int i = 0; i + 1 < kPerLane; i += 2) cmp_swap(k[i], x[i], k[i + 1], x[i + 1]);
        // odd pairs (2m+1, 2m+2): inside the lane, and the lane's last entry
        // with the next lane's first (each side keeps its half of the pair)
#pragma unroll
        for (int i = 1; i + 1 < kPerLane; i += 2) cmp_swap(k[i], x[i], k[i + 1], x[i + 1]);
        const double nk = __shfl_down(k[0], 1, 64);
        const int nx = __shfl_down(x[0], 1, 64);
        const double pk = __shfl_up(k[kPerLane - 1], 1, 64);
        const int px = __shfl_up(x[kPerLane - 1], 1, 64);
        if (lane < 63 && entry_less(nk, nx, k[kPerLane - 1], x[kPerLane - 1])) {
            k[kPerLane - 1] = nk;
            x[kPerLane - 1] = nx;
        }
        if (lane > 0 && entry_less(k[0], x[0], pk, px)) {
            k[0] = pk;
            x[0] = px;
        }
        uns = unsorted();
    }
    if (uns) {
        // bitonic sort over entry e = kPerLane lane + i: partners kPerLane or
        // more apart sit in other lanes (same register), closer ones in this lane
        for (int size = 2; size <= kRow; size <<= 1) {
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                if (stride >= kPerLane) {
                    const int ls = stride / kPerLane;
#pragma unroll
                    for (int i = 0; i < kPerLane; ++i) {
                        const double pk = __shfl_xor(k[i], ls, 64);
                        const int px = __shfl_xor(x[i], ls, 64);
                        const int e = kPerLane * lane + i;
                        const bool ascending = (e & size) == 0;
                        const bool lower = (e & stride) == 0;
                        const bool partner_less = entry_less(pk, px, k[i], x[i]);
                        if ((lower == ascending) ? partner_less : !partner_less) {
                            k[i] = pk;
                            x[i] = px;
                        }
                    }
                } else {
#pragma unroll
                    for (int i = 0; i < kPerLane; ++i) {
                        if (i & stride) continue;
                        const int j = i | stride;
                        const bool ascending = ((kPerLane * lane + i) & size) == 0;
                        if (ascending)
                            cmp_swap(k[i], x[i], k[j], x[j]);
                        else
                            cmp_swap(k[j], x[j], k[i], x[i]);
                    }
                }
            }
        }
    }
    // The scans of this row (colours whose previous centre is a) evaluate
    // entries up to their own bound, which is at most `reach`; P entries lie
    // within it (the own entry first).  A scan reads whole rounds of kWalk
    // entries (entries 0 .. kWalk - 1 first), and the round after one whose
    // last entry is within its bound, so the entries it can read end with
    // the round that holds entry P (at least the first round).  Only those
    // records are written; the centre order, which also gives the scans the
    // centre index of each entry, is written whole, since the next update
    // starts its sort from it.
    int within = 0;
#pragma unroll
    for (int i = 0; i < kPerLane; ++i) within += (kPerLane * lane + i < K && k[i] <= reach) ? 1 : 0;
    const int P = wave_sum(within);
    const int last = P / kWalk * kWalk + kWalk - 1;
    uint32_t four = 0;
#pragma unroll
    for (int i = 0; i < kPerLane; ++i) {
        const int e = kPerLane * lane + i;
        four |= uint32_t(x[i] & 255) << (8 * i);
        if (e >= K || e > last) continue;
        Rec r;
        r.c0 = c[3 * x[i]];
        r.c1 = c[3 * x[i] + 1];
        r.c2 = c[3 * x[i] + 2];
        r.d = x[i] == a ? 0.0 : k[i];
        row[e] = r;
    }
    reinterpret_cast<uint32_t*>(gp(J.ord) + a * kRow)[lane] = four;  // entries past K are never read
}

// Update step, SSE, stopping rule and, in pruned runs, the sorted table and
// colour order of the next iteration.  A pruned job gets ceil(K_j / 4) table
// blocks (one wave per row) followed by its regrouping blocks; an unpruned
// job a single block.  Every table block derives the new centres from this
// iteration's cluster sums in LDS; the job's block 0 alone writes the
// centres, the SSE trace and the control block and clears the statistics of
// the next iteration.  An empty cluster keeps its centre: its global entry is
// neither rewritten nor changed, so the other blocks may read it.
__host__ __device__ __forceinline__ int table_blocks_of(int K, int prune)
{
    return prune ? (K + kRowsPerBlock - 1) / kRowsPerBlock : 1;
}

__device__ __forceinline__ int table_blocks(const JobDev& J) { return table_blocks_of(J.K, J.prune); }

__global__ void __launch_bounds__(kMaxK) k_update(const JobDev* __restrict__ jobs,
                                                  const int* __restrict__ map, int B)
{
    // one LDS buffer, used either by a table block or by a regrouping block
    constexpr int kTableWords = 2 * (3 * kMaxK + kMaxK + kMaxK + 2 * (kMaxK / 64));
    constexpr int kLdsWords = kTableWords > kStartWords + 64 ? kTableWords : kStartWords + 64;
    __shared__ __attribute__((aligned(16))) uint32_t smem[kLdsWords];
    const int jb = find_job(map, B, blockIdx.x);
    const JobDev& J = jobs[jb];
    const int a = blockIdx.x - map[jb];
    Meta* __restrict__ meta = gp(J.meta);
    if (meta->done) return;
    const int it = meta->cur_it;
    const int K = J.K;
    unsigned long long* __restrict__ cur = gp(J.sums) + (it & 1) * kSumStride;
    unsigned long long* __restrict__ nxt = gp(J.sums) + ((it + 1) & 1) * kSumStride;
    const int ntab = table_blocks(J);
    if (a >= ntab) {
        if (regroup_at(it, J.regroup_period))
            regroup(J, a - ntab, it, reinterpret_cast<const uint32_t*>(cur + kSumColours),
                    reinterpret_cast<uint32_t*>(cur + kSumCursor), smem, smem + kStartWords);
        return;
    }
    double* c = reinterpret_cast<double*>(smem);
    double* term = c + 3 * kMaxK;
    unsigned long long* wsum = reinterpret_cast<unsigned long long*>(term + kMaxK);
    unsigned long long* cnt_red = wsum + kMaxK;
    double* __restrict__ centers = gp(J.centers);
    const int k = threadIdx.x;
    const int r = a * kRowsPerBlock + int(threadIdx.x >> 6);  // this wave's table row
    int prev[kPerLane];
    if (J.prune) load_row_order(J, r, K, it, prev);
    double t = 0.0;
    unsigned long long nk = 0;
    if (k < K) {
        nk = cur[kSumN + k];
        if (nk != 0) {
            const unsigned long long s0 = cur[kSumS + 3 * k + 0];
            const unsigned long long s1 = cur[kSumS + 3 * k + 1];
            const unsigned long long s2 = cur[kSumS + 3 * k + 2];
            const unsigned long long q = cur[kSumQ + k];
            const double dn = double(nk);
            c[3 * k + 0] = double(s0) / dn;
            c[3 * k + 1] = double(s1) / dn;
            c[3 * k + 2] = double(s2) / dn;
            if (a == 0) {
                // the cluster's SSE term, exactly from the integer sums
                const unsigned __int128 nq = (unsigned __int128)nk * q;
                const unsigned __int128 ss = (unsigned __int128)s0 * s0 + (unsigned __int128)s1 * s1 +
                                             (unsigned __int128)s2 * s2;
                t = u128_to_f64(nq - ss) / dn;
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
    term[k] = t;  // zero for k >= K, for empty clusters and outside block 0
    wsum[k] = nk;
    {
        // the next iteration's statistics start at zero; the job's table
        // blocks clear a slice each
        const int per = (kSumStride + ntab - 1) / ntab;
        const int end = (a + 1) * per < kSumStride ? (a + 1) * per : kSumStride;
        for (int j = a * per + k; j < end; j += blockDim.x) nxt[j] = 0ull;
    }
    if (a == 0) {
        // distance and near-tie counts of this iteration's assignment blocks
        const int nblk = int((J.n + J.chunk - 1) / J.chunk);
        const unsigned long long* __restrict__ part = gp(J.part);
        unsigned long long pn = 0, pt = 0;
        for (int j = k; j < nblk; j += blockDim.x) {
            pn += part[2 * j];
            pt += part[2 * j + 1];
        }
        pn = wave_sum(pn);
        pt = wave_sum(pt);
        if ((k & 63) == 0) {
            cnt_red[k >> 6] = pn;
            cnt_red[(kMaxK / 64) + (k >> 6)] = pt;
        }
    }
    __syncthreads();
    if (a == 0 && k < 64) {
        const unsigned long long total = wave_sum(wsum[k] + wsum[k + 64] + wsum[k + 128] + wsum[k + 192]);
        if (k == 0) {
            // SSE in ascending cluster order, one addition at a time
            double sse = 0.0;
#pragma unroll 16
            for (int q = 0; q < kMaxK; ++q) sse += term[q];
            unsigned long long pn = 0, pt = 0;
            for (int w = 0; w < kMaxK / 64; ++w) {
                pn += cnt_red[w];
                pt += cnt_red[(kMaxK / 64) + w];
            }
            meta->ndc += pn;
            meta->near_ties += pt;
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
    if (r < K) {
        // Bound of every scan of row r in the next iteration.  A colour x in
        // cluster r was at squared distance at most M from the centre c it
        // was assigned to (the cluster's largest), and the centre moved to
        // c' by s = |c' - c|, so |x - c'| <= sqrt(M) + s, and its scan bound
        // 4 |x - c'|^2 (1 + 1e-12) is at most 4 (sqrt(M) + s)^2 (1 + 1e-12).
        // The relative 1e-9 and absolute 1e-9 on top cover the rounding of
        // every step here and in the scan's own distance.
        const double m = __longlong_as_double((long long)cur[kSumMaxD + r]);
        const double* __restrict__ cp = gp(J.cprev);
        const double s2 = dist_f64(c[3 * r], c[3 * r + 1], c[3 * r + 2], cp[3 * r], cp[3 * r + 1], cp[3 * r + 2]);
        const double rad = __builtin_sqrt(m) + __builtin_sqrt(s2);
        const double reach = 4.0 * rad * rad * (1.0 + 1e-12) * (1.0 + 1e-9) + 1e-9;
        build_row(J, r, K, c, prev, reach);
    }
}

// Pruned runs that grouped their colours: the final cluster of every colour
// back into key order (the keys ascend, so a binary search finds a colour's
// index).  Block b of job j takes the records [b chunk, (b + 1) chunk).
__global__ void __launch_bounds__(kAssignThreads) k_unpermute(const JobDev* __restrict__ jobs,
                                                              const int* __restrict__ map, int B)
{
    const int jb = find_job(map, B, blockIdx.x);
    const JobDev& J = jobs[jb];
    const int lb = blockIdx.x - map[jb];
    const int iters = gp(J.meta)->iters;
    if (!J.prune || iters < 2) return;
    const int64_t n = J.n;
    const uint64_t* __restrict__ g = gp(J.grp) + record_buffer(iters, J.regroup_period) * n;
    const uint32_t* __restrict__ keys = gp(J.keys);
    uint8_t* __restrict__ assign = gp(J.assign);
    const int64_t lo = int64_t(lb) * J.chunk;
    const int64_t hi = lo + J.chunk < n ? lo + J.chunk : n;
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
        const uint32_t v = uint32_t(g[i]);
        const uint32_t key = v & 0xffffffu;
        int64_t l = 0, h = n;  // first index with keys[index] >= key
        while (l < h) {
            const int64_t m = (l + h) >> 1;
            if (keys[m] < key) l = m + 1; else h = m;
        }
        if (l < n) assign[l] = uint8_t(v >> 24);
    }
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
    for (int j = k; j < 2 * kSumStride; j += blockDim.x) gp(J.sums)[j] = 0;
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

// Caller-supplied colours (cq_kmeans): every key must be a 24-bit colour and
// the counts must sum to at most 2^28 (the pixels of the largest image), so
// that a count fits the 28 bits a pruned run's packed record gives it and the
// cluster sums stay exact.  Block b of job j checks the colours
// [b chunk, (b + 1) chunk), flags a key outside the range (bad_input bit 2)
// and adds its counts to total_w; k_check_finish flags a total above 2^28
// (bit 4) and stops a job with any flag before its first iteration.
constexpr uint64_t kMaxTotalWeight = uint64_t(1) << 28;

__global__ void __launch_bounds__(kAssignThreads) k_check_colours(const JobDev* __restrict__ jobs,
                                                                  const int* __restrict__ map, int B)
{
    __shared__ unsigned long long red[kAssignThreads / 64];
    const int jb = find_job(map, B, blockIdx.x);
    const JobDev& J = jobs[jb];
    const int lb = blockIdx.x - map[jb];
    const int64_t lo = int64_t(lb) * J.chunk;
    const int64_t hi = lo + J.chunk < J.n ? lo + J.chunk : J.n;
    const uint32_t* __restrict__ keys = gp(J.keys);
    const uint32_t* __restrict__ counts = gp(J.counts);
    unsigned long long sum = 0;
    bool bad = false;
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
        bad = bad || keys[i] >= kNumKeys;
        sum += counts[i];
    }
    sum = wave_sum(sum);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sum;
    Meta* __restrict__ meta = gp(J.meta);
    if (__syncthreads_or(bad ? 1 : 0) && threadIdx.x == 0) atomicOr(&meta->bad_input, 2);
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < kAssignThreads / 64; ++w) t += red[w];
        atomicAdd(reinterpret_cast<unsigned long long*>(&meta->total_w), t);
    }
}

__global__ void k_check_finish(const JobDev* __restrict__ jobs)
{
    Meta* __restrict__ meta = gp(jobs[blockIdx.x].meta);
    if (threadIdx.x != 0) return;
    int bad = meta->bad_input;
    if (meta->total_w > kMaxTotalWeight) bad |= 4;
    meta->bad_input = bad;
    meta->total_w = 0;
    if (bad) meta->done = 1;
}

cq_status launch_check_colours(const JobDev* jobs, const int* maps, int B, int blocks, hipStream_t s)
{
    if (blocks > 0)
        CQ_TIMED_LAUNCH("k_check_colours", s, k_check_colours<<<blocks, kAssignThreads, 0, s>>>(jobs, maps + kMapAssign * (B + 1), B));
    CQ_TIMED_LAUNCH("k_check_finish", s, k_check_finish<<<B, 64, 0, s>>>(jobs));
    return CQ_OK;
}

// ------------------------------------------------------------------ host
cq_status launch_kmeans_begin(const JobDev* jobs, int B, hipStream_t s)
{
    CQ_TIMED_LAUNCH("k_kmeans_begin", s, k_kmeans_begin<<<B, kMaxK, 0, s>>>(jobs));
    return CQ_OK;
}

// One iteration of every job that has not stopped.  The first iteration is
// a full search for every job; later ones search fully for the unpruned jobs
// and walk the sorted table for the pruned ones.
cq_status launch_kmeans_iter(const JobDev* jobs, const int* maps, int B, bool first, int all_blocks,
                             int full_blocks, int walk_blocks, int update_blocks, bool regroup,
                             int table_blocks, hipStream_t s)
{
    if (first) {
        CQ_TIMED_LAUNCH("k_assign_full", s, k_assign<false><<<all_blocks, kAssignThreads, 0, s>>>(jobs, maps + kMapAssign * (B + 1), B));
    } else {
        if (full_blocks > 0)
            CQ_TIMED_LAUNCH("k_assign_full", s, k_assign<false><<<full_blocks, kAssignThreads, 0, s>>>(jobs, maps + kMapAssignFull * (B + 1), B));
        if (walk_blocks > 0)
            CQ_TIMED_LAUNCH("k_assign_walk", s, k_assign<true><<<walk_blocks, kAssignThreads, 0, s>>>(jobs, maps + kMapAssignWalk * (B + 1), B));
    }
    if (regroup)
        CQ_TIMED_LAUNCH("k_update", s, k_update<<<update_blocks, kMaxK, 0, s>>>(jobs, maps + kMapUpdate * (B + 1), B));
    else
        CQ_TIMED_LAUNCH("k_update", s, k_update<<<table_blocks, kMaxK, 0, s>>>(jobs, maps + kMapUpdateTable * (B + 1), B));
    return CQ_OK;
}

cq_status launch_unpermute(const JobDev* jobs, const int* maps, int B, int blocks, hipStream_t s)
{
    CQ_TIMED_LAUNCH("k_unpermute", s, k_unpermute<<<blocks, kAssignThreads, 0, s>>>(jobs, maps + kMapAssign * (B + 1), B));
    return CQ_OK;
}

// Regrouping blocks of a job: one per assignment block's worth of records.
int64_t regroup_blocks(int64_t n, int64_t chunk) { return (n + chunk - 1) / chunk; }

// Update blocks of a job before its regrouping blocks.
int update_table_blocks(int K, int prune) { return table_blocks_of(K, prune); }


cq_status launch_palette(const JobDev* jobs, int B, hipStream_t s)
{
    CQ_TIMED_LAUNCH("k_palette", s, k_palette<<<B, 3 * kMaxK, 0, s>>>(jobs));
    return CQ_OK;
}

// ------------------------------------------------------------ schedules
// The launch schedule of the iterations: colours per assignment block and
// the regrouping period, by the number of colours one call iterates over.
// Results never depend on it; only the speed does.  The built-in table is
// the one the autotuner measured (paper_1101_0395_amd/autotune.py).
namespace {
constexpr int kMaxSchedules = 32;
const cq_schedule kDefaultSchedule[] = {
    {0, 1024, 1},
    {4149731, 2048, 2},
    {34861447, 8192, 2},
};
struct ScheduleTable {
    std::mutex mu;
    cq_schedule e[kMaxSchedules];
    int n = 0;
};
ScheduleTable& schedules()
{
    static ScheduleTable* t = [] {
        ScheduleTable* x = new ScheduleTable;
        x->n = int(sizeof kDefaultSchedule / sizeof kDefaultSchedule[0]);
        for (int i = 0; i < x->n; ++i) x->e[i] = kDefaultSchedule[i];
        return x;
    }();
    return *t;
}
}  // namespace

cq_schedule schedule_for(int64_t colours)
{
    ScheduleTable& t = schedules();
    std::lock_guard<std::mutex> lock(t.mu);
    cq_schedule s = t.e[0];
    for (int i = 1; i < t.n; ++i)
        if (colours >= t.e[i].min_colours) s = t.e[i];
    return s;
}

cq_status set_schedule(const cq_schedule* table, int32_t n)
{
    if (n < 0 || n > kMaxSchedules) return einval("n = %d outside [0, %d]", n, kMaxSchedules);
    if (n > 0 && !table) return einval("table is null");
    for (int32_t i = 0; i < n; ++i) {
        const cq_schedule& x = table[i];
        if (i == 0 ? x.min_colours != 0 : x.min_colours <= table[i - 1].min_colours)
            return einval("entry %d: min_colours must start at 0 and increase", i);
        if (x.assign_chunk < kAssignThreads || x.assign_chunk > kMaxAssignChunk || x.assign_chunk % kAssignThreads)
            return einval("entry %d: assign_chunk %d is not a multiple of %d in [%d, %d]", i, x.assign_chunk,
                          kAssignThreads, kAssignThreads, kMaxAssignChunk);
        if (x.regroup_period < 1 || x.regroup_period > kMaxIters)
            return einval("entry %d: regroup_period %d outside [1, %d]", i, x.regroup_period, kMaxIters);
    }
    ScheduleTable& t = schedules();
    std::lock_guard<std::mutex> lock(t.mu);
    if (n == 0) {
        t.n = int(sizeof kDefaultSchedule / sizeof kDefaultSchedule[0]);
        for (int i = 0; i < t.n; ++i) t.e[i] = kDefaultSchedule[i];
    } else {
        t.n = n;
        for (int i = 0; i < n; ++i) t.e[i] = table[i];
    }
    return CQ_OK;
}

cq_status get_schedule(cq_schedule* table, int32_t capacity, int32_t* n)
{
    if (!n) return einval("n is null");
    ScheduleTable& t = schedules();
    std::lock_guard<std::mutex> lock(t.mu);
    *n = t.n;
    if (capacity < 0) return einval("capacity is negative");
    if (capacity > 0 && !table) return einval("table is null");
    for (int i = 0; i < t.n && i < capacity; ++i) table[i] = t.e[i];
    return CQ_OK;
}

// Colours per assignment / colour-table block of a job of n colours under
// the schedule's chunk: at least enough that the job needs at most
// kMaxAssignBlocks blocks, a multiple of the block size, at most
// kMaxAssignChunk (the per-block counters of (cluster, bucket) pairs are
// 16 bits wide).
int64_t assign_chunk(int64_t n, int32_t scheduled)
{
    int64_t chunk = scheduled;
    if ((n + chunk - 1) / chunk > kMaxAssignBlocks) chunk = (n + kMaxAssignBlocks - 1) / kMaxAssignBlocks;
    chunk = (chunk + kAssignThreads - 1) / kAssignThreads * kAssignThreads;
    return chunk < kMaxAssignChunk ? chunk : kMaxAssignChunk;
}


}  // namespace cq
