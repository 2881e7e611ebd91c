// WU initialization (the initializer of WSM-WU, Section 3.3): Wu's greedy
// orthogonal bipartitioning of the colour space (X. Wu, "Efficient
// statistical computations for optimal color quantization", Graphics Gems II,
// 1991).
//
// Each channel is cut into 32 levels (value >> 3).  A box is an inclusive
// range of levels per channel; the statistics of a box are five exact
// integers: pixels w, channel sums sr, sg, sb, and s2 = the sum of
// r^2 + g^2 + b^2.  Starting from the whole grid, the box of largest weighted
// variance s2 - |m|^2 / w (ties to the lowest box index; a box of one cell, or
// one found to have no allowed cut, counts 0, and so does a value below zero by
// rounding) is split at the plane that maximizes |m_l|^2 / w_l + |m_u|^2 / w_u
// over its two non-empty parts (first plane of a channel, then the channel,
// R before G before B, on ties); the lower part keeps the box's index and the
// upper part becomes the next box.  This ends at K boxes or when every
// variance is 0.  The centres are the boxes' means; if fewer than K boxes
// result, the remaining centres repeat the first box's mean.  The criteria
// are FP64 with the operations in a fixed order and no contraction.
//
// Kernels (every launch covers all jobs; jobs of other schemes return):
//   k_wu_clear    the job's table of 5 x 33^3 uint64 (a zero border at index
//                 0 of each axis, cell c at index c + 1) cleared;
//   k_wu_accum    per block of colours: each colour's count, sums and s2 added
//                 to its cell (summed over runs of one cell in a wave first);
//   k_wu_prefix   three launches: cumulative sums along b, then g, then r,
//                 so that entry (r, g, b) holds the statistics of the cells
//                 below it on every axis and a box's statistics are an
//                 8-corner inclusion-exclusion;
//   k_wu_split    per job, one wave: the greedy splitting, the centres.
#include "cq_internal.h"

#pragma clang fp contract(off)

namespace cq {

constexpr int kWuSide = 33;
constexpr int kWuPlane = kWuSide * kWuSide * kWuSide;  // entries of one statistic
constexpr int kWuStats = 5;                             // w, sr, sg, sb, s2
constexpr int kWuClearThreads = 256;
constexpr int kWuClearBlocks = (kWuStats * kWuPlane + kWuClearThreads * 16 - 1) / (kWuClearThreads * 16);
constexpr int kWuAccumThreads = 256;
constexpr int kWuColoursPerBlock = 4096;

static_assert(sizeof(uint64_t) * kWuStats * kWuPlane <= kWuTableBytes, "WU table region");

__device__ __forceinline__ bool wu_job(const JobDev& J) { return J.scheme == CQ_INIT_WU && J.n > J.K; }

__device__ __forceinline__ uint64_t* wu_table(const JobDev& J) { return reinterpret_cast<uint64_t*>(gp(J.d2)); }

__device__ __forceinline__ int wu_at(int r, int g, int b) { return (r * kWuSide + g) * kWuSide + b; }

__global__ void __launch_bounds__(kWuClearThreads) k_wu_clear(const JobDev* __restrict__ jobs)
{
    const JobDev& J = jobs[blockIdx.x / kWuClearBlocks];
    if (!wu_job(J)) return;
    uint64_t* __restrict__ t = wu_table(J);
    const int base = (blockIdx.x % kWuClearBlocks) * kWuClearThreads * 16;
    for (int u = 0; u < 16; ++u) {
        const int i = base + u * kWuClearThreads + threadIdx.x;
        if (i < kWuStats * kWuPlane) t[i] = 0ull;
    }
}

__global__ void __launch_bounds__(kWuAccumThreads) k_wu_accum(const JobDev* __restrict__ jobs,
                                                              const int* __restrict__ map, int B)
{
    const int jb = find_job(map, B, blockIdx.x);
    const JobDev& J = jobs[jb];
    const int64_t lo = int64_t(blockIdx.x - map[jb]) * kWuColoursPerBlock;
    const int64_t hi = lo + kWuColoursPerBlock < J.n ? lo + kWuColoursPerBlock : J.n;
    const uint32_t* __restrict__ keys = gp(J.keys);
    const uint32_t* __restrict__ counts = gp(J.counts);
    unsigned long long* __restrict__ t = reinterpret_cast<unsigned long long*>(wu_table(J));
    const int lane = threadIdx.x & 63;
    // the colours of a wave are consecutive in key order, so lanes of the same
    // cell mostly sit next to each other: each run of equal cells is summed in
    // the wave and added once, by its last lane
    for (int64_t i0 = lo; i0 < hi; i0 += kWuAccumThreads) {
        const int64_t i = i0 + threadIdx.x;
        const bool valid = i < hi;
        int r = 0, g = 0, b = 0;
        uint64_t w = 0;
        int c = -1;
        if (valid) {
            key_rgb(keys[i], r, g, b);
            w = counts[i];
            c = wu_at((r >> 3) + 1, (g >> 3) + 1, (b >> 3) + 1);
        }
        const uint64_t v[kWuStats] = {w, w * uint64_t(r), w * uint64_t(g), w * uint64_t(b),
                                      w * uint64_t(r * r + g * g + b * b)};
        const int c_prev = __shfl(c, lane > 0 ? lane - 1 : 0, 64);
        const int c_next = __shfl(c, lane < 63 ? lane + 1 : 63, 64);
        const bool head = lane == 0 || c_prev != c;
        const bool tail = lane == 63 || c_next != c;
        const int head_lane = wave_incl_max(head ? lane : 0);  // the first lane of this lane's run
#pragma unroll
        for (int q = 0; q < kWuStats; ++q) {
            const uint64_t incl = wave_incl_scan(v[q]);
            const uint64_t before = __shfl(incl - v[q], head_lane, 64);  // the scan just before the run
            if (valid && tail) atomicAdd(t + q * kWuPlane + c, (unsigned long long)(incl - before));
        }
    }
}

// Cumulative sums along one axis (0: b, 1: g, 2: r), one line (a statistic
// and the two other indices) per thread; the whole line is loaded before
// anything is stored.  Three launches, one per axis, each over every job.
constexpr int kWuLines = kWuStats * kWuSide * kWuSide;
constexpr int kWuPrefixThreads = 256;
constexpr int kWuPrefixBlocks = (kWuLines + kWuPrefixThreads - 1) / kWuPrefixThreads;

template <int kAxis>
__global__ void __launch_bounds__(kWuPrefixThreads) k_wu_prefix(const JobDev* __restrict__ jobs)
{
    const JobDev& J = jobs[blockIdx.x / kWuPrefixBlocks];
    if (!wu_job(J)) return;
    const int l = (blockIdx.x % kWuPrefixBlocks) * kWuPrefixThreads + threadIdx.x;
    if (l >= kWuLines) return;
    const int q = l / (kWuSide * kWuSide), rest = l - q * kWuSide * kWuSide;
    const int u = rest / kWuSide, v = rest % kWuSide;
    constexpr int step = kAxis == 0 ? 1 : (kAxis == 1 ? kWuSide : kWuSide * kWuSide);
    const int first = kAxis == 0 ? wu_at(u, v, 0) : (kAxis == 1 ? wu_at(u, 0, v) : wu_at(0, u, v));
    uint64_t* __restrict__ p = wu_table(J) + q * kWuPlane + first;
    uint64_t x[kWuSide - 1];
#pragma unroll
    for (int i = 1; i < kWuSide; ++i) x[i - 1] = p[i * step];
    uint64_t acc = 0;
#pragma unroll
    for (int i = 1; i < kWuSide; ++i) {
        acc += x[i - 1];
        p[i * step] = acc;
    }
}

struct WuMom {
    uint64_t m[kWuStats];
};

// Statistics of the box of cells [lo, hi] (inclusive, per channel).
__device__ __forceinline__ WuMom wu_box(const uint64_t* __restrict__ t, const int lo[3], const int hi[3])
{
    const int r0 = lo[0], r1 = hi[0] + 1, g0 = lo[1], g1 = hi[1] + 1, b0 = lo[2], b1 = hi[2] + 1;
    const int c[8] = {wu_at(r1, g1, b1), wu_at(r0, g1, b1), wu_at(r1, g0, b1), wu_at(r1, g1, b0),
                      wu_at(r0, g0, b1), wu_at(r0, g1, b0), wu_at(r1, g0, b0), wu_at(r0, g0, b0)};
    uint64_t v[kWuStats][8];
#pragma unroll
    for (int q = 0; q < kWuStats; ++q)
#pragma unroll
        for (int k = 0; k < 8; ++k) v[q][k] = t[q * kWuPlane + c[k]];
    WuMom m;
#pragma unroll
    for (int q = 0; q < kWuStats; ++q)
        m.m[q] = v[q][0] - v[q][1] - v[q][2] - v[q][3] + v[q][4] + v[q][5] + v[q][6] - v[q][7];
    return m;
}

// |m|^2 / w as ((sr^2 + sg^2) + sb^2) / w.
__device__ __forceinline__ double wu_spread(const WuMom& a)
{
    const double r = double(a.m[1]), g = double(a.m[2]), b = double(a.m[3]);
    return (r * r + g * g + b * b) / double(a.m[0]);
}

__device__ __forceinline__ double wu_var(const int lo[3], const int hi[3], const WuMom& a)
{
    const int vol = (hi[0] - lo[0] + 1) * (hi[1] - lo[1] + 1) * (hi[2] - lo[2] + 1);
    if (vol <= 1 || a.m[0] == 0) return 0.0;
    const double v = double(a.m[4]) - wu_spread(a);
    return v > 0.0 ? v : 0.0;
}

// The greedy splitting, one wave per job.  Candidate planes are numbered
// ci = 32 a + (t - lo_a) for channel a and plane t in [lo_a, hi_a - 1] (the
// lower part ends at t); lane l evaluates ci = l (channels R and G) and
// ci = 64 + l (channel B, lanes 0-31).  Among the allowed cuts the largest
// value wins, then the smallest ci, which is the first plane of the lowest
// channel.  Values of allowed cuts are positive, so they order as their bit
// patterns, and a largest value of 0 means no allowed cut.
__global__ void __launch_bounds__(64) k_wu_split(const JobDev* __restrict__ jobs)
{
    __shared__ int s_lo[kMaxK][3], s_hi[kMaxK][3];
    __shared__ uint64_t s_m[kMaxK][kWuStats];
    __shared__ double s_var[kMaxK];
    const JobDev& J = jobs[blockIdx.x];
    if (!wu_job(J)) return;
    const uint64_t* __restrict__ t = wu_table(J);
    const int lane = threadIdx.x;
    const int K = J.K;
    if (lane == 0) {
        for (int a = 0; a < 3; ++a) {
            s_lo[0][a] = 0;
            s_hi[0][a] = 31;
        }
        const WuMom all = wu_box(t, s_lo[0], s_hi[0]);
        for (int q = 0; q < kWuStats; ++q) s_m[0][q] = all.m[q];
        s_var[0] = wu_var(s_lo[0], s_hi[0], all);
    }
    __syncthreads();
    int nb = 1;
    while (nb < K) {
        // the box to split: largest variance, lowest index on ties (variances
        // are never negative, so they order as their bit patterns); each lane
        // keeps the first largest of its boxes k = lane, lane + 64, ...
        constexpr uint32_t kNone = 0xffffffffu;
        uint64_t vb = 0;
        uint32_t vi = kNone;
        for (int k = lane; k < nb; k += 64) {
            const uint64_t bits = __builtin_bit_cast(uint64_t, s_var[k]);
            if (vi == kNone || bits > vb) {
                vb = bits;
                vi = uint32_t(k);
            }
        }
        const uint64_t vmax = wave_max(vb);
        if (vmax == 0) break;  // every variance is 0
        // the lowest index among the lanes holding the largest variance
        const uint32_t next = kNone - wave_max(vi != kNone && vb == vmax ? kNone - vi : 0u);
        int lo[3], hi[3];
        for (int a = 0; a < 3; ++a) {
            lo[a] = s_lo[next][a];
            hi[a] = s_hi[next][a];
        }
        WuMom whole;
        for (int q = 0; q < kWuStats; ++q) whole.m[q] = s_m[next][q];
        // this lane's two candidates
        WuMom low[2];
        uint64_t val[2];
        for (int p = 0; p < 2; ++p) {
            const int a = p == 0 ? (lane >> 5) : 2;
            const int cut = lo[a] + (lane & 31);
            val[p] = 0;
            for (int q = 0; q < kWuStats; ++q) low[p].m[q] = 0;
            if ((p == 1 && lane >= 32) || cut >= hi[a]) continue;
            int h2[3] = {hi[0], hi[1], hi[2]};
            h2[a] = cut;
            low[p] = wu_box(t, lo, h2);
            WuMom up;
            for (int q = 0; q < kWuStats; ++q) up.m[q] = whole.m[q] - low[p].m[q];
            if (low[p].m[0] == 0 || up.m[0] == 0) continue;
            val[p] = __builtin_bit_cast(uint64_t, wu_spread(low[p]) + wu_spread(up));
        }
        const int mine = val[1] > val[0] ? 1 : 0;  // ci = 64 + lane beats ci = lane only if strictly larger
        const uint64_t cmax = wave_max(val[mine]);
        if (cmax == 0) {  // no allowed cut: never try this box again
            if (lane == 0) s_var[next] = 0.0;
            __syncthreads();
            continue;
        }
        const uint32_t my_ci = uint32_t(mine * 64 + lane);
        const uint32_t ci = 0xffffffffu - wave_max(val[mine] == cmax ? 0xffffffffu - my_ci : 0u);
        const int src = int(ci & 63), pass = int(ci >> 6);
        const int axis = pass == 1 ? 2 : (src >> 5);
        const int cut = lo[axis] + (src & 31);
        WuMom lw;
        for (int q = 0; q < kWuStats; ++q) lw.m[q] = read_lane(pass == 1 ? low[1].m[q] : low[0].m[q], src);
        if (lane == 0) {
            WuMom up;
            for (int q = 0; q < kWuStats; ++q) up.m[q] = whole.m[q] - lw.m[q];
            for (int a = 0; a < 3; ++a) {
                s_lo[nb][a] = lo[a];
                s_hi[nb][a] = hi[a];
            }
            s_lo[nb][axis] = cut + 1;
            s_hi[next][axis] = cut;
            for (int q = 0; q < kWuStats; ++q) {
                s_m[next][q] = lw.m[q];
                s_m[nb][q] = up.m[q];
            }
            s_var[next] = wu_var(s_lo[next], s_hi[next], lw);
            s_var[nb] = wu_var(s_lo[nb], s_hi[nb], up);
        }
        ++nb;
        __syncthreads();
    }
    double* __restrict__ centers = gp(J.centers);
    for (int k = lane; k < K; k += 64) {
        const int src = k < nb ? k : 0;
        const double w = double(s_m[src][0]);
        for (int c = 0; c < 3; ++c) centers[3 * k + c] = double(s_m[src][1 + c]) / w;
    }
}

// ------------------------------------------------------------------ host
int wu_accum_blocks(int64_t n) { return int((n + kWuColoursPerBlock - 1) / kWuColoursPerBlock); }

cq_status launch_wu(const JobDev* jobs, const int* maps, int B, int accum_blocks, hipStream_t s)
{
    CQ_TIMED_LAUNCH("k_wu_clear", s, k_wu_clear<<<B * kWuClearBlocks, kWuClearThreads, 0, s>>>(jobs));
    CQ_TIMED_LAUNCH("k_wu_accum", s,
                    k_wu_accum<<<accum_blocks, kWuAccumThreads, 0, s>>>(jobs, maps + kMapWu * (B + 1), B));
    CQ_TIMED_LAUNCH("k_wu_prefix", s, k_wu_prefix<0><<<B * kWuPrefixBlocks, kWuPrefixThreads, 0, s>>>(jobs));
    CQ_TIMED_LAUNCH("k_wu_prefix", s, k_wu_prefix<1><<<B * kWuPrefixBlocks, kWuPrefixThreads, 0, s>>>(jobs));
    CQ_TIMED_LAUNCH("k_wu_prefix", s, k_wu_prefix<2><<<B * kWuPrefixBlocks, kWuPrefixThreads, 0, s>>>(jobs));
    CQ_TIMED_LAUNCH("k_wu_split", s, k_wu_split<<<B, 64, 0, s>>>(jobs));
    return CQ_OK;
}

}  // namespace cq
