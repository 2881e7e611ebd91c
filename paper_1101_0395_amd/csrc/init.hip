// Initialization schemes of Section 2.3 on the N' unique colours: Forgy (FGY),
// farthest-first / max-min (MMX) and k-means++ (KPP, weighted by pixel count).
//
// Every chosen centre is a colour, so D^2 (squared distance to the nearest
// chosen centre) is an exact integer and the sampling weights n_i D_i^2 are
// exact uint64 values.  MMX and KPP run as one cooperative launch with a grid
// barrier per round (below); FGY is a single wave.  The draw order is the one
// documented for cq_init in cq.h.
#include <stdlib.h>

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

// FGY: partial Fisher-Yates over positions [0, N').  Position j swaps with
// r_j = j + U(N' - j); the values held by displaced positions are kept in a
// small map searched by one wave.
__global__ void __launch_bounds__(64) k_forgy(const JobDev* __restrict__ jobs)
{
    const JobDev& J = jobs[blockIdx.x];
    if (J.scheme != CQ_INIT_FORGY || J.n <= J.K) return;
    const uint32_t* __restrict__ keys = gp(J.keys);
    const int64_t n = J.n;
    const int K = J.K;
    Meta* __restrict__ meta = gp(J.meta);
    double* __restrict__ centers = gp(J.centers);
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

// Per job: seed the stream and reset the team barrier; for N' <= K the
// centres are the colours followed by zeros (whatever the scheme).
__global__ void __launch_bounds__(kMaxK) k_init_begin(const JobDev* __restrict__ jobs)
{
    const JobDev& J = jobs[blockIdx.x];
    const int k = threadIdx.x;
    if (k == 0) {
        gp(J.meta)->rng = J.seed;
        gp(J.meta)->barrier = 0;
        gp(J.meta)->sync_error = 0;
        gp(J.meta)->pick_epoch = 0;
    }
    if (J.n > J.K || k >= J.K) return;
    if (k < J.n) {
        write_center(J.centers, k, gp(J.keys)[k]);
    } else {
        gp(J.centers)[3 * k] = gp(J.centers)[3 * k + 1] = gp(J.centers)[3 * k + 2] = 0.0;
    }
}

// ------------------------------------------------------------------------
// Cooperative MMX / KPP: one launch runs all K rounds of every job, each job
// with its own team of blocks.  Block b of a team owns the colours
// [b C, (b+1) C).  Round j:
//   1. every block lowers D^2 of its colours with the colour picked in round
//      j-1 and publishes one value for its chunk: the sum of n D^2 (KPP; the
//      counts alone in round 0) or the packed arg-max of (D^2, -index) (MMX);
//   2. team barrier;
//   3. every block reads the team's chunk values.  MMX: the largest packed
//      value names the colour.  KPP: every block draws r = U(total) from its
//      own copy of the splitmix64 stream and finds the chunk holding r; the
//      block owning that chunk finds the colour inside its own chunk and
//      publishes it with a release flag, which the other blocks wait for.
// Chunk values and published picks are double-buffered by round parity, so a
// block never rewrites what another block may still be reading.
constexpr int kCoopThreads = 256;
constexpr int kCoopMaxSegs = 4;    // up to 1024 blocks per team
constexpr int kCoopLdsCap = 4096;  // colours per block kept in LDS (48 KiB)
constexpr int kRun = kCoopLdsCap / kCoopThreads;  // colours per thread per pass of a chunk search

// kLds: the block's colours (key, count, D^2) stay in LDS for all rounds;
// otherwise they are streamed from global memory every round (D^2 in d2buf).
template <bool kLds>
__global__ void __launch_bounds__(kCoopThreads) k_init_coop(const JobDev* __restrict__ jobs,
                                                            const int* __restrict__ map, int B)
{
    __shared__ uint64_t tmp[64];
    __shared__ uint64_t s_r;
    __shared__ int s_chunk;
    __shared__ uint64_t s_before;
    __shared__ int64_t s_pick;
    __shared__ uint32_t lkey[kLds ? kCoopLdsCap : 1];
    __shared__ uint32_t lcnt[kLds ? kCoopLdsCap : 1];
    __shared__ uint32_t ld2[kLds ? kCoopLdsCap : 1];
    const int jb = find_job(map, B, blockIdx.x);
    const JobDev& J = jobs[jb];
    const int G = J.init_blocks;  // team size, <= kCoopMaxSegs * kCoopThreads
    const int tb = blockIdx.x - map[jb];
    const uint32_t* __restrict__ keys = gp(J.keys);
    const uint32_t* __restrict__ counts = gp(J.counts);
    const int64_t n = J.n;
    const int K = J.K;
    const int kpp = J.scheme == CQ_INIT_KMEANSPP;
    const int64_t C = J.init_C;
    uint32_t* __restrict__ d2own = gp(J.d2);
    uint64_t* __restrict__ vals = gp(J.vals);
    Meta* __restrict__ meta = gp(J.meta);
    double* __restrict__ centers = gp(J.centers);
    const int64_t lo = int64_t(tb) * C;
    const int64_t hi = lo + C < n ? lo + C : n;
    const int mine_n = hi > lo ? int(hi - lo) : 0;
    const int nseg = (G + kCoopThreads - 1) / kCoopThreads;
    if (kLds) {
        // all loads issued before the stores (mine_n <= kCoopLdsCap)
        uint32_t kk[kRun], cc[kRun];
#pragma unroll
        for (int r = 0; r < kRun; ++r) {
            const int q = r * kCoopThreads + threadIdx.x;
            kk[r] = q < mine_n ? keys[lo + q] : 0u;
            cc[r] = q < mine_n ? counts[lo + q] : 0u;
        }
#pragma unroll
        for (int r = 0; r < kRun; ++r) {
            const int q = r * kCoopThreads + threadIdx.x;
            if (q < mine_n) {
                lkey[q] = kk[r];
                lcnt[q] = cc[r];
                ld2[q] = 0xFFFFFFFFu;
            }
        }
    }
    uint64_t rng = J.seed;  // the stream lives in thread 0 of every block
    int64_t pick = -1;
    int cr = 0, cg = 0, cb = 0;
    for (int j = 0; j < K; ++j) {
        __syncthreads();  // the previous round's readers of tmp and s_* are done
        const int par = j & 1;
        // 1. own chunk
        uint64_t acc = 0;
        if (j > 0 || kpp) {
            // four colours per thread per step, loads first
            for (int q0 = threadIdx.x; q0 < mine_n; q0 += 4 * kCoopThreads) {
                uint32_t kq[4], cq[4], oq[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int q = q0 + u * kCoopThreads;
                    const int64_t i = lo + q;
                    const bool in = q < mine_n;
                    kq[u] = in ? (kLds ? lkey[q] : keys[i]) : 0u;
                    cq[u] = in ? (kLds ? lcnt[q] : counts[i]) : 0u;
                    oq[u] = (in && j > 1) ? (kLds ? ld2[q] : d2own[i]) : 0xFFFFFFFFu;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int q = q0 + u * kCoopThreads;
                    if (q >= mine_n) continue;
                    const int64_t i = lo + q;
                    if (j == 0) {
                        acc += cq[u];
                        continue;
                    }
                    int r, g, b;
                    key_rgb(kq[u], r, g, b);
                    const uint32_t d = dist_u32(r, g, b, cr, cg, cb);
                    const uint32_t m = oq[u] < d ? oq[u] : d;
                    if (kLds)
                        ld2[q] = m;
                    else
                        d2own[i] = m;
                    if (kpp) {
                        acc += uint64_t(cq[u]) * m;
                    } else {
                        const uint64_t packed = (uint64_t(m) << 32) | uint64_t(0xFFFFFFFFu - uint32_t(i));
                        acc = packed > acc ? packed : acc;
                    }
                }
            }
            acc = kpp ? wave_sum(acc) : wave_max(acc);
            if ((threadIdx.x & 63) == 0) tmp[threadIdx.x >> 6] = acc;
            __syncthreads();
            if (threadIdx.x == 0) {
                uint64_t v = tmp[0];
                for (int w = 1; w < kCoopThreads / 64; ++w)
                    v = kpp ? v + tmp[w] : (tmp[w] > v ? tmp[w] : v);
                vals[int64_t(par) * G + tb] = v;
            }
        }
        // 2. everyone has published
        if (!grid_barrier(&meta->barrier, uint32_t(j + 1) * uint32_t(G), &meta->sync_error)) return;
        const uint64_t* v_now = vals + int64_t(par) * G;
        // 3. the same pick in every block
        if (!kpp) {
            if (j == 0) {
                if (threadIdx.x == 0) s_pick = int64_t(uniform_below(rng, uint64_t(n)));
                __syncthreads();
                pick = s_pick;
            } else {
                uint64_t best = 0;
                for (int c = threadIdx.x; c < G; c += kCoopThreads) best = v_now[c] > best ? v_now[c] : best;
                best = wave_max(best);
                if ((threadIdx.x & 63) == 0) tmp[threadIdx.x >> 6] = best;
                __syncthreads();
                for (int w = 0; w < kCoopThreads / 64; ++w) best = tmp[w] > best ? tmp[w] : best;
                pick = int64_t(0xFFFFFFFFu - uint32_t(best & 0xFFFFFFFFull));
                if (pick >= n) pick = 0;  // unreachable: every colour packs a non-zero value
            }
        } else {
            // exclusive prefix of the chunk values, one segment of 256 blocks at a time
            uint64_t ex[kCoopMaxSegs], vv[kCoopMaxSegs];
            uint64_t carry = 0;
#pragma unroll
            for (int q = 0; q < kCoopMaxSegs; ++q) {
                ex[q] = vv[q] = 0;
                if (q >= nseg) continue;
                const int c = q * kCoopThreads + threadIdx.x;
                const uint64_t v = c < G ? v_now[c] : 0;
                uint64_t tot = 0;
                const uint64_t e = block_exclusive_scan<uint64_t>(v, tmp, &tot);
                ex[q] = carry + e;
                vv[q] = v;
                carry += tot;
            }
            if (threadIdx.x == 0) {
                s_r = carry ? uniform_below(rng, carry) : 0;
                s_chunk = -1;
            }
            __syncthreads();
            const uint64_t r = s_r;
#pragma unroll
            for (int q = 0; q < kCoopMaxSegs; ++q) {
                if (vv[q] != 0 && ex[q] <= r && r < ex[q] + vv[q]) {
                    s_chunk = q * kCoopThreads + threadIdx.x;
                    s_before = ex[q];
                }
            }
            __syncthreads();
            int c = s_chunk;
            const uint64_t rr = c >= 0 ? r - s_before : 0;
            if (c < 0) c = 0;  // unreachable: the chunk values sum to carry > 0
            if (c == tb) {
                // the owner finds the colour in its own chunk: each thread takes
                // a run of kRun consecutive colours per pass, loads first
                if (threadIdx.x == 0) s_pick = -1;
                uint64_t before = 0;
                for (int pbase = 0; pbase < mine_n; pbase += kCoopThreads * kRun) {
                    const int tlo = pbase + threadIdx.x * kRun;
                    uint32_t cq[kRun], dq[kRun];
#pragma unroll
                    for (int q = 0; q < kRun; ++q) {
                        const int qq = tlo + q;
                        const bool in = qq < mine_n;
                        cq[q] = in ? (kLds ? lcnt[qq] : counts[lo + qq]) : 0u;
                        dq[q] = (in && j > 0) ? (kLds ? ld2[qq] : d2own[lo + qq]) : 1u;
                    }
                    uint64_t mine = 0;
#pragma unroll
                    for (int q = 0; q < kRun; ++q) mine += uint64_t(cq[q]) * dq[q];
                    uint64_t tot = 0;
                    const uint64_t off = before + block_exclusive_scan<uint64_t>(mine, tmp, &tot);
                    if (mine != 0 && off <= rr && rr < off + mine) {
                        uint64_t acc2 = off;
#pragma unroll
                        for (int q = 0; q < kRun; ++q) {
                            acc2 += uint64_t(cq[q]) * dq[q];
                            if (acc2 > rr) {
                                s_pick = lo + tlo + q;
                                break;
                            }
                        }
                    }
                    before += tot;
                }
                __syncthreads();
                if (threadIdx.x == 0) {
                    int64_t pk = s_pick;
                    if (pk < 0) pk = lo;  // unreachable when the weights are consistent
                    meta->pick_slot[par] = pk;
                    __hip_atomic_store(&meta->pick_epoch, uint32_t(j + 1), __ATOMIC_RELEASE,
                                       __HIP_MEMORY_SCOPE_AGENT);
                    s_pick = pk;
                }
                __syncthreads();
                pick = s_pick;
            } else {
                if (!wait_flag(&meta->pick_epoch, uint32_t(j + 1), &meta->sync_error)) return;
                pick = __hip_atomic_load(&meta->pick_slot[par], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        const uint32_t pick_key = keys[pick];
        if (threadIdx.x == 0 && tb == 0) {
            write_center(centers, j, pick_key);
            if (j == K - 1) meta->rng = rng;
        }
        key_rgb(pick_key, cr, cg, cb);
    }
}

// ------------------------------------------------------------------ host
// Co-resident blocks of k_init_coop<true> on this device (0: no cooperative launch).
int coop_capacity()
{
    static int max_coop = -1;
    if (max_coop < 0) {
        int dev = 0, cus = 0, per_cu = 0, coop_ok = 0;
        max_coop = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&coop_ok, hipDeviceAttributeCooperativeLaunch, dev) == hipSuccess &&
            coop_ok &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &per_cu, reinterpret_cast<const void*>(k_init_coop<true>), kCoopThreads, 0) == hipSuccess)
            max_coop = cus * per_cu;
    }
    return max_coop;
}

// Preferred team size for a job of n colours (before the whole-launch cap).
int coop_team_blocks(int64_t n)
{
    static int override_blocks = -1;
    if (override_blocks < 0) {
        const char* env = getenv("CQ_INIT_BLOCKS");
        override_blocks = env ? atoi(env) : 0;
    }
    int64_t g = override_blocks > 0 ? override_blocks : (n + kCoopLdsCap - 1) / kCoopLdsCap;
    if (g < 1) g = 1;
    if (g > kCoopMaxSegs * kCoopThreads) g = kCoopMaxSegs * kCoopThreads;
    return int(g);
}

bool coop_fits_lds(int64_t C) { return C <= kCoopLdsCap; }

cq_status launch_init_begin(const JobDev* jobs, int B, hipStream_t s)
{
    CQ_TIMED_LAUNCH("k_init_begin", s, k_init_begin<<<B, kMaxK, 0, s>>>(jobs));
    return CQ_OK;
}

cq_status launch_forgy(const JobDev* jobs, int B, hipStream_t s)
{
    CQ_TIMED_LAUNCH("k_forgy", s, k_forgy<<<B, 64, 0, s>>>(jobs));
    return CQ_OK;
}

// One cooperative launch running the teams of `B` jobs (`total` blocks).
cq_status launch_init_coop(const JobDev* jobs, const int* map, int B, int total, bool lds, hipStream_t s)
{
    void* args[] = {(void*)&jobs, (void*)&map, (void*)&B};
    const void* fn = lds ? reinterpret_cast<const void*>(k_init_coop<true>)
                         : reinterpret_cast<const void*>(k_init_coop<false>);
    timer_begin("k_init_coop", s);
    const hipError_t e = hipLaunchCooperativeKernel(fn, dim3(total), dim3(kCoopThreads), args, 0, s);
    timer_end("k_init_coop", s);
    if (e != hipSuccess) {
        set_error("cooperative init launch failed: %s", hipGetErrorString(e));
        return CQ_EDEVICE;
    }
    return CQ_OK;
}

}  // namespace cq
