// Initialization schemes of Section 2.3 on the N' unique colours: Forgy (FGY),
// farthest-first / max-min (MMX) and k-means++ (KPP, weighted by pixel count).
//
// Every chosen centre is a colour, so D^2 (squared distance to the nearest
// chosen centre) is an exact integer and the sampling weights n_i D_i^2 are
// exact uint64 values.  MMX and KPP run as one cooperative launch with a grid
// barrier per round (below); FGY is a single wave.  The draw order is the one
// documented for cq_init in cq.h.
#include <stdlib.h>

#include <math.h>

#include <algorithm>
#include <vector>

#include "batch.h"

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

// ------------------------------------------------------------------------
// VAR (maximum variance), read on the pixel data set: colour i stands for
// counts[i] identical pixels.  The channel is the one with the largest pixel
// variance (N S2 - S1^2, exact; ties to the lower channel, R before G before
// B); the pixels in ascending (channel value, key) order are cut into K groups
// [floor(g N / K), floor((g+1) N / K)) and centre g is the pixel at the
// group's lower median.  The colours are in key order, so within one channel
// value they are already in key order: a tile of kVarTile colours keeps the
// pixel count of every value of every channel, and the pixel at a given
// position is found by value, then tile, then colour.
constexpr int kVarTile = 1024;
constexpr int kVarThreads = 1024;
constexpr int kVarStats = 7;  // per tile: pixels, then n x and n x^2 for R, G, B

__host__ __device__ __forceinline__ int64_t var_tiles(int64_t n) { return (n + kVarTile - 1) / kVarTile; }

// Per-tile statistics in the work region: pixel counts per (channel, value)
// as uint32 [T][3][256], then the sums as uint64 [T][kVarStats].
__device__ __forceinline__ uint32_t* var_hist(const JobDev& J) { return gp(J.d2); }
__device__ __forceinline__ unsigned long long* var_sums(const JobDev& J)
{
    return reinterpret_cast<unsigned long long*>(gp(J.d2) + var_tiles(J.n) * 3 * 256);  // 3 KiB per tile: aligned
}

__device__ __forceinline__ int key_channel(uint32_t key, int c) { return int((key >> (16 - 8 * c)) & 255u); }

__global__ void __launch_bounds__(kVarThreads) k_var_tiles(const JobDev* __restrict__ jobs, const int* __restrict__ map,
                                                          int B)
{
    __shared__ uint32_t h[3 * 256];
    __shared__ unsigned long long red[kVarStats][kVarThreads / 64];
    const int jb = find_job(map, B, blockIdx.x);
    const JobDev& J = jobs[jb];
    const int64_t t = blockIdx.x - map[jb];
    const int k = threadIdx.x, lane = k & 63, wave = k >> 6;
    for (int i = k; i < 3 * 256; i += blockDim.x) h[i] = 0u;
    __syncthreads();
    const int64_t i = t * kVarTile + k;
    unsigned long long st[kVarStats] = {0, 0, 0, 0, 0, 0, 0};
    if (i < J.n) {
        const uint32_t key = gp(J.keys)[i];
        const uint32_t cnt = gp(J.counts)[i];
        st[0] = cnt;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const unsigned x = unsigned(key_channel(key, c));
            atomicAdd(&h[c * 256 + int(x)], cnt);
            st[1 + 2 * c] = (unsigned long long)cnt * x;
            st[2 + 2 * c] = (unsigned long long)cnt * (x * x);
        }
    }
#pragma unroll
    for (int q = 0; q < kVarStats; ++q) {
        const unsigned long long v = wave_sum(st[q]);
        if (lane == 0) red[q][wave] = v;
    }
    __syncthreads();
    uint32_t* __restrict__ out = var_hist(J) + t * 3 * 256;
    for (int q = k; q < 3 * 256; q += blockDim.x) out[q] = h[q];
    if (k < kVarStats) {
        unsigned long long v = 0;
        for (int w = 0; w < kVarThreads / 64; ++w) v += red[k][w];
        var_sums(J)[t * kVarStats + k] = v;
    }
}

// One block per job: the channel, then each group's median pixel as (value,
// position among the pixels of that value), packed for k_var_find as
// channel << 48 | value << 32 | position.
__global__ void __launch_bounds__(kVarThreads) k_var_pick(const JobDev* __restrict__ jobs)
{
    const JobDev& J = jobs[blockIdx.x];
    if (J.scheme != CQ_INIT_VAR || J.n <= J.K) return;
    __shared__ unsigned long long red[kVarStats][kVarThreads / 64];
    __shared__ unsigned long long tot[kVarStats];
    __shared__ int s_ch;
    __shared__ uint32_t part[kVarThreads / 256][256];
    __shared__ unsigned long long start[257];
    const int k = threadIdx.x, lane = k & 63, wave = k >> 6;
    const int64_t T = var_tiles(J.n);
    const unsigned long long* __restrict__ sums = var_sums(J);
    unsigned long long st[kVarStats] = {0, 0, 0, 0, 0, 0, 0};
    for (int64_t t = k; t < T; t += blockDim.x)
#pragma unroll
        for (int q = 0; q < kVarStats; ++q) st[q] += sums[t * kVarStats + q];
#pragma unroll
    for (int q = 0; q < kVarStats; ++q) {
        const unsigned long long v = wave_sum(st[q]);
        if (lane == 0) red[q][wave] = v;
    }
    __syncthreads();
    if (k < kVarStats) {
        unsigned long long v = 0;
        for (int w = 0; w < kVarThreads / 64; ++w) v += red[k][w];
        tot[k] = v;
    }
    __syncthreads();
    const unsigned long long N = tot[0];
    if (k == 0) {
        int ch = 0;
        unsigned __int128 best = 0;
        for (int c = 0; c < 3; ++c) {
            const unsigned __int128 v = (unsigned __int128)N * tot[2 + 2 * c] -
                                        (unsigned __int128)tot[1 + 2 * c] * tot[1 + 2 * c];
            if (c == 0 || v > best) {
                best = v;
                ch = c;
            }
        }
        s_ch = ch;
    }
    __syncthreads();
    const int ch = s_ch;
    // pixels per value of the channel: thread k sums value k % 256 over every
    // (kVarThreads / 256)-th tile
    {
        const int v = k & 255, q = k >> 8;
        const uint32_t* __restrict__ h = var_hist(J);
        uint32_t c = 0;
        for (int64_t t = q; t < T; t += kVarThreads / 256) c += h[t * 3 * 256 + ch * 256 + v];
        part[q][v] = c;
    }
    __syncthreads();
    if (k < 256) {
        unsigned long long c = 0;
        for (int q = 0; q < kVarThreads / 256; ++q) c += part[q][k];
        start[k + 1] = c;  // pixels of value k; a prefix sum below
    }
    __syncthreads();
    if (k == 0) {
        start[0] = 0;
        for (int v = 0; v < 256; ++v) start[v + 1] += start[v];
    }
    __syncthreads();
    if (k < J.K) {
        const unsigned long long lo = (unsigned long long)(((unsigned __int128)k * N) / unsigned(J.K));
        const unsigned long long hi = (unsigned long long)(((unsigned __int128)(k + 1) * N) / unsigned(J.K));
        const unsigned long long m = lo + (hi - lo - 1) / 2;
        int l = 0, r = 256;  // last value whose first pixel is at or before m
        while (r - l > 1) {
            const int mid = (l + r) >> 1;
            if (start[mid] <= m) l = mid; else r = mid;
        }
        gp(J.vals)[k] = (uint64_t(ch) << 48) | (uint64_t(l) << 32) | (m - start[l]);
    }
}

// One block per centre: the tile holding the group's median pixel (a scan of
// the tiles' counts of that value), then the colour in the tile.
__global__ void __launch_bounds__(kVarThreads) k_var_find(const JobDev* __restrict__ jobs, const int* __restrict__ map,
                                                         int B)
{
    __shared__ uint32_t tmp[64];
    __shared__ int64_t s_tile;
    __shared__ uint32_t s_off;
    const int jb = find_job(map, B, blockIdx.x);
    const JobDev& J = jobs[jb];
    const int g = blockIdx.x - map[jb];
    const int k = threadIdx.x;
    const uint64_t target = gp(J.vals)[g];
    const int ch = int(target >> 48), v = int((target >> 32) & 255u);
    const uint32_t pos = uint32_t(target);
    const int64_t T = var_tiles(J.n);
    const uint32_t* __restrict__ h = var_hist(J);
    if (k == 0) s_tile = -1;
    __syncthreads();
    uint32_t carry = 0;
    for (int64_t t0 = 0; t0 < T; t0 += blockDim.x) {
        const int64_t t = t0 + k;
        const uint32_t c = t < T ? h[t * 3 * 256 + ch * 256 + v] : 0u;
        uint32_t total = 0;
        const uint32_t ex = block_exclusive_scan<uint32_t>(c, tmp, &total);
        if (c > 0 && carry + ex <= pos && pos < carry + ex + c) {
            s_tile = t;
            s_off = pos - (carry + ex);
        }
        __syncthreads();
        if (s_tile >= 0) break;
        carry += total;
    }
    const int64_t t = s_tile;
    if (t < 0) return;  // unreachable: the position lies below the value's pixel count
    const uint32_t off = s_off;
    const int64_t i = t * kVarTile + k;
    uint32_t key = 0, w = 0;
    if (i < J.n) {
        key = gp(J.keys)[i];
        w = key_channel(key, ch) == v ? gp(J.counts)[i] : 0u;
    }
    const uint32_t ex = block_exclusive_scan<uint32_t>(w, tmp, nullptr);
    if (w > 0 && ex <= off && off < ex + w) write_center(gp(J.centers), g, key);
}

// ------------------------------------------------------------------------
// SFF (subset farthest first): the first L = max(K, ceil(2 K ln K)) positions
// (at most N') of a partial Fisher-Yates shuffle of the colours, drawn as FGY
// draws them, then MMX on that subset in draw order: the first centre is
// subset[U(L)], then K - 1 farthest-first picks by integer D^2, ties to the
// lowest subset position.  One block per job.
//
// The draws are taken in parallel: the stream is counter-based, and a draw
// uses the next output unless it falls below U's rejection threshold (about
// T / 2^64, T < 2^28), so draw j uses output j unless an earlier draw was
// rejected; if any draw would be, the block falls back to drawing one at a
// time.  Position j of the shuffle then holds the colour index that was at
// position r_j just before step j: the value W of the last earlier step k
// with r_k = r_j, or r_j itself if there is none, where W(k), the value at
// position k before step k, is in turn W of the last earlier step that wrote
// position k, or k.  Those last-writer links come from one sort of the
// (r_j, j) pairs.  The sequential fallback keeps the displaced positions in
// an LDS hash map (open addressing) from position to colour index.
constexpr int kSffMax = 2840;    // L at K = 256
constexpr int kSffSort = 4096;   // sort width, a power of two >= kSffMax
constexpr int kSffHash = 8192;   // fallback slots, more than twice the 2 L entries
constexpr int kSffThreads = 1024;

__device__ __forceinline__ int sff_slot(const int32_t* hk, int32_t pos)
{
    uint32_t h = (uint32_t(pos) * 2654435761u) >> (32 - 13);
    while (hk[h] != -1 && hk[h] != pos) h = (h + 1) & (kSffHash - 1);
    return int(h);
}

__global__ void __launch_bounds__(kSffThreads) k_sff(const JobDev* __restrict__ jobs)
{
    const JobDev& J = jobs[blockIdx.x];
    if (J.scheme != CQ_INIT_SFF || J.n <= J.K) return;
    // the sort (fast path) and the hash map (fallback) share one buffer
    __shared__ __attribute__((aligned(16))) uint64_t buf[kSffHash];  // 64 KiB
    __shared__ int32_t rr[kSffMax];    // r_j
    __shared__ int32_t hit[kSffMax];   // the last step before k that wrote position k
    __shared__ uint32_t sub[kSffMax];  // subset keys, in draw order
    __shared__ uint32_t d2[kSffMax];
    __shared__ unsigned long long wbest[kSffThreads / 64];
    __shared__ int s_pick, s_rejected;
    const int k = threadIdx.x, lane = k & 63, wave = k >> 6;
    const uint32_t* __restrict__ keys = gp(J.keys);
    const int64_t n = J.n;
    const int K = J.K;
    const int L = int(J.init_C);  // subset size, set by the host
    Meta* __restrict__ meta = gp(J.meta);
    const uint64_t s0 = meta->rng;
    if (k == 0) s_rejected = J.init_blocks;  // nonzero: the host asks for the draws one at a time
    __syncthreads();
    // every draw, assuming no rejection: r_j = j + (output_j mod (N' - j)); the
    // first pick, output_L mod L
    for (int j = k; j <= L; j += blockDim.x) {
        const uint64_t T = j < L ? uint64_t(n - j) : uint64_t(L);
        const uint64_t out = splitmix64_at(s0, uint64_t(j));
        if (out < mod_u64(0ull - T, T)) s_rejected = 1;
        const uint64_t v = mod_u64(out, T);
        if (j < L) rr[j] = int32_t(j + int64_t(v));
        else s_pick = int(v);
    }
    __syncthreads();
    if (!s_rejected) {
        for (int i = k; i < kSffSort; i += blockDim.x)
            buf[i] = i < L ? (uint64_t(uint32_t(rr[i])) << 12) | uint64_t(i) : ~0ull;
        __syncthreads();
        // bitonic sort of the (r, step) pairs
        for (int size = 2; size <= kSffSort; size <<= 1) {
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                for (int i = k; i < kSffSort / 2; i += blockDim.x) {
                    const int lo = 2 * i - (i & (stride - 1));
                    const int hi = lo + stride;
                    const bool up = (lo & size) == 0;
                    const uint64_t a = buf[lo], b = buf[hi];
                    if ((a > b) == up) {
                        buf[lo] = b;
                        buf[hi] = a;
                    }
                }
                __syncthreads();
            }
        }
        // the links (no array is both read and written between two barriers):
        // d2[j] <- the last earlier step with r = r_j (its sorted predecessor
        // with the same r), hit[k] <- the last step before k with r = k (binary
        // search for (k, k)); ~0 / -1 for none
        for (int q = k; q < L; q += blockDim.x) {
            const uint64_t e = buf[q];
            const bool same = q > 0 && (buf[q - 1] >> 12) == (e >> 12);
            d2[e & 4095u] = same ? uint32_t(buf[q - 1] & 4095u) : 0xFFFFFFFFu;
        }
        for (int j = k; j < L; j += blockDim.x) {
            const uint64_t probe = (uint64_t(uint32_t(j)) << 12) | uint64_t(j);
            int l = 0, r = L;  // first sorted entry >= probe
            while (l < r) {
                const int m = (l + r) >> 1;
                if (buf[m] < probe) l = m + 1; else r = m;
            }
            hit[j] = (l > 0 && (buf[l - 1] >> 12) == uint64_t(j)) ? int(buf[l - 1] & 4095u) : -1;
        }
        __syncthreads();
        // position j's colour index: W(last) if a step before j drew r_j, else
        // r_j; W follows the last-writer links down to a position never written
        for (int j = k; j < L; j += blockDim.x) {
            int v = rr[j];
            if (d2[j] != 0xFFFFFFFFu) {
                int c = int(d2[j]);
                while (hit[c] >= 0) c = hit[c];
                v = c;
            }
            sub[j] = keys[v];
        }
        __syncthreads();  // d2 is cleared below
        if (k == 0) meta->rng = s0 + uint64_t(L + 1) * 0x9E3779B97F4A7C15ull;
    } else if (k == 0) {
        int32_t* hk = reinterpret_cast<int32_t*>(buf);
        int32_t* hv = hk + kSffHash;
        for (int i = 0; i < kSffHash; ++i) hk[i] = -1;
        uint64_t rng = s0;
        auto value_at = [&](int32_t p) {
            const int h = sff_slot(hk, p);
            return hk[h] == p ? hv[h] : p;
        };
        auto set_at = [&](int32_t p, int32_t val) {
            const int h = sff_slot(hk, p);
            hk[h] = p;
            hv[h] = val;
        };
        for (int j = 0; j < L; ++j) {
            const int32_t r = int32_t(j + int64_t(uniform_below(rng, uint64_t(n - j))));
            const int32_t vj = value_at(j), vr = value_at(r);
            set_at(j, vr);
            set_at(r, vj);
            sub[j] = keys[vr];
        }
        s_pick = int(uniform_below(rng, uint64_t(L)));
        meta->rng = rng;
    }
    for (int q = k; q < L; q += blockDim.x) d2[q] = 0xFFFFFFFFu;
    __syncthreads();
    double* __restrict__ centers = gp(J.centers);
    for (int j = 0; j < K; ++j) {
        const uint32_t pk = sub[s_pick];
        if (k == 0) write_center(centers, j, pk);
        int cr, cg, cb;
        key_rgb(pk, cr, cg, cb);
        // lower D^2 with the new centre; the farthest subset colour, lowest
        // position on ties, packed as D^2 << 32 | (2^32 - 1 - position)
        unsigned long long best = 0;
        for (int q = k; q < L; q += blockDim.x) {
            int r, g, b;
            key_rgb(sub[q], r, g, b);
            const uint32_t d = dist_u32(r, g, b, cr, cg, cb);
            const uint32_t m = d < d2[q] ? d : d2[q];
            d2[q] = m;
            const unsigned long long packed = (uint64_t(m) << 32) | uint64_t(0xFFFFFFFFu - uint32_t(q));
            best = packed > best ? packed : best;
        }
        best = wave_max(best);
        if (lane == 0) wbest[wave] = best;
        __syncthreads();
        if (k == 0) {
            unsigned long long b = 0;
            for (int w = 0; w < kSffThreads / 64; ++w) b = wbest[w] > b ? wbest[w] : b;
            s_pick = int(0xFFFFFFFFu - uint32_t(b));
        }
        __syncthreads();
    }
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
    // round tags of the cooperative initialization start below round 1: the
    // block slots and the pick slots
    uint64_t* __restrict__ vals = gp(J.vals);
    for (int t = k; t < 2 * kInitMaxBlocks + 2; t += blockDim.x) vals[t] = 0ull;
    if (J.n > J.K || k >= J.K) return;
    if (k < J.n) {
        write_center(J.centers, k, gp(J.keys)[k]);
    } else {
        gp(J.centers)[3 * k] = gp(J.centers)[3 * k + 1] = gp(J.centers)[3 * k + 2] = 0.0;
    }
}

// ------------------------------------------------------------------------
// Cooperative MMX / KPP: one launch runs all K rounds of every job, each job
// with its own team of G co-resident blocks.  Block b of a team owns the
// colours [b C, (b+1) C); thread t of a block owns the run of R = C / T
// (rounded up, T threads per block) consecutive colours from t R on.  Round j:
//   1. every thread lowers D^2 of its run with the colour picked in round j-1;
//      KPP: it keeps the sum of n D^2 over its run (the counts alone in round
//      0) in LDS, and the block publishes the sum over its colours in its own
//      slot; MMX: the block publishes the largest (D^2, -index) packed into 46
//      bits.  A published value carries the tag j + 1 (bits 46-63);
//   2. every block waits until all G slots carry the tag j + 1 (a shared
//      arrival counter would serialize G atomics on one address);
//   3. MMX: the largest value names the colour, the same in every block.
//      KPP: r = U(total) from the block's own copy of the splitmix64 stream
//      (every block draws the same values), and the block whose inclusive
//      prefix of block sums first exceeds r.  That block alone finds the run
//      and the colour holding r from its own data and publishes the colour's
//      key, tagged, in the team's pick slot; the others wait for it.
// Published values are written and read with agent-scope relaxed atomics and
// each reader checks the tag of the value it uses, so no fence (and no
// write-back or invalidation of the L2) is needed: a value that is not there
// yet is read again.  They are double-buffered by round parity: a block
// writes a parity again only after every block has published the next round,
// that is after all of them have finished reading it.  Per-thread data of a
// run is stored transposed (entry u of thread t at u T + t), so the threads
// of a wave touch consecutive words.
//
// Two kernels run these rounds: k_init_reg keeps a block's colours on chip
// (the usual case), k_init_coop reads them from global memory every round
// (teams whose colours exceed what kInitMaxBlocks blocks hold on chip).
constexpr int kTagShift = 46;      // KPP sums stay below 2^46 (2^28 pixels x 3 x 255^2)
constexpr uint64_t kValMask = (1ull << kTagShift) - 1ull;
constexpr uint32_t kIndexBits = 28;  // MMX: colour index below 2^28, D^2 below 2^18

// One wave: the first of `cnt` weights (read through `get`) whose running
// sum, started at *base, exceeds r; *base becomes the sum before it.  Returns
// -1 if there is none.
template <typename F>
__device__ __forceinline__ int64_t wave_find(int64_t cnt, uint64_t r, uint64_t* base, F get)
{
    const int lane = threadIdx.x & 63;
    uint64_t carry = *base;
    for (int64_t c0 = 0; c0 < cnt; c0 += 64) {
        const int64_t c = c0 + lane;
        const uint64_t v = c < cnt ? get(c) : 0ull;
        const uint64_t incl = carry + wave_incl_scan(v);
        const unsigned long long hit = __ballot(c < cnt && incl > r);
        if (hit) {
            const int l = __ffsll(hit) - 1;
            *base = __shfl(incl - v, l, 64);
            return c0 + l;
        }
        carry = __shfl(incl, 63, 64);
    }
    return -1;
}

__device__ __forceinline__ uint64_t load_tagged(const uint64_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void store_tagged(uint64_t* p, uint64_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Colours of every block read from global memory in every round, each
// thread keeping the D^2 of its run in global memory (teams too large for the
// register kernel below).
__global__ void __launch_bounds__(kInitThreads) k_init_coop(const JobDev* __restrict__ jobs,
                                                            const int* __restrict__ map, int B)
{
    __shared__ uint64_t tmp[64];
    __shared__ uint64_t s_val[kInitMaxBlocks];
    __shared__ uint64_t s_run[kInitThreads];  // KPP: the threads' run sums of n D^2
    __shared__ int64_t s_pick;
    __shared__ uint32_t s_key;
    __shared__ int s_ok;
    const int jb = find_job(map, B, blockIdx.x);
    const JobDev& J = jobs[jb];
    const int G = J.init_blocks;  // team size, <= kInitMaxBlocks
    const int tb = blockIdx.x - map[jb];
    const uint32_t* __restrict__ keys = gp(J.keys);
    const uint32_t* __restrict__ counts = gp(J.counts);
    const int64_t n = J.n;
    const int K = J.K;
    const bool kpp = J.scheme == CQ_INIT_KMEANSPP;
    const int64_t C = J.init_C;
    const int R = int((C + kInitThreads - 1) / kInitThreads);  // run length
    const int64_t Cb = int64_t(R) * kInitThreads;             // D^2 slots per block
    uint32_t* __restrict__ d2own = gp(J.d2) + int64_t(tb) * Cb;             // [G Cb], transposed runs
    uint64_t* __restrict__ tags = gp(J.vals);                               // [2][kInitMaxBlocks]
    uint64_t* __restrict__ pick = gp(J.vals) + 2 * kInitMaxBlocks;          // [2]: KPP picked key
    Meta* __restrict__ meta = gp(J.meta);
    double* __restrict__ centers = gp(J.centers);
    const int64_t lo = int64_t(tb) * C;
    const int64_t hi = lo + C < n ? lo + C : n;
    const int mine_n = hi > lo ? int(hi - lo) : 0;
    const int t = threadIdx.x;
    const int wave = t >> 6, lane = t & 63;
    const int qlo = t * R;  // this thread's run, block-local colour indices
    const int qn = mine_n - qlo >= R ? R : (mine_n > qlo ? mine_n - qlo : 0);
    uint64_t rng = J.seed;  // wave 0 draws; every block draws the same values
    int cr = 0, cg = 0, cb = 0;
    for (int j = 0; j < K; ++j) {
        const int par = j & 1;
        const uint64_t tag = uint64_t(j + 1) << kTagShift;
        __syncthreads();  // the previous round's readers of the shared values are done
        if (!kpp && j == 0) {
            if (t == 0) s_pick = int64_t(uniform_below(rng, uint64_t(n)));
        } else {
            // 1. own run
            uint64_t acc = 0;
            auto step = [&](int u, uint32_t key, uint32_t cnt, uint32_t old) -> uint32_t {
                uint32_t m = 1u;  // KPP round 0: the weights are the counts
                if (j > 0) {
                    int r, g, b;
                    key_rgb(key, r, g, b);
                    const uint32_t d = dist_u32(r, g, b, cr, cg, cb);
                    m = old < d ? old : d;
                }
                if (kpp) {
                    acc += uint64_t(cnt) * m;
                } else {
                    const uint64_t packed = (uint64_t(m) << kIndexBits) |
                                            uint64_t(((1u << kIndexBits) - 1u) - uint32_t(lo + qlo + u));
                    acc = packed > acc ? packed : acc;
                }
                return m;
            };
            for (int u = 0; u < qn; ++u) {
                const int x = u * kInitThreads + t;
                const int64_t i = lo + qlo + u;
                const uint32_t m = step(u, keys[i], counts[i], j > 1 ? d2own[x] : 0xFFFFFFFFu);
                if (j > 0) d2own[x] = m;
            }
            if (kpp) s_run[t] = acc;
            acc = kpp ? wave_sum(acc) : wave_max(acc);
            if (lane == 0) tmp[wave] = acc;
            __syncthreads();
            if (t == 0) {
                uint64_t v = tmp[0];
                for (int w = 1; w < kInitThreads / 64; ++w) v = kpp ? v + tmp[w] : (tmp[w] > v ? tmp[w] : v);
                store_tagged(&tags[par * kInitMaxBlocks + tb], tag | v);
            }
            // 2. wave 0 waits for the team's tags
            if (wave == 0) {
                int ok = 1;
                uint32_t spins = 0;
                auto keep_waiting = [&]() {
                    if (__hip_atomic_load(&meta->sync_error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
                        ++spins > kSpinLimit)
                        return false;
                    __builtin_amdgcn_s_sleep(1);
                    return true;
                };
                for (int c0 = 0; c0 < G; c0 += 64) {
                    const int c = c0 + lane;
                    if (c >= G) continue;
                    uint64_t v;
                    for (;;) {
                        v = load_tagged(&tags[par * kInitMaxBlocks + c]);
                        if ((v & ~kValMask) == tag) break;
                        if (!keep_waiting()) {
                            ok = 0;
                            break;
                        }
                    }
                    s_val[c] = v & kValMask;
                }
                if (kpp && __ballot(ok == 0) == 0ull) {
                    // 3. the block holding r
                    uint64_t total = 0;
                    for (int c0 = 0; c0 < G; c0 += 64) total += wave_sum(c0 + lane < G ? s_val[c0 + lane] : 0ull);
                    const uint64_t r = total ? uniform_below(rng, total) : 0ull;
                    uint64_t base = 0;
                    const int64_t c = wave_find(G, r, &base, [&](int64_t x) { return s_val[x]; });
                    uint32_t key = 0u;
                    if (c == tb) {
                        // this block: the run (lane l holds runs [l S, (l + 1) S)) and
                        // the colour in it, both from its own data
                        constexpr int S = kInitThreads / 64;
                        uint64_t rv[S];
                        uint64_t lsum = 0;
#pragma unroll
                        for (int u = 0; u < S; ++u) {
                            rv[u] = s_run[lane * S + u];
                            lsum += rv[u];
                        }
                        const uint64_t lincl = base + wave_incl_scan(lsum);
                        const unsigned long long hitl = __ballot(lincl > r);
                        int64_t pk = -1;
                        if (hitl) {
                            const int l = __ffsll(hitl) - 1;
                            uint64_t acc2 = __shfl(lincl - lsum, l, 64);  // sum before lane l's runs
                            int tr = -1;
#pragma unroll
                            for (int u = 0; u < S; ++u) {
                                const uint64_t v = __shfl(rv[u], l, 64);
                                if (tr < 0 && acc2 + v > r) tr = l * S + u;
                                else if (tr < 0) acc2 += v;
                            }
                            if (tr >= 0) {
                                const int rn = mine_n - tr * R < R ? mine_n - tr * R : R;
                                uint64_t carry = acc2;
                                for (int x0 = 0; x0 < rn && pk < 0; x0 += 64) {
                                    const int u = x0 + lane;
                                    const bool in = u < rn;
                                    uint64_t w = 0;
                                    uint32_t kx = 0;
                                    if (in) {
                                        const int x = u * kInitThreads + tr;
                                        const int64_t i = lo + int64_t(tr) * R + u;
                                        kx = keys[i];
                                        w = uint64_t(counts[i]) * (j == 0 ? 1u : d2own[x]);
                                    }
                                    const uint64_t incl = carry + wave_incl_scan(w);
                                    const unsigned long long hit = __ballot(in && incl > r);
                                    if (hit) {
                                        const int hl = __ffsll(hit) - 1;
                                        pk = lo + int64_t(tr) * R + x0 + hl;
                                        key = __builtin_amdgcn_readlane(kx, hl);
                                    }
                                    carry = __shfl(incl, 63, 64);
                                }
                            }
                        }
                        if (pk < 0) key = keys[0];  // unreachable: r < total
                        if (lane == 0) store_tagged(&pick[par], tag | key);
                    } else {
                        // another block holds r: wait for its pick
                        uint64_t v = 0;
                        for (;;) {
                            v = load_tagged(&pick[par]);
                            if ((v & ~kValMask) == tag) break;
                            if (!keep_waiting()) {
                                ok = 0;
                                break;
                            }
                        }
                        key = uint32_t(v) & 0xffffffu;
                    }
                    if (lane == 0) s_key = key;
                }
                const bool all_ok = __ballot(ok == 0) == 0ull;
                if (!all_ok && lane == 0)
                    __hip_atomic_store(&meta->sync_error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (lane == 0) s_ok = all_ok ? 1 : 0;
            }
            __syncthreads();
            if (!s_ok) return;
            if (!kpp) {
                uint64_t best = 0;
                for (int c = t; c < G; c += kInitThreads) best = s_val[c] > best ? s_val[c] : best;
                best = wave_max(best);
                if (lane == 0) tmp[wave] = best;
                __syncthreads();
                if (t == 0) {
                    for (int w = 0; w < kInitThreads / 64; ++w) best = tmp[w] > best ? tmp[w] : best;
                    const int64_t pk =
                        int64_t(((1u << kIndexBits) - 1u) - uint32_t(best & ((1u << kIndexBits) - 1u)));
                    s_pick = pk < n ? pk : 0;  // every colour packs a non-zero value, so pk < n
                }
            }
        }
        __syncthreads();
        // a KPP pick arrives with its key
        const uint32_t pick_key = kpp ? s_key : keys[s_pick];
        if (t == 0 && tb == 0) {
            write_center(centers, j, pick_key);
            if (j == K - 1) meta->rng = rng;
        }
        key_rgb(pick_key, cr, cg, cb);
    }
}

// Inclusive scan within each row of 16 lanes (lane 15 of a row holds the
// row's sum).
__device__ __forceinline__ uint64_t row16_incl_scan(uint64_t x)
{
    const uint64_t z = 0;
    x += dpp_move<kDppRowShr1, 0xf>(z, x);
    x += dpp_move<kDppRowShr2, 0xf>(z, x);
    x += dpp_move<kDppRowShr4, 0xf>(z, x);
    x += dpp_move<kDppRowShr8, 0xf>(z, x);
    return x;
}

// ------------------------------------------------------------------------
// The same rounds with every thread's run of up to R colours on chip: the
// keys and D^2 in VGPRs, the counts (KPP) in dynamic LDS, transposed (entry
// u of thread t at u T + t).  A block holds up to R T colours (32768 at
// R = 32).  A team of one block (G = 1) exchanges nothing through memory:
// the block's total is the job's total and its own threads find the pick.  In a team of several blocks the protocol above carries the block
// totals and the pick.  In the block that holds r, the thread that holds it
// finds the colour among its own registers.
template <int R>
__global__ void __launch_bounds__(kInitThreads) k_init_reg(const JobDev* __restrict__ jobs,
                                                           const int* __restrict__ map, int B)
{
    extern __shared__ uint32_t lcnt[];                 // [R T] counts, transposed
    __shared__ uint64_t s_wave[kInitThreads / 64];     // MMX: per-wave maxima
    __shared__ uint64_t s_run[kInitThreads];           // KPP: the threads' run sums of n D^2
    __shared__ uint64_t s_grp[kInitThreads / 16];      // KPP: sums of 16 consecutive threads' runs
    __shared__ uint64_t s_val[kInitMaxBlocks];
    __shared__ uint64_t s_rloc;  // r minus the weights before the owner thread's run
    __shared__ uint32_t s_key;   // the colour picked in this round
    __shared__ int s_owner;      // the thread of this block holding r
    __shared__ int s_state;      // 0: a wait gave up, 1: pick in s_key, 2: this block holds r
    const int jb = find_job(map, B, blockIdx.x);
    const JobDev& J = jobs[jb];
    const int G = J.init_blocks;  // team size, <= kInitMaxBlocks
    const int tb = blockIdx.x - map[jb];
    const uint32_t* __restrict__ keys = gp(J.keys);
    const uint32_t* __restrict__ counts = gp(J.counts);
    const int64_t n = J.n;
    const int K = J.K;
    const bool kpp = J.scheme == CQ_INIT_KMEANSPP;
    const int64_t C = J.init_C;                                // colours per block, <= R T
    const int Rr = int((C + kInitThreads - 1) / kInitThreads);  // run length, <= R
    uint64_t* __restrict__ tags = gp(J.vals);                       // [2][kInitMaxBlocks]
    uint64_t* __restrict__ pick = gp(J.vals) + 2 * kInitMaxBlocks;  // [2]: KPP picked key
    Meta* __restrict__ meta = gp(J.meta);
    double* __restrict__ centers = gp(J.centers);
    const int64_t lo = int64_t(tb) * C;
    const int64_t hi = lo + C < n ? lo + C : n;
    const int mine_n = hi > lo ? int(hi - lo) : 0;
    const int t = threadIdx.x;
    const int wave = t >> 6, lane = t & 63;
    const int qlo = t * Rr;
    const int qn = mine_n - qlo >= Rr ? Rr : (mine_n > qlo ? mine_n - qlo : 0);
    // coalesced loads through the LDS array: the keys first (into registers),
    // then the counts (which stay).  A thread pads its run to R entries with
    // D^2 0 and count 0, which weigh nothing and never hold the largest D^2
    // (some real colour of the job is farther than 0 from every centre
    // while fewer than N' are chosen).
    uint32_t ky[R], d2[R];
    for (int p = 0; p < Rr; ++p) {
        const int q = p * kInitThreads + t;
        if (q < mine_n) lcnt[(q % Rr) * kInitThreads + q / Rr] = keys[lo + q];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < R; ++u) {
        ky[u] = u < qn ? lcnt[u * kInitThreads + t] : 0u;
        d2[u] = u < qn ? 0xFFFFFFFFu : 0u;
    }
    __syncthreads();
    if (kpp) {
        for (int p = 0; p < Rr; ++p) {
            const int q = p * kInitThreads + t;
            if (q < mine_n) lcnt[(q % Rr) * kInitThreads + q / Rr] = counts[lo + q];
        }
        for (int u = qn; u < R; ++u) lcnt[u * kInitThreads + t] = 0u;
    }
    __syncthreads();  // the counts are in place (a thread wrote other threads' entries)
    uint64_t run_n = 0;  // KPP: the run's pixel count (the weights of round 0)
    if (kpp) {
#pragma unroll
        for (int u = 0; u < R; ++u) run_n += lcnt[u * kInitThreads + t];
    }
    uint64_t rng = J.seed;  // wave 0 draws; every block draws the same values
    uint32_t pick_key = 0;
    for (int j = 0; j < K; ++j) {
        const int par = j & 1;
        const uint64_t tag = uint64_t(j + 1) << kTagShift;
        // No barrier is needed here: this round's first shared writes (run
        // and group sums, MMX wave maxima) were last read by wave 0 before
        // the previous round's barrier after step 2, and the values every
        // thread reads at the end of a round (state, owner, key) are written
        // again only after this round's barrier after step 1.
        // 1. own run: D^2 against the previous pick (from four-byte dot
        // products of the packed colours: |x - c|^2 = x.x + c.c - 2 x.c),
        // then the run's sum of n D^2 (KPP; the counts alone in round 0) or
        // its largest D^2, first position on ties (MMX).  In round 0 there is
        // no pick (pick_key is 0): c.c is replaced by 2^31 - 1, so every
        // colour's value, x.x + 2^31 - 1, exceeds any squared distance of
        // two colours (at most 3 * 255^2), and the first real pick replaces
        // it; padding keeps D^2 0.  All R entries, padding included, in
        // straight-line code: the registers of the run are never under a
        // branch.
        const uint32_t cc = j == 0 ? 0x7FFFFFFFu : __builtin_amdgcn_udot4(pick_key, pick_key, 0u, false);
#pragma unroll
        for (int u = 0; u < R; ++u) {
            asm volatile("" : "+v"(ky[u]));  // keeps x.x from being held across rounds
            const uint32_t xxcc = __builtin_amdgcn_udot4(ky[u], ky[u], cc, false);  // x.x + c.c
            const uint32_t xc = __builtin_amdgcn_udot4(ky[u], pick_key, 0u, false);
            const uint32_t d = xxcc - 2u * xc;
            d2[u] = d2[u] < d ? d2[u] : d;
        }
        uint64_t acc = 0;
        if (kpp) {
            // weight n D^2 in two sums, so that the multiply-adds form two
            // chains; in round 0 the weights are the counts (the run's sum,
            // taken once; padding has count 0).  The branch only reads the
            // run's registers.
            if (j == 0) {
                acc = run_n;
            } else {
                uint64_t acc1 = 0;
#pragma unroll
                for (int u = 0; u < R; u += 2) {
                    acc += uint64_t(lcnt[u * kInitThreads + t]) * d2[u];
                    if (u + 1 < R) acc1 += uint64_t(lcnt[(u + 1) * kInitThreads + t]) * d2[u + 1];
                }
                acc += acc1;
            }
        } else {
            uint32_t best_m = d2[0], best_u = 0;
#pragma unroll
            for (int u = 1; u < R; ++u) {
                best_u = d2[u] > best_m ? uint32_t(u) : best_u;
                best_m = d2[u] > best_m ? d2[u] : best_m;
            }
            if (qn > 0)
                acc = (uint64_t(best_m) << kIndexBits) |
                      uint64_t(((1u << kIndexBits) - 1u) - uint32_t(lo + qlo + int(best_u)));
        }
        if (!kpp && j == 0) {
            // MMX: the first colour uniform over the colours
            if (t == 0) {
                s_key = keys[uniform_below(rng, uint64_t(n))];
                s_state = 1;
            }
        } else {
            if (kpp) {
                s_run[t] = acc;
                // the sum of each row of 16 lanes (threads 16 g .. 16 g + 15)
                const uint64_t rs = row16_incl_scan(acc);
                if ((lane & 15) == 15) s_grp[t >> 4] = rs;
            } else {
                acc = wave_max(acc);
                if (lane == 0) s_wave[wave] = acc;
            }
            __syncthreads();
            if (wave == 0) {
                // 2. the block's value, then the team's; KPP: lane l holds
                // the sum of the runs of threads [16 l, 16 l + 16)
                static_assert(kInitThreads == 1024, "64 groups of 16 threads, one per lane of wave 0");
                const uint64_t grp = kpp ? s_grp[lane] : 0ull;
                uint64_t v = kpp ? wave_sum(grp) : wave_max(lane < kInitThreads / 64 ? s_wave[lane] : 0ull);
                uint64_t total = v;
                int ok = 1;
                uint32_t spins = 0;
                // the team's error flag is read every 64th spin only, so that a
                // poll is one load
                auto keep_waiting = [&]() {
                    if (++spins > kSpinLimit ||
                        ((spins & 63u) == 0 &&
                         __hip_atomic_load(&meta->sync_error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0))
                        return false;
                    __builtin_amdgcn_s_sleep(1);
                    return true;
                };
                if (G > 1) {
                    if (lane == 0) store_tagged(&tags[par * kInitMaxBlocks + tb], tag | v);
                    uint64_t part = 0;
                    for (int c0 = 0; c0 < G; c0 += 64) {
                        const int c = c0 + lane;
                        uint64_t x = 0;
                        if (c < G) {
                            for (;;) {
                                x = load_tagged(&tags[par * kInitMaxBlocks + c]);
                                if ((x & ~kValMask) == tag) break;
                                if (!keep_waiting()) {
                                    ok = 0;
                                    break;
                                }
                            }
                            x &= kValMask;
                            s_val[c] = x;
                        }
                        part = kpp ? part + x : (x > part ? x : part);
                    }
                    total = kpp ? wave_sum(part) : wave_max(part);
                }
                int state = 1;
                if (__ballot(ok == 0) != 0ull) {
                    state = 0;
                } else if (kpp) {
                    // 3. the block holding r, then (there) the thread holding it
                    const uint64_t r = total ? uniform_below(rng, total) : 0ull;
                    uint64_t base = 0;
                    const int64_t c = G > 1 ? wave_find(G, r, &base, [&](int64_t x) { return s_val[x]; }) : 0;
                    if (c == tb) {
                        // the thread holding r: one scan of the 64 group sums
                        // finds the group, a second one of the group's 16 run
                        // sums (one per lane) the thread
                        state = 2;
                        const uint64_t lincl = base + wave_incl_scan(grp);
                        const unsigned long long hitl = __ballot(lincl > r);
                        const int l = hitl ? __ffsll(hitl) - 1 : 63;  // hitl != 0 since r < total
                        const uint64_t gbefore = __shfl(lincl - grp, l, 64);
                        const uint64_t rv = lane < 16 ? s_run[16 * l + lane] : 0ull;
                        const uint64_t incl2 = gbefore + wave_incl_scan(rv);
                        const unsigned long long hitu = __ballot(lane < 16 && incl2 > r);
                        const int u = hitu ? __ffsll(hitu) - 1 : 15;
                        const uint64_t before = __shfl(incl2 - rv, u, 64);
                        if (lane == 0) {
                            s_owner = 16 * l + u;
                            s_rloc = r - before;
                        }
                    } else {
                        uint64_t x = 0;
                        for (;;) {
                            x = load_tagged(&pick[par]);
                            if ((x & ~kValMask) == tag) break;
                            if (!keep_waiting()) {
                                ok = 0;
                                break;
                            }
                        }
                        if (__ballot(ok == 0) != 0ull) state = 0;
                        if (lane == 0) s_key = uint32_t(x) & 0xffffffu;
                    }
                } else {
                    // MMX: the largest (D^2, -index) names the colour
                    const int64_t pk =
                        int64_t(((1u << kIndexBits) - 1u) - uint32_t(total & ((1u << kIndexBits) - 1u)));
                    if (lane == 0) s_key = keys[pk < n ? pk : 0];  // every colour packs a non-zero value
                }
                if (state == 0 && lane == 0)
                    __hip_atomic_store(&meta->sync_error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (lane == 0) s_state = state;
            }
        }
        __syncthreads();
        const int state = s_state;
        if (state == 0) return;
        if (state == 2) {
            // the owner thread walks its own run
            if (t == s_owner) {
                const uint64_t rl = s_rloc;
                uint64_t acc = 0;
                uint32_t key = ky[0];
                bool found = false;
#pragma unroll
                for (int u = 0; u < R; ++u) {
                    const uint64_t w = uint64_t(lcnt[u * kInitThreads + t]) * (j == 0 ? 1u : d2[u]);
                    const bool hit = !found && acc + w > rl;
                    key = hit ? ky[u] : key;
                    acc += found || hit ? 0ull : w;
                    found = found || hit;
                }
                s_key = key;
                if (G > 1) store_tagged(&pick[par], tag | key);
            }
            __syncthreads();
        }
        pick_key = s_key;
        if (t == 0 && tb == 0) {
            write_center(centers, j, pick_key);
            if (j == K - 1) meta->rng = rng;
        }
    }
}

// ------------------------------------------------------------------ host
// Colours per thread of the register kernels, smallest first.
constexpr int kCoopVariants = 5;
constexpr int kCoopR[kCoopVariants] = {4, 8, 16, 24, 32};

// Colours per block of the register kernels (R colours per thread).
int64_t coop_reg_colours(int R) { return int64_t(R) * kInitThreads; }

static size_t coop_dyn_lds(int variant) { return variant > 0 ? sizeof(uint32_t) * size_t(variant) * kInitThreads : 0; }

static const void* coop_kernel(int variant)
{
    switch (variant) {
    case 4: return reinterpret_cast<const void*>(k_init_reg<4>);
    case 8: return reinterpret_cast<const void*>(k_init_reg<8>);
    case 16: return reinterpret_cast<const void*>(k_init_reg<16>);
    case 24: return reinterpret_cast<const void*>(k_init_reg<24>);
    case 32: return reinterpret_cast<const void*>(k_init_reg<32>);
    default: return reinterpret_cast<const void*>(k_init_coop);
    }
}

// Co-resident blocks of a cooperative initialization kernel on this device
// (0: no cooperative launch).  variant: 4, 8, 16, 24 or 32, the register kernels
// with that many colours per thread; 0, the kernel that keeps D^2 in global
// memory.
int coop_capacity(int variant)
{
    static int cached[kCoopVariants + 1] = {-1, -1, -1, -1, -1, -1};
    int slot = kCoopVariants;
    for (int v = 0; v < kCoopVariants; ++v)
        if (kCoopR[v] == variant) slot = v;
    if (cached[slot] < 0) {
        int dev = 0, cus = 0, per_cu = 0, coop_ok = 0;
        cached[slot] = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&coop_ok, hipDeviceAttributeCooperativeLaunch, dev) == hipSuccess &&
            coop_ok &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, coop_kernel(variant), kInitThreads,
                                                         coop_dyn_lds(variant)) == hipSuccess)
            cached[slot] = cus * per_cu;
    }
    return cached[slot];
}

// The launch plan (coop_plan.h) on this device's co-resident capacities.
cq_status plan_coop(const std::vector<int64_t>& n, std::vector<CoopLaunch>& plan)
{
    plan.clear();
    if (std::none_of(n.begin(), n.end(), [](int64_t x) { return x > 0; })) return CQ_OK;
    int cap[kCoopVariants];
    for (int v = 0; v < kCoopVariants; ++v) cap[v] = coop_capacity(kCoopR[v]);
    const int cap0 = coop_capacity(0);
    for (int v = 0; v < kCoopVariants; ++v)
        if (cap[v] <= 0 || cap0 <= 0) {
            set_error("cooperative launch is not available on this device");
            return CQ_EDEVICE;
        }
    plan_coop_with(n, kCoopR, cap, kCoopVariants, cap0, kInitMaxBlocks, kInitThreads, plan);
    return CQ_OK;
}

cq_status launch_init_begin(const JobDev* jobs, int B, hipStream_t s)
{
    CQ_TIMED_LAUNCH("k_init_begin", s, k_init_begin<<<B, kMaxK, 0, s>>>(jobs));
    return CQ_OK;
}

// ------------------------------------------------------------------ DEN
// DEN (Section 2.3, density-based): the colour cube in 512 uniform cells
// (value >> 5 per channel); cell c with u_c of the N' colours gets
// floor(K u_c / N') centres and the K - (their sum) left over go one each to
// the cells of largest remainder K u_c mod N' (ties to the lower cell); per
// cell in index order the quota is drawn without replacement from the cell's
// colours in key order, as FGY draws, all from the one splitmix64 stream.
//   k_den_tiles  per tile of kDenTile key-ordered colours: its colours per
//                cell, into a tile x cell matrix;
//   k_den_pick   per job, one thread per cell: the matrix column turned into
//                the exclusive prefix over the tiles, the quotas; then one
//                thread takes the K draws in order, the Fisher-Yates swaps of
//                a cell kept in LDS as (position, value) pairs, and records
//                (cell, position in the cell) per centre;
//   k_den_find   per centre: the tile holding that position (binary search on
//                the prefixes) and the colour in it (a block scan).
constexpr int kDenCells = 512;
constexpr int kDenTile = 1024;

__host__ __device__ __forceinline__ int64_t den_tiles(int64_t n) { return (n + kDenTile - 1) / kDenTile; }

__device__ __forceinline__ uint32_t* den_matrix(const JobDev& J) { return gp(J.d2); }

__device__ __forceinline__ int den_cell(uint32_t key)
{
    return int(((key >> 21) & 7u) * 64u + ((key >> 13) & 7u) * 8u + ((key >> 5) & 7u));
}

__global__ void __launch_bounds__(kDenCells) k_den_tiles(const JobDev* __restrict__ jobs,
                                                         const int* __restrict__ map, int B)
{
    __shared__ uint32_t cnt[kDenCells];
    const int jb = find_job(map, B, blockIdx.x);
    const JobDev& J = jobs[jb];
    const int64_t t = blockIdx.x - map[jb];
    cnt[threadIdx.x] = 0u;
    __syncthreads();
    for (int k = threadIdx.x; k < kDenTile; k += kDenCells) {
        const int64_t i = t * kDenTile + k;
        if (i < J.n) atomicAdd(&cnt[den_cell(gp(J.keys)[i])], 1u);
    }
    __syncthreads();
    den_matrix(J)[t * kDenCells + threadIdx.x] = cnt[threadIdx.x];
}

__global__ void __launch_bounds__(kDenCells) k_den_pick(const JobDev* __restrict__ jobs)
{
    __shared__ uint64_t s_rem[kDenCells];
    __shared__ uint32_t s_u[kDenCells], s_q[kDenCells];
    __shared__ uint32_t s_pos[2 * kMaxK], s_val[2 * kMaxK];
    __shared__ uint32_t tmp[64];
    const JobDev& J = jobs[blockIdx.x];
    if (J.scheme != CQ_INIT_DEN || J.n <= J.K) return;
    const int c = threadIdx.x;
    const int64_t T = den_tiles(J.n);
    uint32_t* __restrict__ h = den_matrix(J);
    uint32_t u = 0;
    constexpr int kBatch = 16;  // loads issued before the stores of a batch
    for (int64_t t0 = 0; t0 < T; t0 += kBatch) {
        uint32_t v[kBatch];
#pragma unroll
        for (int e = 0; e < kBatch; ++e) v[e] = t0 + e < T ? h[(t0 + e) * kDenCells + c] : 0u;
#pragma unroll
        for (int e = 0; e < kBatch; ++e) {
            if (t0 + e < T) h[(t0 + e) * kDenCells + c] = u;
            u += v[e];
        }
    }
    const uint64_t n = uint64_t(J.n);
    const uint64_t share = uint64_t(J.K) * u;
    uint32_t q = uint32_t(share / n);
    const uint64_t rem = share - uint64_t(q) * n;
    s_rem[c] = rem;
    uint32_t given = 0;
    block_exclusive_scan<uint32_t>(q, tmp, &given);  // also orders the s_rem stores before the reads
    const uint32_t left = uint32_t(J.K) - given;
    if (rem > 0) {
        uint32_t rank = 0;
        for (int d = 0; d < kDenCells; ++d) {
            const uint64_t o = s_rem[d];
            rank += (o > rem || (o == rem && d < c)) ? 1u : 0u;
        }
        if (rank < left) ++q;
    }
    s_q[c] = q;
    s_u[c] = u;
    __syncthreads();
    if (c != 0) return;
    uint64_t st = J.seed;
    uint64_t* __restrict__ sel = gp(J.vals);
    int slot = 0;
    for (int cell = 0; cell < kDenCells; ++cell) {
        const uint32_t qc = s_q[cell], uc = s_u[cell];
        int len = 0;  // displaced positions of this cell so far
        for (uint32_t j = 0; j < qc; ++j) {
            const uint32_t r = j + uint32_t(uniform_below(st, uint64_t(uc - j)));
            uint32_t a = j, b = r;
            int ia = -1, ib = -1;
            for (int e = 0; e < len; ++e) {
                if (s_pos[e] == j) {
                    a = s_val[e];
                    ia = e;
                }
                if (s_pos[e] == r) {
                    b = s_val[e];
                    ib = e;
                }
            }
            // position j takes the value at r, and r the value at j
            if (ia < 0) {
                ia = len++;
                s_pos[ia] = j;
            }
            s_val[ia] = b;
            if (r != j) {
                if (ib < 0) {
                    ib = len++;
                    s_pos[ib] = r;
                }
                s_val[ib] = a;
            }
            sel[slot++] = (uint64_t(cell) << 32) | b;
        }
    }
}

__global__ void __launch_bounds__(kDenTile) k_den_find(const JobDev* __restrict__ jobs, const int* __restrict__ map,
                                                       int B)
{
    __shared__ uint32_t tmp[64];
    __shared__ int64_t s_tile;
    const int jb = find_job(map, B, blockIdx.x);
    const JobDev& J = jobs[jb];
    const int g = blockIdx.x - map[jb];
    const uint64_t target = gp(J.vals)[g];
    const int cell = int(target >> 32);
    const uint32_t pos = uint32_t(target);
    const uint32_t* __restrict__ h = den_matrix(J);
    if (threadIdx.x == 0) {
        // the last tile whose prefix for the cell is at most pos holds it
        int64_t lo = 0, hi = den_tiles(J.n);
        while (hi - lo > 1) {
            const int64_t mid = (lo + hi) >> 1;
            if (h[mid * kDenCells + cell] <= pos) lo = mid; else hi = mid;
        }
        s_tile = lo;
    }
    __syncthreads();
    const int64_t t = s_tile;
    const uint32_t off = pos - h[t * kDenCells + cell];
    const int64_t i = t * kDenTile + threadIdx.x;
    uint32_t key = 0, f = 0;
    if (i < J.n) {
        key = gp(J.keys)[i];
        f = den_cell(key) == cell ? 1u : 0u;
    }
    const uint32_t ex = block_exclusive_scan<uint32_t>(f, tmp, nullptr);
    if (f && ex == off) write_center(gp(J.centers), g, key);
}

int den_tile_count(int64_t n) { return int(den_tiles(n)); }

cq_status launch_den(const JobDev* jobs, const int* maps, int B, int tiles, int centres, hipStream_t s)
{
    CQ_TIMED_LAUNCH("k_den_tiles", s,
                    k_den_tiles<<<tiles, kDenCells, 0, s>>>(jobs, maps + kMapDenTiles * (B + 1), B));
    CQ_TIMED_LAUNCH("k_den_pick", s, k_den_pick<<<B, kDenCells, 0, s>>>(jobs));
    CQ_TIMED_LAUNCH("k_den_find", s,
                    k_den_find<<<centres, kDenTile, 0, s>>>(jobs, maps + kMapDenCentres * (B + 1), B));
    return CQ_OK;
}

// LBG stage of each job of a batch (one block per job): with init_C = 0 the
// single centre is set to zero (the start of the iteration that yields the
// centroid); otherwise the first K - init_C of the init_C centres are split,
// centre j becoming c_j - eps in place and c_j + eps at index init_C + j, with
// eps = (1, 1, 1).
__global__ void __launch_bounds__(kMaxK) k_lbg_stage(const JobDev* __restrict__ jobs)
{
    const JobDev& J = jobs[blockIdx.x];
    double* __restrict__ c = gp(J.centers);
    const int m = int(J.init_C);
    if (m == 0) {
        if (threadIdx.x < 3) c[threadIdx.x] = 0.0;
        return;
    }
    const int split = J.K - m;
    for (int t = threadIdx.x; t < 3 * split; t += blockDim.x) {
        const double v = c[t];
        c[3 * m + t] = v + kLbgEps;
        c[t] = v - kLbgEps;
    }
}

cq_status launch_lbg_stage(const JobDev* jobs, int B, hipStream_t s)
{
    CQ_TIMED_LAUNCH("k_lbg_stage", s, k_lbg_stage<<<B, kMaxK, 0, s>>>(jobs));
    return CQ_OK;
}

cq_status launch_var(const JobDev* jobs, const int* maps, int B, int tiles, int groups, hipStream_t s)
{
    CQ_TIMED_LAUNCH("k_var_tiles", s, k_var_tiles<<<tiles, kVarThreads, 0, s>>>(jobs, maps + kMapVarTiles * (B + 1), B));
    CQ_TIMED_LAUNCH("k_var_pick", s, k_var_pick<<<B, kVarThreads, 0, s>>>(jobs));
    CQ_TIMED_LAUNCH("k_var_find", s, k_var_find<<<groups, kVarThreads, 0, s>>>(jobs, maps + kMapVarGroups * (B + 1), B));
    return CQ_OK;
}

int var_tile_count(int64_t n) { return int(var_tiles(n)); }

cq_status launch_sff(const JobDev* jobs, int B, hipStream_t s)
{
    CQ_TIMED_LAUNCH("k_sff", s, k_sff<<<B, kSffThreads, 0, s>>>(jobs));
    return CQ_OK;
}

// SFF subset size: max(K, ceil(2 K ln K)), at most n (at most kSffMax).
int64_t sff_subset(int32_t K, int64_t n)
{
    int64_t L = int64_t(ceil(2.0 * double(K) * log(double(K))));
    if (L < K) L = K;
    return L < n ? L : n;
}

cq_status launch_forgy(const JobDev* jobs, int B, hipStream_t s)
{
    CQ_TIMED_LAUNCH("k_forgy", s, k_forgy<<<B, 64, 0, s>>>(jobs));
    return CQ_OK;
}

// One cooperative launch running the teams of `B` jobs (`total` blocks) with
// the kernel `variant` (see coop_capacity).
cq_status launch_init_coop(const JobDev* jobs, const int* map, int B, int total, int variant, hipStream_t s)
{
    void* args[] = {(void*)&jobs, (void*)&map, (void*)&B};
    timer_begin("k_init_coop", s);
    const hipError_t e = hipLaunchCooperativeKernel(coop_kernel(variant), dim3(total), dim3(kInitThreads), args,
                                                    coop_dyn_lds(variant), s);
    timer_end("k_init_coop", s);
    if (e != hipSuccess) {
        set_error("cooperative init launch failed: %s", hipGetErrorString(e));
        return CQ_EDEVICE;
    }
    return CQ_OK;
}

}  // namespace cq
