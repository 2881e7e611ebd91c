// Launch plan of the cooperative k-means++ and max-min initializations of a
// batch (host code only, so that it can be checked without a GPU).
#pragma once

#include <cstdint>
#include <algorithm>
#include <vector>

namespace cq {

struct CoopLaunch {
    int variant = 32;
    std::vector<int> jobs;
    std::vector<int> blocks;
};

// The plan: n[j] colours of job j (0: none); R[0 .. nv - 1] the register
// variants' colours per thread, ascending (R[nv - 1] = 32); cap[v] the
// co-resident blocks of variant v and cap0 those of the kernel that keeps D^2
// in global memory (a launch's variant 0); max_blocks the blocks of a team at
// most; threads the threads per block (1024, so C = R[nv - 1] x threads =
// 32768 colours per block).  Jobs are taken largest first, in three classes,
// each in launches that fit the co-resident capacity of the kernel that runs
// them:
//  - at most C colours: one register block each (a team of one block
//    exchanges nothing through memory), with the smallest R that holds the
//    launch's largest job;
//  - up to max_blocks x C colours: teams of ceil(n / (R threads)) register
//    blocks, with the smallest R for which the launch's teams fit the
//    capacity (fewer colours per thread, less of each round's work per
//    block), R = 32 when only that fits; while jobs of the first class are
//    left, such a launch keeps R = 32 and fills the CUs its teams leave with
//    them (largest first), so that they need fewer launches of their own;
//  - more: max_blocks blocks of the kernel that keeps D^2 in global memory.
inline void plan_coop_with(const std::vector<int64_t>& n, const int* R, const int* cap, int nv, int cap0,
                           int max_blocks, int threads, std::vector<CoopLaunch>& plan)
{
    plan.clear();
    std::vector<int> order;
    for (int j = 0; j < int(n.size()); ++j)
        if (n[j] > 0) order.push_back(j);
    if (order.empty()) return;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return n[a] > n[b]; });
    const int kBig = nv - 1;
    const int64_t cmax = int64_t(R[kBig]) * threads;
    auto blocks_at = [](int64_t cnt, int64_t per) { return int((cnt + per - 1) / per); };
    auto cls = [&](int j) { return n[j] > cmax * max_blocks ? 0 : (n[j] > cmax ? 1 : 2); };
    auto fit = [&](int64_t cnt) {  // smallest variant holding cnt colours in one block
        int v = 0;
        while (v < kBig && int64_t(R[v]) * threads < cnt) ++v;
        return v;
    };
    // single-block jobs not yet placed: the tail of `order`, largest first,
    // from `small`; a launch of teams takes them into the CUs its teams leave
    std::vector<char> placed(n.size(), 0);
    size_t small = order.size();
    while (small > 0 && cls(order[small - 1]) == 2) --small;
    size_t q = 0;
    while (q < order.size()) {
        if (placed[order[q]]) {
            ++q;
            continue;
        }
        const int c = cls(order[q]);
        CoopLaunch w;
        const int v0 = c == 2 ? fit(n[order[q]]) : kBig;  // the launch's largest job comes first
        const int capw = c == 0 ? cap0 : cap[v0];
        int used = 0;
        while (q < order.size() && cls(order[q]) == c) {
            const int j = order[q];
            if (placed[j]) {
                ++q;
                continue;
            }
            int g = 1;
            if (c == 0) g = max_blocks < capw ? max_blocks : capw;
            if (c == 1) g = blocks_at(n[j], cmax);
            if (used > 0 && used + g > capw) break;
            w.jobs.push_back(j);
            w.blocks.push_back(g);
            used += g;
            ++q;
        }
        w.variant = c == 0 ? 0 : R[v0];
        bool smalls_left = false;
        for (size_t i = small; i < order.size() && !smalls_left; ++i) smalls_left = !placed[order[i]];
        if (c == 1 && !smalls_left) {
            // the smallest R whose teams fit
            for (int v = 0; v < kBig; ++v) {
                const int64_t per = int64_t(R[v]) * threads;
                int need = 0;
                bool ok = true;
                for (int j : w.jobs) {
                    const int g = blocks_at(n[j], per);
                    ok = ok && g <= max_blocks;
                    need += g;
                }
                if (ok && need <= cap[v]) {
                    w.variant = R[v];
                    for (size_t i = 0; i < w.jobs.size(); ++i) w.blocks[i] = blocks_at(n[w.jobs[i]], per);
                    break;
                }
            }
        }
        if (c == 1 && smalls_left) {
            // R = 32 (the fewest blocks per team) and the CUs left over to
            // single-block jobs, largest first: they then need no launch of
            // their own
            for (size_t i = small; i < order.size() && used < capw; ++i) {
                const int j = order[i];
                if (placed[j]) continue;
                w.jobs.push_back(j);
                w.blocks.push_back(1);
                placed[j] = 1;
                ++used;
            }
        }
        plan.push_back(std::move(w));
    }
}

}  // namespace cq
