// Host check of the launch plan of the cooperative k-means++ / max-min
// initializations: on random batches every job with colours is placed once,
// a launch holds at most its kernel's co-resident blocks, every job's
// colours fit its blocks, a team never exceeds the block cap, and a launch of
// single-block jobs only exists once every launch of teams is full; plus two
// plans worked out by hand.
#include <cstdio>
#include <cstdint>
#include <vector>

#include "coop_plan.h"

static uint64_t next(uint64_t& s)  // splitmix64 as a plain input generator
{
    s += 0x9E3779B97F4A7C15ull;
    uint64_t z = s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static const int R[5] = {4, 8, 16, 24, 32};
static const int kCap = 256, kMaxBlocks = 256, kThreads = 1024;
static const int64_t C = 32 * 1024;

static int fail(const char* what, int t)
{
    std::printf("FAIL %s (batch %d)\n", what, t);
    return 1;
}

int main()
{
    const int cap[5] = {kCap, kCap, kCap, kCap, kCap};
    std::vector<cq::CoopLaunch> plan;
    // worked by hand: a team of 2 blocks at R = 32 takes the two small jobs
    // into the same launch, largest first
    cq::plan_coop_with({40000, 100, 200}, R, cap, 5, kCap, kMaxBlocks, kThreads, plan);
    if (plan.size() != 1 || plan[0].variant != 32 || plan[0].jobs != std::vector<int>{0, 2, 1} ||
        plan[0].blocks != std::vector<int>{2, 1, 1})
        return fail("teams and small jobs in one launch", -1);
    // no small jobs: the smallest R whose teams fit (R = 4: 10 + 18 blocks)
    cq::plan_coop_with({40000, 70000}, R, cap, 5, kCap, kMaxBlocks, kThreads, plan);
    if (plan.size() != 1 || plan[0].variant != 4 || plan[0].jobs != std::vector<int>{1, 0} ||
        plan[0].blocks != std::vector<int>{18, 10})
        return fail("smallest R without small jobs", -2);
    uint64_t seed = 7;
    for (int t = 0; t < 2000; ++t) {
        const int B = 1 + int(next(seed) % 600);
        std::vector<int64_t> n(B);
        for (int j = 0; j < B; ++j) {
            const uint64_t r = next(seed) % 100;
            if (r < 5) n[j] = 0;
            else if (r < 60) n[j] = 1 + int64_t(next(seed) % C);                    // one block
            else if (r < 97) n[j] = C + 1 + int64_t(next(seed) % (40 * C));         // a team
            else n[j] = kMaxBlocks * C + 1 + int64_t(next(seed) % (4 * kMaxBlocks * C));  // global D^2
        }
        cq::plan_coop_with(n, R, cap, 5, kCap, kMaxBlocks, kThreads, plan);
        std::vector<int> seen(B, 0);
        bool small_only = false, team_not_full = false;
        for (const cq::CoopLaunch& w : plan) {
            if (w.jobs.empty() || w.jobs.size() != w.blocks.size()) return fail("launch shape", t);
            int used = 0;
            bool small = true, team = false;
            for (size_t i = 0; i < w.jobs.size(); ++i) {
                const int j = w.jobs[i], g = w.blocks[i];
                if (j < 0 || j >= B || n[j] <= 0) return fail("job without colours placed", t);
                ++seen[j];
                used += g;
                if (g < 1 || g > kMaxBlocks) return fail("team size", t);
                if (w.variant == 0) {
                    if (n[j] <= kMaxBlocks * C) return fail("global D^2 kernel for a job that fits registers", t);
                } else if (int64_t(g) * w.variant * kThreads < n[j]) {
                    return fail("colours do not fit the blocks", t);
                }
                small = small && n[j] <= C;
                team = team || n[j] > C;
            }
            if (used > kCap) return fail("launch above capacity", t);
            if (w.variant != 0 && small) small_only = true;
            if (w.variant != 0 && team && used < kCap) team_not_full = true;
        }
        for (int j = 0; j < B; ++j)
            if (seen[j] != (n[j] > 0 ? 1 : 0)) return fail("job placed other than once", t);
        if (small_only && team_not_full) return fail("single-block launch while a team launch has room", t);
    }
    std::printf("ok\n");
    return 0;
}
