// Host check of the serving engine's pool allocator against a byte-map model:
// random allocations and releases; every granted range must be free in the
// model and be the lowest-offset free run of the rounded size (first fit),
// a refusal must mean no such run exists, and the used byte count and the
// free-range invariants must agree with the model after every operation.
#include <cstdio>
#include <cstdint>
#include <vector>

#include "pool.h"

static uint64_t next(uint64_t& s)  // splitmix64 as a plain input generator
{
    s += 0x9E3779B97F4A7C15ull;
    uint64_t z = s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

int main()
{
    const size_t align = 16, units = 512, total = units * align + 7;  // a ragged tail the pool must drop
    long bad = 0, ops = 0, refusals = 0;
    for (uint64_t seed = 1; seed <= 200; ++seed) {
        uint64_t s = seed;
        cq::ExtentPool pool(total, align);
        std::vector<int> owner(units, 0);  // model: 0 free, else allocation id
        struct A { size_t off, bytes; int id; };
        std::vector<A> live;
        int id = 0;
        if (pool.total() != units * align) ++bad;
        for (int step = 0; step < 2000; ++step) {
            ++ops;
            if (live.empty() || next(s) % 3 != 0) {
                const size_t bytes = 1 + next(s) % (align * 64);
                const size_t need = (bytes + align - 1) / align;
                // first free run of `need` units in the model
                long want = -1;
                for (size_t u = 0, run = 0; u < units; ++u) {
                    run = owner[u] ? 0 : run + 1;
                    if (run == need) { want = long(u + 1 - need); break; }
                }
                size_t off = 0;
                const bool ok = pool.alloc(bytes, &off);
                if (ok != (want >= 0) || (ok && off != size_t(want) * align)) {
                    if (bad < 5) std::printf("seed %llu step %d: alloc(%zu) -> %d @%zu, model %ld\n",
                                             (unsigned long long)seed, step, bytes, int(ok), off, want);
                    ++bad;
                    continue;
                }
                if (!ok) { ++refusals; continue; }
                ++id;
                for (size_t u = 0; u < need; ++u) owner[off / align + u] = id;
                live.push_back({off, bytes, id});
            } else {
                const size_t i = next(s) % live.size();
                const A a = live[i];
                live[i] = live.back();
                live.pop_back();
                pool.release(a.off, a.bytes);
                for (size_t u = 0; u < (a.bytes + align - 1) / align; ++u) {
                    if (owner[a.off / align + u] != a.id) ++bad;
                    owner[a.off / align + u] = 0;
                }
            }
            // used bytes, largest free run and number of maximal free runs
            size_t used = 0, largest = 0, runs = 0;
            for (size_t u = 0, run = 0; u < units; ++u) {
                if (owner[u]) { used += align; run = 0; continue; }
                if (run == 0) ++runs;
                ++run;
                largest = run * align > largest ? run * align : largest;
            }
            if (pool.used() != used || pool.largest_free() != largest || pool.free_ranges() != runs) {
                if (bad < 5) std::printf("seed %llu step %d: used %zu/%zu largest %zu/%zu ranges %zu/%zu\n",
                                         (unsigned long long)seed, step, pool.used(), used, pool.largest_free(),
                                         largest, pool.free_ranges(), runs);
                ++bad;
            }
        }
    }
    std::printf("%ld operations, %ld refusals, %ld mismatches\n", ops, refusals, bad);
    return bad == 0 && refusals > 0 ? 0 : 1;
}
