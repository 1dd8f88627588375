// Host check of the serving loop's output allocator (smap::Arena): random
// allocation and release sequences against a byte-map model.  Checks that
// every allocation is inside the arena, 256-aligned, disjoint from the live
// ones, that first fit returns the lowest free run that fits, and that
// releasing everything merges the free list back into one range.
#include "../../paper_2208_11617_amd/csrc/smap_serve.hpp"

#include <cstdio>
#include <random>
#include <vector>

int main()
{
    long bad = 0;
    std::mt19937_64 rng(2208);
    for (int trial = 0; trial < 200; ++trial) {
        const uint64_t size = 256ull * (1 + rng() % 512);
        smap::Arena a(size);
        const uint64_t units = size / 256;
        std::vector<int> used(units, 0);                 // the model, one flag per 256-byte unit
        std::vector<std::pair<uint64_t, uint64_t>> live; // (offset, bytes)
        for (int op = 0; op < 400; ++op) {
            if (live.empty() || rng() % 3 != 0) {
                const uint64_t bytes = 1 + rng() % (size / 4 + 1);
                const uint64_t need = smap::Arena::round(bytes) / 256;
                // first fit in the model: lowest start with `need` free units
                int64_t want = -1;
                for (uint64_t s = 0, run = 0; s < units; ++s) {
                    run = used[s] ? 0 : run + 1;
                    if (run == need) { want = (int64_t)(s + 1 - need); break; }
                }
                uint64_t off = 0;
                const bool ok = a.alloc(bytes, &off);
                if (ok != (want >= 0)) { ++bad; std::printf("trial %d: alloc %llu ok=%d model=%lld\n", trial, (unsigned long long)bytes, ok, (long long)want); continue; }
                if (!ok) continue;
                if (off % 256 != 0 || off + need * 256 > size || (int64_t)(off / 256) != want) {
                    ++bad;
                    std::printf("trial %d: alloc %llu at %llu, first fit %lld\n", trial, (unsigned long long)bytes,
                                (unsigned long long)off, (long long)want);
                }
                for (uint64_t u = off / 256; u < off / 256 + need && u < units; ++u) {
                    if (used[u]) { ++bad; std::printf("trial %d: overlap at unit %llu\n", trial, (unsigned long long)u); }
                    used[u] = 1;
                }
                live.push_back({off, bytes});
            } else {
                const size_t k = rng() % live.size();
                const auto [off, bytes] = live[k];
                a.release(off, bytes);
                for (uint64_t u = off / 256; u < off / 256 + smap::Arena::round(bytes) / 256; ++u) used[u] = 0;
                live[k] = live.back();
                live.pop_back();
            }
        }
        for (const auto &[off, bytes] : live) a.release(off, bytes);
        uint64_t off = 0;
        if (!a.alloc(size, &off) || off != 0) { ++bad; std::printf("trial %d: free list not merged\n", trial); }
    }
    std::printf("bad=%ld\n", bad);
    return bad != 0;
}
