// Randomised check of the session's arena allocator against a byte-map model:
// regions never overlap, stay inside the arena and are 256-byte aligned; after
// every free the allocator's free space equals the model's; when everything is
// freed one region spans the whole arena again (frees coalesce).
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../paper_2605_29604_amd/csrc/arena.hpp"

int main() {
    using tcmis::Arena;
    const size_t cap = 1 << 20;   // 4096 granules
    Arena a;
    a.init(cap + 100);            // the tail below a granule is not usable
    if (a.capacity() != cap || a.largest_free() != cap) { std::puts("bad init"); return 1; }
    std::vector<int> owner(cap / 256, -1);
    struct R { size_t off, bytes; };
    std::vector<R> live;
    unsigned long long x = 88172645463325252ull;
    auto rnd = [&]() { x ^= x << 13; x ^= x >> 7; x ^= x << 17; return x; };
    int allocs = 0, refusals = 0;
    for (int step = 0; step < 200000; ++step) {
        if (live.empty() || rnd() % 100 < 55) {
            const size_t want = 1 + rnd() % (rnd() % 8 == 0 ? 200000 : 5000);
            size_t off = 0;
            if (!a.alloc(want, &off)) {
                // refusal is only allowed when no free run of granules is long enough
                size_t g = (want + 255) / 256, run = 0, best = 0;
                for (int o : owner) { run = o < 0 ? run + 1 : 0; best = run > best ? run : best; }
                if (best >= g) { std::printf("refused %zu with a free run of %zu granules\n", want, best); return 1; }
                ++refusals;
                continue;
            }
            if (off % 256 || off + tcmis::round256(want) > cap) { std::puts("misplaced region"); return 1; }
            for (size_t gi = off / 256; gi < (off + tcmis::round256(want)) / 256; ++gi) {
                if (owner[gi] >= 0) { std::puts("overlap"); return 1; }
                owner[gi] = step;
            }
            live.push_back({off, want});
            ++allocs;
        } else {
            const size_t i = rnd() % live.size();
            const R r = live[i];
            live[i] = live.back();
            live.pop_back();
            a.release(r.off, r.bytes);
            for (size_t gi = r.off / 256; gi < (r.off + tcmis::round256(r.bytes)) / 256; ++gi) owner[gi] = -1;
            size_t used = 0;
            for (int o : owner) used += o >= 0 ? 256 : 0;
            if (used != a.used()) { std::puts("used bytes disagree"); return 1; }
        }
    }
    for (const R& r : live) a.release(r.off, r.bytes);
    if (a.used() != 0 || a.largest_free() != cap) { std::puts("frees did not coalesce"); return 1; }
    std::printf("ok %d allocations %d refusals\n", allocs, refusals);
    return 0;
}
