// Randomised check of the job service's pool sub-allocator (host code only):
// blocks never overlap, stay inside the pool and 256-byte aligned, the used
// byte count matches the live blocks, and freeing everything coalesces the
// pool back into one free range.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "pool.h"

int main() {
    using stk::PoolAllocator;
    std::mt19937_64 rng(12345);
    for (int trial = 0; trial < 50; ++trial) {
        const uint64_t size = (1 + rng() % 64) << 20;
        PoolAllocator P(size);
        struct B { uint64_t off, bytes; };
        std::vector<B> live;
        uint64_t used = 0, high = 0;
        for (int step = 0; step < 2000; ++step) {
            if (live.empty() || rng() % 3) {
                const uint64_t bytes = 1 + rng() % (size / 8);
                uint64_t off = 0;
                if (P.alloc(bytes, &off)) {
                    const uint64_t rb = PoolAllocator::round_up(bytes);
                    if (off % 256 || off + rb > P.size()) { std::puts("out of range"); return 1; }
                    for (const B &b : live)
                        if (off < b.off + PoolAllocator::round_up(b.bytes) && b.off < off + rb) {
                            std::puts("overlap");
                            return 1;
                        }
                    live.push_back({off, bytes});
                    used += rb;
                    if (used > high) high = used;
                } else if (P.largest_free() >= PoolAllocator::round_up(bytes)) {
                    std::puts("refused a block that fits");
                    return 1;
                }
            } else {
                const size_t k = rng() % live.size();
                P.release(live[k].off, live[k].bytes);
                used -= PoolAllocator::round_up(live[k].bytes);
                live.erase(live.begin() + k);
            }
            if (P.used() != used || P.high_water() != high) { std::puts("accounting"); return 1; }
        }
        for (const B &b : live) P.release(b.off, b.bytes);
        if (P.used() != 0 || P.free_ranges() != 1 || P.largest_free() != P.size()) {
            std::puts("no coalesce");
            return 1;
        }
    }
    std::puts("pool ok");
    return 0;
}
