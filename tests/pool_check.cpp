// Randomized check of the serving engines' arena allocator (pool.h) against a
// reference model that tracks every 256-byte unit: blocks lie inside the
// range, never overlap, start on a unit, come from the lowest free run that
// fits (first fit), and releasing everything leaves one free run; a request of
// at most total() bytes fits an empty pool whatever the range's length.
// Built and run by tests/test_pool.py with the host compiler; prints "ok".
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "pool.h"

namespace {

int fail(const char* what, unsigned long a, unsigned long b) {
    std::printf("FAIL %s %lu %lu\n", what, a, b);
    return 1;
}

}  // namespace

int main() {
    std::mt19937_64 rng(2508);
    // every range length around a few unit boundaries: the empty pool takes
    // any request up to total()
    for (size_t len = 0; len < 2048; ++len) {
        lvs::Pool p;
        p.init(len);
        if (p.total() != (len / 256) * 256) return fail("total", len, p.total());
        size_t off = 1;
        if (p.total() && (!p.alloc(p.total(), &off) || off != 0)) return fail("fit total", len, off);
        lvs::Pool q;
        q.init(len);
        if (q.total() && !q.alloc(q.total() - 255, &off)) return fail("fit near total", len, off);
        if (q.alloc(q.total() + 1, &off)) return fail("over total", len, off);
    }
    for (int trial = 0; trial < 200; ++trial) {
        const size_t units = 1 + rng() % 64;
        const size_t len = units * 256 + rng() % 256;
        lvs::Pool p;
        p.init(len);
        std::vector<int> owner(units, -1);   // unit -> live block id
        struct Block {
            size_t off, bytes;
            bool live;
        };
        std::vector<Block> blocks;
        for (int op = 0; op < 400; ++op) {
            const bool do_alloc = blocks.empty() || rng() % 3 != 0;
            if (do_alloc) {
                const size_t bytes = 1 + rng() % (units * 256 / 3 + 1);
                const size_t need = (bytes + 255) / 256;
                // the model's first fit: the lowest start of `need` free units,
                // which is the start of the lowest free run that holds them
                // (so a pool that failed to merge adjacent free runs differs)
                long want = -1;
                for (size_t u = 0; u + need <= units && want < 0; ++u) {
                    bool free_run = true;
                    for (size_t k = u; k < u + need; ++k) free_run = free_run && owner[k] < 0;
                    if (free_run) want = long(u);
                }
                size_t off = 0;
                const bool got = p.alloc(bytes, &off);
                if (got != (want >= 0)) return fail("alloc success", bytes, size_t(want));
                if (!got) continue;
                if (off % 256) return fail("alignment", off, bytes);
                const size_t u0 = off / 256;
                if (u0 + need > units) return fail("inside range", off, bytes);
                for (size_t k = u0; k < u0 + need; ++k)
                    if (owner[k] >= 0) return fail("overlap", off, k);
                if (u0 != size_t(want)) return fail("first fit", u0, size_t(want));
                for (size_t k = u0; k < u0 + need; ++k) owner[k] = int(blocks.size());
                blocks.push_back({off, bytes, true});
            } else {
                std::vector<size_t> live;
                for (size_t b = 0; b < blocks.size(); ++b)
                    if (blocks[b].live) live.push_back(b);
                if (live.empty()) continue;
                Block& b = blocks[live[rng() % live.size()]];
                p.release(b.off, b.bytes);
                b.live = false;
                for (size_t k = b.off / 256; k < b.off / 256 + (b.bytes + 255) / 256; ++k) owner[k] = -1;
            }
        }
        for (Block& b : blocks)
            if (b.live) p.release(b.off, b.bytes);
        size_t off = 1;
        if (!p.alloc(units * 256, &off) || off != 0) return fail("coalesced", units, off);
    }
    std::printf("ok\n");
    return 0;
}
