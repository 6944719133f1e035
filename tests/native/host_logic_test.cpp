// CPU test of the allocation table and the shadow pool allocator (built with
// sanitizers by tests/test_abi.py).  Checks against a brute-force model.
#include <cassert>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <vector>

#include "../../paper_1310_0901_amd/csrc/host_logic.h"
#include "xfercheck.h"

#define CHECK(x)                                                     \
    do {                                                             \
        if (!(x)) {                                                  \
            std::printf("FAILED %s at line %d\n", #x, __LINE__);     \
            std::exit(1);                                            \
        }                                                            \
    } while (0)

static void table_basics()
{
    xc::AllocTable t;
    CHECK(t.check_insert(100, 0) == CG_EINVAL);
    CHECK(t.check_insert(~0ull - 3, 8) == CG_EINVAL);
    CHECK(t.check_insert(~0ull - 8, 8) == CG_OK);
    CHECK(t.check_insert(100, 50) == CG_OK);
    t.insert(100, 50, 0);
    CHECK(t.check_insert(150, 10) == CG_OK);    // adjacent is fine
    CHECK(t.check_insert(149, 10) == CG_EOVERLAP);
    CHECK(t.check_insert(90, 11) == CG_EOVERLAP);
    CHECK(t.check_insert(90, 10) == CG_OK);
    CHECK(t.check_insert(0, 1000) == CG_EOVERLAP);
    t.insert(150, 10, 256);
    uint64_t base = 0;
    CHECK(t.find(149, &base) && base == 100);
    CHECK(t.find(150, &base) && base == 150);
    CHECK(!t.find(160, &base));
    CHECK(!t.find(99, &base));
    xc::AllocEntry e;
    CHECK(t.erase(101, &e) == CG_ENOTFOUND);    // not a base
    CHECK(t.erase(100, &e) == CG_OK && e.size == 50);
    CHECK(t.erase(100, &e) == CG_ENOTFOUND);    // double free
    CHECK(t.size() == 1);
}

static void pool_random()
{
    std::mt19937_64 rng(5);
    xc::PoolAllocator p(1 << 20, 256);
    std::map<uint64_t, uint64_t> live;   // off -> size
    for (int it = 0; it < 20000; ++it) {
        if (live.empty() || rng() % 3) {
            const uint64_t sz = 1 + rng() % 20000;
            uint64_t off;
            if (p.alloc(sz, &off)) {
                CHECK(off % 256 == 0);
                CHECK(off + p.rounded(sz) <= p.capacity());
                // disjoint from every live block
                auto nx = live.lower_bound(off);
                if (nx != live.end()) CHECK(off + p.rounded(sz) <= nx->first);
                if (nx != live.begin()) {
                    auto pv = std::prev(nx);
                    CHECK(pv->first + p.rounded(pv->second) <= off);
                }
                live[off] = sz;
            }
        } else {
            auto it2 = live.begin();
            std::advance(it2, rng() % live.size());
            p.release(it2->first, it2->second);
            live.erase(it2);
        }
        uint64_t used = 0;
        for (auto &kv : live) used += p.rounded(kv.second);
        CHECK(used == p.used());
    }
    for (auto &kv : live) p.release(kv.first, kv.second);
    CHECK(p.used() == 0);
    CHECK(p.free_blocks() == 1);   // everything merged back
    uint64_t off;
    CHECK(p.alloc(1 << 20, &off) && off == 0);
    CHECK(!p.alloc(1, &off));       // exhausted
}

int main()
{
    table_basics();
    pool_random();
    std::printf("all host logic checks passed\n");
    return 0;
}
