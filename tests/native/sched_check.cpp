// Host-only checks of the serving executor's pool allocator and batch
// planning (csrc/gf_sched.hpp), built with the address and undefined-behaviour
// sanitizers by tests/test_sched_native.py.  Exit status 0 when every check
// holds; the first failure is printed.
#include <stdio.h>
#include <stdlib.h>

#include <iterator>
#include <map>
#include <random>
#include <vector>

#include "gf_sched.hpp"

#define CHECK(c)                                                           \
    do {                                                                   \
        if (!(c)) {                                                        \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            return 1;                                                      \
        }                                                                  \
    } while (0)

static int pool_checks(unsigned seed) {
    std::mt19937_64 g(seed);
    const size_t budget = 1 << 20;
    gfs::Pool p;
    p.reset(budget);
    std::map<size_t, size_t> live;  // offset -> bytes
    for (int step = 0; step < 20000; ++step) {
        bool do_alloc = live.empty() || (g() % 3 != 0);
        if (do_alloc) {
            size_t bytes = gfs::kAlign * (1 + g() % 64);
            size_t off;
            bool ok = p.alloc(bytes, &off);
            if (ok) {
                CHECK(off % gfs::kAlign == 0);
                CHECK(off + bytes <= budget);
                auto nxt = live.lower_bound(off);
                if (nxt != live.end()) CHECK(off + bytes <= nxt->first);
                if (nxt != live.begin()) {
                    auto prv = std::prev(nxt);
                    CHECK(prv->first + prv->second <= off);
                }
                live[off] = bytes;
            } else {
                // first fit: no free block is large enough
                for (auto& b : p.freel) CHECK(b.size < bytes);
            }
        } else {
            auto it = live.begin();
            std::advance(it, g() % live.size());
            p.release(it->first, it->second);
            live.erase(it);
        }
        size_t held = 0;
        for (auto& kv : live) held += kv.second;
        CHECK(held == p.held);
        // free list sorted, coalesced, disjoint from the live blocks
        size_t free_total = 0;
        for (size_t i = 0; i < p.freel.size(); ++i) {
            free_total += p.freel[i].size;
            CHECK(p.freel[i].size > 0);
            if (i + 1 < p.freel.size()) CHECK(p.freel[i].off + p.freel[i].size < p.freel[i + 1].off);
        }
        CHECK(free_total + held == budget);
    }
    for (auto& kv : live) p.release(kv.first, kv.second);
    CHECK(p.held == 0 && p.freel.size() == 1 && p.freel[0].off == 0 && p.freel[0].size == budget);
    return 0;
}

static int plan_checks(unsigned seed) {
    std::mt19937_64 g(seed);
    std::vector<gfs::SchedReq> reqs(40);
    std::vector<gfs::SchedReq*> active;
    for (size_t i = 0; i < reqs.size(); ++i) {
        gfs::SchedReq& r = reqs[i];
        r.id = i;
        r.n = 1 + (int)(g() % 70000);
        r.spp = 1 + (int)(g() % 4);
        r.multiple = (g() & 1) != 0;
        r.bytes = gfs::request_bytes(r.n, 1, r.spp);
        r.off = 0;
        r.next_ray = r.rays_done = 0;
        active.push_back(&r);
    }
    std::vector<int> covered(reqs.size(), 0);
    for (int batch = 0;; ++batch) {
        std::vector<double> before;
        for (auto* r : active) before.push_back(gfs::remaining_work(r));
        std::vector<gfs::TileRef> t = gfs::plan_batch(active, 4096, 1 + (int)(g() % 16));
        if (t.empty()) break;
        CHECK(batch < 100000);
        double last = -1.0;
        for (size_t k = 0; k < t.size(); ++k) {
            CHECK(t[k].count >= 1 && t[k].count <= 4096);
            size_t i = t[k].r->id;
            // tiles continue each request where it left off
            CHECK(t[k].first == covered[i]);
            covered[i] += t[k].count;
            // requests enter the batch in order of remaining work
            if (k == 0 || t[k].r != t[k - 1].r) {
                CHECK(before[i] >= last);
                last = before[i];
            }
        }
    }
    for (size_t i = 0; i < reqs.size(); ++i) CHECK(covered[i] == reqs[i].n && reqs[i].next_ray == reqs[i].n);
    return 0;
}

int main() {
    for (unsigned s = 1; s <= 5; ++s) {
        if (pool_checks(s)) return 1;
        if (plan_checks(s)) return 1;
    }
    printf("sched checks passed\n");
    return 0;
}
