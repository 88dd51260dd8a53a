// Host-only checks of the serving loop's resident-set accounting
// (paper_2105_13678_amd/csrc/pa_resident.hpp): first-fit placement inside
// the budget, least-recently-used eviction of sets no request holds, held
// sets never evicted, nothing evicted when the new set cannot be placed.
// Built and run by tests/test_host_checks.py; prints "ok" on success.
#include <cstdio>
#include <cstdlib>

#include "pa_resident.hpp"

using pa::ResidentCache;
using pa::ResidentKey;

static int failures = 0;
#define CHECK(c)                                                      \
    do {                                                              \
        if (!(c)) {                                                   \
            std::printf("FAILED line %d: %s\n", __LINE__, #c);        \
            ++failures;                                               \
        }                                                             \
    } while (0)

static ResidentKey K(uint32_t i) { return ResidentKey{1, i, 1000 + i, 7}; }

int main() {
    {  // fill, then LRU eviction in stamp order until a first-fit place exists
        ResidentCache C(4096);
        std::vector<ResidentCache::Entry> ev;
        ResidentCache::Entry *a = C.insert(K(0), 1024, &ev);
        ResidentCache::Entry *b = C.insert(K(1), 1024, &ev);
        ResidentCache::Entry *c = C.insert(K(2), 1024, &ev);
        CHECK(a && b && c && ev.empty());
        CHECK(a->off == 0 && b->off == 1024 && c->off == 2048 && C.used() == 3072);
        CHECK(C.find(K(0)) == a);  // A is now the most recently used
        ResidentCache::Entry *d = C.insert(K(3), 2048, &ev);
        // B (oldest) goes first; [1024, 2048) + [3072, 4096) is not contiguous,
        // so C goes too; D lands at 1024
        CHECK(d && ev.size() == 2 && ev[0].key == K(1) && ev[1].key == K(2));
        CHECK(d->off == 1024 && C.count() == 2 && C.find(K(0)) && !C.find(K(1)) && !C.find(K(2)));
    }
    {  // held sets are never evicted; no room -> nothing evicted, nullptr
        ResidentCache C(4096);
        std::vector<ResidentCache::Entry> ev;
        ResidentCache::Entry *a = C.insert(K(0), 2048, &ev);
        ResidentCache::Entry *b = C.insert(K(1), 2048, &ev);
        C.acquire(a);
        C.acquire(b);
        CHECK(C.insert(K(2), 256, &ev) == nullptr && ev.empty() && C.count() == 2);
        C.release(b);
        ResidentCache::Entry *c = C.insert(K(2), 1024, &ev);
        CHECK(c && ev.size() == 1 && ev[0].key == K(1) && C.find(K(0)) == a && a->refs == 1);
        CHECK(c->off == 2048);
        C.release(a);
        CHECK(a->refs == 0);
        C.release(a);  // releasing below zero keeps zero
        CHECK(a->refs == 0);
    }
    {  // a set larger than the budget never fits; duplicates are refused
        ResidentCache C(4096);
        std::vector<ResidentCache::Entry> ev;
        CHECK(C.insert(K(0), 4097, &ev) == nullptr);
        CHECK(C.insert(K(1), 4096, &ev) != nullptr);
        CHECK(C.insert(K(1), 256, &ev) == nullptr);
        CHECK(C.used() == 4096);
    }
    {  // sizes are rounded to 256 bytes; first fit reuses the lowest gap
        ResidentCache C(2048);
        std::vector<ResidentCache::Entry> ev;
        ResidentCache::Entry *a = C.insert(K(0), 100, &ev);
        ResidentCache::Entry *b = C.insert(K(1), 300, &ev);
        CHECK(a->bytes == 256 && b->off == 256 && b->bytes == 512);
        C.erase(K(0));
        ResidentCache::Entry *c = C.insert(K(2), 200, &ev);
        CHECK(c && c->off == 0 && ev.empty());
    }
    {  // a long random run: placements never overlap and stay in the budget
        ResidentCache C(1 << 20);
        std::srand(12345);
        std::vector<ResidentCache::Entry> ev;
        for (int step = 0; step < 20000; ++step) {
            const uint32_t id = std::rand() % 64;
            if (ResidentCache::Entry *e = C.find(K(id))) {
                if (std::rand() % 2) C.acquire(e); else C.release(e);
                continue;
            }
            ev.clear();
            C.insert(K(id), (size_t)(1 + std::rand() % 8) * 20000, &ev);
            for (const auto &x : ev) CHECK(x.refs == 0);
            const auto all = C.all();
            size_t used = 0;
            for (size_t i = 0; i < all.size(); ++i) {
                CHECK(all[i].off + all[i].bytes <= C.budget());
                used += all[i].bytes;
                for (size_t j = i + 1; j < all.size(); ++j)
                    CHECK(all[i].off + all[i].bytes <= all[j].off || all[j].off + all[j].bytes <= all[i].off);
            }
            CHECK(used == C.used() && used <= C.budget());
        }
    }
    if (failures) return 1;
    std::printf("ok\n");
    return 0;
}
