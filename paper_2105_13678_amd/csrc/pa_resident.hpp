// Accounting of the serving loop's resident device memory: the twiddle
// tables of each transform length and the seed transforms of each (session,
// output class, transform shape) stay on the device between requests, inside
// one fixed budget.  A set is placed first-fit in the budget's byte range;
// when a new set does not fit, sets that no admitted request holds are
// evicted, least recently used first, until it does.  Pure host logic (no
// device calls), so the same class is exercised by a CPU test.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <map>
#include <tuple>
#include <vector>

namespace pa {

struct ResidentKey {
    uint32_t kind;     // 0: twiddle tables, 1: seed transforms
    uint32_t session;  // seed transforms: the session
    uint64_t gamma;    // seed transforms: the output class
    uint32_t shape;    // transform shape (limb width << 8 | length key)
    bool operator<(const ResidentKey &o) const {
        return std::tie(kind, session, gamma, shape) < std::tie(o.kind, o.session, o.gamma, o.shape);
    }
    bool operator==(const ResidentKey &o) const {
        return kind == o.kind && session == o.session && gamma == o.gamma && shape == o.shape;
    }
};

class ResidentCache {
public:
    struct Entry {
        ResidentKey key;
        size_t off = 0, bytes = 0;
        uint32_t refs = 0;    // admitted requests holding the set
        uint64_t stamp = 0;   // last use (larger is more recent)
        void *data = nullptr; // owner's handle (device address of the set, its ready event, ...)
        void *aux = nullptr;
    };

    explicit ResidentCache(size_t budget) : budget_(budget) {}

    size_t budget() const { return budget_; }
    size_t used() const {
        size_t u = 0;
        for (const auto &kv : sets_) u += kv.second.bytes;
        return u;
    }
    size_t count() const { return sets_.size(); }

    // The set with this key, marked used now, or nullptr.
    Entry *find(const ResidentKey &k) {
        auto it = sets_.find(k);
        if (it == sets_.end()) return nullptr;
        it->second.stamp = ++clock_;
        return &it->second;
    }

    // Room for a new set of `bytes`: evicts unreferenced sets, least recently
    // used first, until a first-fit place exists (their entries are appended
    // to *evicted so the owner can free what they point to).  Returns the new
    // entry (refs 0), or nullptr when the set cannot be placed now because
    // the sets in use leave no room; nothing is evicted then.  A set larger
    // than the whole budget never fits.
    Entry *insert(const ResidentKey &k, size_t bytes, std::vector<Entry> *evicted) {
        if (bytes > budget_ || sets_.count(k)) return nullptr;
        bytes = align(bytes);
        size_t off = 0;
        if (!place(bytes, nullptr, &off)) {
            // would evicting every unreferenced set make room?  then evict in LRU order until it does
            std::vector<const Entry *> idle;
            for (const auto &kv : sets_)
                if (kv.second.refs == 0) idle.push_back(&kv.second);
            if (!place(bytes, &idle, &off)) return nullptr;
            std::vector<std::pair<uint64_t, ResidentKey>> order;
            for (const Entry *e : idle) order.emplace_back(e->stamp, e->key);
            std::sort(order.begin(), order.end());  // oldest use first
            for (const auto &o : order) {
                auto it = sets_.find(o.second);
                if (evicted) evicted->push_back(it->second);
                sets_.erase(it);
                if (place(bytes, nullptr, &off)) break;
            }
        }
        Entry &e = sets_[k];
        e.key = k;
        e.off = off;
        e.bytes = bytes;
        e.refs = 0;
        e.stamp = ++clock_;
        return &e;
    }

    void acquire(Entry *e) {
        ++e->refs;
        e->stamp = ++clock_;
    }
    void release(Entry *e) {
        if (e->refs) --e->refs;
    }
    // Remove a set outright (e.g. its build failed); it must not be held.
    void erase(const ResidentKey &k) { sets_.erase(k); }

    // Every set, for the owner's clean-up.
    std::vector<Entry> all() const {
        std::vector<Entry> v;
        for (const auto &kv : sets_) v.push_back(kv.second);
        return v;
    }

private:
    static size_t align(size_t x) { return (x + 255) & ~(size_t)255; }

    // First-fit offset for `bytes` among the current sets, ignoring those in
    // `skip` (as if evicted).
    bool place(size_t bytes, const std::vector<const Entry *> *skip, size_t *off) const {
        std::map<size_t, size_t> used;
        for (const auto &kv : sets_) {
            bool skipped = false;
            if (skip)
                for (const Entry *e : *skip) skipped |= e == &kv.second;
            if (!skipped) used[kv.second.off] = kv.second.bytes;
        }
        size_t start = 0;
        for (const auto &u : used) {
            if (u.first >= start && u.first - start >= bytes) break;
            start = align(u.first + u.second);
        }
        if (start > budget_ || budget_ - start < bytes) return false;
        *off = start;
        return true;
    }

    size_t budget_;
    uint64_t clock_ = 0;
    std::map<ResidentKey, Entry> sets_;
};

}  // namespace pa
