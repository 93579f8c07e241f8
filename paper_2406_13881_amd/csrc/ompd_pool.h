// Host-side bookkeeping of the serving loop (no device code): the first-fit
// byte pool that admits requests against the device-memory budget and the
// pinned staging pool, and the rule that forms a step from the pending
// requests.  Kept apart from the HIP sources so that it can be unit-tested
// on the CPU.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <deque>
#include <map>

namespace ompd_pool {

inline size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

// First-fit allocator over a byte range (256-byte granularity, coalescing).
struct Pool {
    size_t size = 0, used = 0;
    std::map<size_t, size_t> free_;   // offset -> bytes
    void init(size_t n)
    {
        size = n & ~(size_t)255;
        used = 0;
        free_.clear();
        if (size) free_[0] = size;
    }
    bool alloc(size_t n, size_t& off)
    {
        n = a256(std::max<size_t>(n, 1));
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            off = it->first;
            const size_t rest = it->second - n, o2 = it->first + n;
            free_.erase(it);
            if (rest) free_[o2] = rest;
            used += n;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t n)
    {
        n = a256(std::max<size_t>(n, 1));
        used -= n;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

// Launch tables of one step, laid out in the step's table region: the CFG
// descriptors, the tiles, the pass items (each array 256-byte aligned), the
// launch's work counters, then (pinned side only) each CFG's status words.
struct TableBytes {
    size_t cfg = 0, tiles = 0, items = 0, counters = 256, info = 0;
    size_t device() const { return cfg + tiles + items + counters; }
    size_t pinned() const { return cfg + tiles + items + info; }
};
inline TableBytes table_bytes(size_t n_cfgs, size_t n_tiles, size_t n_items, size_t cfg_sz, size_t tile_sz,
                              size_t item_sz, size_t info_sz)
{
    TableBytes t;
    t.cfg = a256(cfg_sz * n_cfgs);
    t.tiles = a256(tile_sz * std::max<size_t>(n_tiles, 1));
    t.items = a256(item_sz * std::max<size_t>(n_items, 1));
    t.info = a256(info_sz * n_cfgs);
    return t;
}
// What one request adds to a step's tables, with room for the alignment of
// every array: the sum over a step's requests bounds the step's tables.
inline size_t request_table_bytes(size_t n_tiles, size_t n_items, size_t cfg_sz, size_t tile_sz, size_t item_sz,
                                  size_t info_sz)
{
    return cfg_sz + tile_sz * n_tiles + item_sz * n_items + info_sz;
}
constexpr size_t TABLE_SLACK = 5 * 256;   // alignment of the four arrays, the work counters

// How many of the pending requests (front first) the next step takes: as many
// as fit a table region of `region` bytes, at most `max_reqs`.  A request that
// does not fit an empty region is never admitted (the caller checks at
// submit), so a non-empty queue always yields a step of at least one.
inline int take_step(const std::deque<size_t>& pending_table_bytes, size_t region, int max_reqs)
{
    size_t used = TABLE_SLACK;
    int k = 0;
    for (size_t b : pending_table_bytes) {
        if (k >= max_reqs || used + b > region) break;
        used += b;
        ++k;
    }
    return k;
}

}  // namespace ompd_pool
