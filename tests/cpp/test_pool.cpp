// CPU unit test of the serving loop's bookkeeping (paper_2406_13881_amd/csrc/ompd_pool.h).
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "ompd_pool.h"

using namespace ompd_pool;

#define CHECK(c)                                                                 \
    do {                                                                         \
        if (!(c)) {                                                              \
            std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
            std::exit(1);                                                        \
        }                                                                        \
    } while (0)

int main()
{
    // a budget filled exactly: 16 requests of 64 KiB in 1 MiB
    Pool p;
    p.init(1 << 20);
    std::vector<size_t> off(16);
    for (int i = 0; i < 16; ++i) CHECK(p.alloc(64 << 10, off[i]));
    CHECK(p.used == p.size);
    size_t x = 0;
    CHECK(!p.alloc(1, x));                      // full: pushes back
    p.release(off[5], 64 << 10);
    CHECK(!p.alloc((64 << 10) + 1, x));         // one byte more than the hole
    CHECK(p.alloc(64 << 10, x) && x == off[5]); // exactly the hole
    for (int i = 0; i < 16; ++i) p.release(off[i], 64 << 10);
    CHECK(p.used == 0 && p.free_.size() == 1 && p.free_.begin()->second == p.size);   // coalesced
    // odd sizes round to 256 bytes; fragmentation then a full coalesce
    std::vector<size_t> o2;
    size_t t = 0;
    while (p.alloc(1000, t)) o2.push_back(t);
    CHECK(o2.size() == (1 << 20) / 1024);
    for (size_t i = 0; i < o2.size(); i += 2) p.release(o2[i], 1000);
    CHECK(!p.alloc(2048, t));                   // every hole is 1 KiB
    for (size_t i = 1; i < o2.size(); i += 2) p.release(o2[i], 1000);
    CHECK(p.used == 0 && p.free_.size() == 1);

    // steps: requests whose tables fill a region exactly all go in one step
    const size_t region = 8 << 20;
    std::deque<size_t> q;
    const size_t each = (region - TABLE_SLACK) / 4;
    for (int i = 0; i < 4; ++i) q.push_back(each);
    CHECK(take_step(q, region, 256) == 4);
    q.push_back(1);
    CHECK(take_step(q, region, 256) == 4);      // the fifth waits for the next step
    q.clear();
    q.push_back(region - TABLE_SLACK);          // the largest admissible request
    CHECK(take_step(q, region, 256) == 1);
    q.clear();
    for (int i = 0; i < 1000; ++i) q.push_back(100);
    CHECK(take_step(q, region, 256) == 256);    // capped by requests per step
    q.clear();
    CHECK(take_step(q, region, 256) == 0);
    // the bound holds: the tables of any taken set fit the region
    for (int n = 1; n <= 64; ++n) {
        const size_t cfg = 304, tile = 16, item = 16, info = 64;
        std::deque<size_t> rq;
        for (int i = 0; i < n; ++i) rq.push_back(request_table_bytes(3, 257, cfg, tile, item, info));
        const int k = take_step(rq, 64 << 10, 256);
        const TableBytes tb = table_bytes(k, 3 * k, 257 * k, cfg, tile, item, info);
        CHECK(tb.device() <= (size_t)(64 << 10) && tb.pinned() <= (size_t)(64 << 10));
    }
    std::printf("pool and step rules ok\n");
    return 0;
}
