// Host check of the serving pool allocator (compiled with g++ by
// test_serve_host.py): first fit, merging on release, peak, and random
// alloc/release sequences that never overlap or exceed the capacity.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "pool_alloc.h"

#define CHECK(c)                                              \
  do {                                                        \
    if (!(c)) {                                               \
      std::printf("check failed line %d: %s\n", __LINE__, #c); \
      return 1;                                               \
    }                                                         \
  } while (0)

int main() {
  using trstmi::PoolAllocator;
  {
    PoolAllocator a(4096);
    uint64_t x, y, z, t;
    CHECK(a.alloc(1000, &x) && x == 0);  // rounds to 1024
    CHECK(a.alloc(1024, &y) && y == 1024);
    CHECK(a.alloc(2048, &z) && z == 2048);
    CHECK(!a.alloc(1, &t) && a.used() == 4096 && a.peak() == 4096);
    a.release(y, 1024);
    CHECK(!a.alloc(2048, &t));  // only 1024 free
    a.release(x, 1000);
    CHECK(a.free_ranges().size() == 1 && a.free_ranges().begin()->first == 0 &&
          a.free_ranges().begin()->second == 2048);  // merged with the neighbour
    CHECK(a.alloc(2048, &t) && t == 0);
    a.release(0, 2048);
    a.release(z, 2048);
    CHECK(a.free_ranges().size() == 1 && a.free_ranges().begin()->second == 4096 && a.used() == 0);
    CHECK(!a.alloc(0, &t));
    PoolAllocator b(1000);  // capacity rounds down to whole 256-byte units
    CHECK(b.capacity() == 768 && !b.alloc(1000, &t) && b.alloc(768, &t) && t == 0);
  }
  {
    std::mt19937_64 rnd(0);
    PoolAllocator a(1 << 20);
    std::vector<std::pair<uint64_t, uint64_t>> live;
    for (int it = 0; it < 20000; ++it) {
      if (!live.empty() && (rnd() & 1)) {
        const size_t k = rnd() % live.size();
        a.release(live[k].first, live[k].second);
        live.erase(live.begin() + k);
      } else {
        const uint64_t size = 1 + rnd() % (1 << 16);
        uint64_t off;
        if (a.alloc(size, &off)) {
          CHECK(off % 256 == 0 && off + PoolAllocator::round(size) <= a.capacity());
          for (auto& l : live)
            CHECK(off + PoolAllocator::round(size) <= l.first || l.first + PoolAllocator::round(l.second) <= off);
          live.push_back({off, size});
        }
      }
      CHECK(a.used() <= a.capacity() && a.peak() <= a.capacity());
    }
    for (auto& l : live) a.release(l.first, l.second);
    CHECK(a.used() == 0 && a.free_ranges().size() == 1 && a.free_ranges().begin()->second == a.capacity());
  }
  std::printf("ok\n");
  return 0;
}
