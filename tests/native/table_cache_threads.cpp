// Eight threads look up eleven keys in a four-entry LruCache (the per-sequence
// cache of step tables) and use what they get while the others evict it.
// Every value must stay intact while held, be built only on a miss, and be
// destroyed exactly once, after its last holder let go. Built with g++ and
// ThreadSanitizer by tests/test_table_cache.py (no GPU involved).
#include <atomic>
#include <chrono>
#include <cstdio>
#include <thread>
#include <vector>

#include "../../paper_1506_05393_amd/csrc/table_cache.h"

namespace {
std::atomic<int> live{0}, built{0}, destroyed{0};

struct Value {
  int key;
  std::vector<int> payload;
  explicit Value(int k) : key(k), payload(4096, k) { ++live; }
  ~Value() {
    for (int x : payload)
      if (x != key) std::abort();
    payload.assign(payload.size(), -1);
    --live;
    ++destroyed;
  }
};
}  // namespace

int main() {
  mrf::LruCache<std::pair<unsigned long, int>, Value> cache(4);
  std::atomic<int> bad{0};
  std::vector<std::thread> th;
  for (int t = 0; t < 8; ++t) {
    th.emplace_back([&, t]() {
      for (int it = 0; it < 4000; ++it) {
        const int k = (it * 7 + t * 3) % 11;
        std::shared_ptr<const Value> v;
        const int rc = cache.get(std::make_pair((unsigned long)k * 977u, k % 3),
                                 [&](std::shared_ptr<Value>* out) {
                                   ++built;
                                   *out = std::make_shared<Value>(k);
                                   return 0;
                                 },
                                 &v);
        if (rc != 0 || !v || v->key != k) ++bad;
        if (cache.size() > 4) ++bad;
        // use it while other threads evict it
        if (it % 64 == 0) std::this_thread::sleep_for(std::chrono::microseconds(50));
        long s = 0;
        for (int x : v->payload) s += x;
        if (s != (long)k * (long)v->payload.size()) ++bad;
      }
      // a failed build inserts nothing
      std::shared_ptr<const Value> none;
      if (cache.get(std::make_pair(999999ul, 0), [](std::shared_ptr<Value>*) { return 7; },
                    &none) != 7 ||
          none)
        ++bad;
    });
  }
  for (auto& x : th) x.join();
  const int before_clear = live.load();
  cache.clear();
  std::printf("built %d destroyed %d live before clear %d after %d bad %d\n", built.load(),
              destroyed.load(), before_clear, live.load(), bad.load());
  if (bad.load() != 0 || live.load() != 0 || before_clear > 4 ||
      built.load() != destroyed.load() || built.load() < 11)
    return 1;
  return 0;
}
