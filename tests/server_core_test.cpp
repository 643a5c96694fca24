// CPU test of the serving runtime's host state (mhm_server_core.h): the
// factor arena, admission and completion bookkeeping, checked against a
// plain model after every operation.  Built by test_server_core_cpu.py with
// the address and undefined-behaviour sanitizers; prints "ok" on success.
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <random>
#include <set>
#include <string>
#include <vector>

#include "../paper_1703_10435_amd/csrc/mhm_server_core.h"

using namespace mhm_srv;

static int g_fail = 0;
#define CHECK(c)                                                      \
  do {                                                                \
    if (!(c)) {                                                       \
      std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
      ++g_fail;                                                       \
    }                                                                 \
  } while (0)

static void arena_ok(const Cache& c) {
  std::string why;
  const bool ok = c.check(&why);
  if (!ok) std::fprintf(stderr, "arena inconsistent: %s\n", why.c_str());
  CHECK(ok);
}

struct Q {
  Key key;
  bool keyed;
  int s, l;
  uint64_t ticket;
};

// Random allocations, touches and erasures with pins: the arena stays
// consistent, eviction takes only unpinned entries, and allocation fails only
// when the unpinned entries plus the free space cannot hold the request.
static void test_arena_random() {
  std::mt19937_64 rng(7);
  Cache c;
  c.init(1000);
  std::vector<Key> live;
  for (int step = 0; step < 20000; ++step) {
    const int op = (int)(rng() % 4);
    if (op == 0 || live.empty()) {
      const size_t bytes = 1 + rng() % 120;
      const Key k{rng() | 1, rng()};
      size_t pinned_bytes = 0;
      for (const auto& kv : c.map)
        if (kv.second.pins > 0) pinned_bytes += kv.second.bytes;
      std::set<uint64_t> before;
      for (const auto& kv : c.map) before.insert(kv.first.hi);
      size_t off = 0;
      std::set<uint64_t> unpinned;
      for (const auto& kv : c.map)
        if (kv.second.pins == 0) unpinned.insert(kv.first.hi);
      const bool got = c.alloc(bytes, off);
      // the entries that vanished (evicted, whether or not the allocation
      // succeeded) were all unpinned; the pinned ones are all still there
      for (const auto& kv : c.map) before.erase(kv.first.hi);
      for (uint64_t h : before) CHECK(unpinned.count(h) == 1);
      for (auto it = live.begin(); it != live.end();) {
        if (before.count(it->hi)) it = live.erase(it);
        else ++it;
      }
      CHECK(c.evictions >= before.size());
      if (got) {
        c.insert(k, off, bytes);
        live.push_back(k);
      } else {
        // everything unpinned was evicted, and no free block is large enough
        for (const auto& kv : c.map) CHECK(kv.second.pins > 0);
        for (const auto& fb : c.free_) CHECK(fb.second < bytes);
        CHECK(c.used == pinned_bytes);
      }
    } else if (op == 1) {
      const Key k = live[rng() % live.size()];
      Entry& e = c.map.at(k);
      if (rng() % 2) e.pins++;
      else if (e.pins > 0) e.pins--;
    } else if (op == 2) {
      const Key k = live[rng() % live.size()];
      c.touch(k);
      CHECK(c.lru.front() == k);
    } else {
      const size_t i = rng() % live.size();
      c.erase(live[i]);
      live.erase(live.begin() + (long)i);
    }
    arena_ok(c);
    CHECK(c.map.size() == live.size());
  }
  // unpin and erase everything: one free block again
  for (const Key& k : live) c.erase(k);
  arena_ok(c);
  CHECK(c.used == 0 && c.free_.size() == 1 && c.free_.begin()->second == 1000);
}

// LRU order decides the victim: the least recently used unpinned entry.
static void test_lru_victim() {
  Cache c;
  c.init(300);
  size_t off;
  const Key a{1, 1}, b{2, 2}, d{3, 3};
  CHECK(c.alloc(100, off)); c.insert(a, off, 100);
  CHECK(c.alloc(100, off)); c.insert(b, off, 100);
  CHECK(c.alloc(100, off)); c.insert(d, off, 100);
  for (auto* k : {&a, &b, &d}) c.map.at(*k).pins = 0;
  c.touch(a);                       // order now a, d, b (b least recent)
  const Key e{4, 4};
  CHECK(c.alloc(100, off));
  c.insert(e, off, 100);
  CHECK(c.map.count(b) == 0 && c.map.count(a) == 1 && c.map.count(d) == 1);
  CHECK(c.evictions == 1);
  c.map.at(a).pins = 1;             // pinned entries are never victims
  c.map.at(d).pins = 1;
  CHECK(c.alloc(100, off) == false);   // e is pinned too (inserted with one pin)
  CHECK(c.map.count(e) == 1 && c.map.size() == 3);
  arena_ok(c);
}

static size_t fbytes(int s) { return (size_t)s * 10; }

// Admission: arrival order, duplicate keys deferred, hits pinned, a full
// arena stops admission, and completion makes fresh keyed factors valid.
static void test_admission_and_completion() {
  Cache c;
  c.init(1000);
  std::deque<Q> queue;
  uint64_t t = 1;
  auto push = [&](uint64_t key, int s) { queue.push_back(Q{Key{key, key}, key != 0, s, 1, t++}); };
  push(11, 10);   // fresh keyed
  push(11, 10);   // same key: deferred to a later launch
  push(0, 20);    // unkeyed: scratch region
  push(12, 30);   // fresh keyed
  const Limits lim{64, 1 << 20, 1 << 20, true};
  std::vector<Q> taken;
  Admitted a;
  int n = admit(c, queue, lim, fbytes, taken, a);
  CHECK(n == 3);
  CHECK(queue.size() == 1 && queue.front().key.hi == 11);
  CHECK(taken[0].ticket == 1 && taken[1].ticket == 3 && taken[2].ticket == 4);
  CHECK(a.state[0] == 0 && a.fresh[0] && a.keyed[0] && !a.keyed[1] && a.fresh[2]);
  CHECK(c.used == 100 + 200 + 300);
  arena_ok(c);
  // while the launch runs, the deferred request stays queued (factor not valid yet)
  std::vector<Q> t2;
  Admitted a2;
  CHECK(admit(c, queue, lim, fbytes, t2, a2) == 0 && queue.size() == 1);
  // completion: element 0 ok, element 2 (key 12) failed
  settle(c, a, 0, true, 0);
  settle(c, a, 1, true, 0);
  settle(c, a, 2, true, 7);
  CHECK(c.map.count(Key{11, 11}) == 1 && c.map.at(Key{11, 11}).valid && c.map.at(Key{11, 11}).pins == 0);
  CHECK(c.map.count(Key{~0ull, 3}) == 0);    // scratch region freed
  CHECK(c.map.count(Key{12, 12}) == 0);      // failed element: factor dropped
  CHECK(c.used == 100);
  arena_ok(c);
  // the deferred request now reuses the stored factor
  n = admit(c, queue, lim, fbytes, t2, a2);
  CHECK(n == 1 && a2.state[0] == 1 && a2.hits == 1 && a2.foff[0] == c.map.at(Key{11, 11}).off);
  CHECK(c.map.at(Key{11, 11}).pins == 1);
  settle(c, a2, 0, true, 0);
  CHECK(c.map.at(Key{11, 11}).pins == 0 && c.map.at(Key{11, 11}).valid);
  arena_ok(c);
  // admission by memory: requests that do not fit wait, in order
  push(21, 50);   // 500 bytes
  push(22, 50);   // 500 bytes: only 400 free + the unpinned 100 evictable
  push(23, 1);
  n = admit(c, queue, lim, fbytes, taken, a);
  CHECK(n == 1 && taken[0].key.hi == 21 && queue.size() == 2 && queue.front().key.hi == 22);
  arena_ok(c);
  // batch and capacity limits
  const Limits small{1, 1 << 20, 1 << 20, true};
  settle(c, a, 0, true, 0);
  n = admit(c, queue, small, fbytes, taken, a);
  CHECK(n == 1 && queue.size() == 1);
  settle(c, a, 0, true, 0);
  const Limits tiny{64, 0, 1 << 20, true};
  CHECK(admit(c, queue, tiny, fbytes, taken, a) == 0 && queue.size() == 1);
  arena_ok(c);
}

// A failed launch: its fresh factors are dropped (never valid), reused ones
// are kept and unpinned, scratch regions freed; a later request with the
// same key factors again instead of reusing a factor that was never computed.
static void test_failed_launch() {
  Cache c;
  c.init(1000);
  std::deque<Q> queue;
  queue.push_back(Q{Key{5, 5}, true, 10, 1, 1});
  std::vector<Q> taken;
  Admitted a;
  const Limits lim{64, 1 << 20, 1 << 20, true};
  CHECK(admit(c, queue, lim, fbytes, taken, a) == 1);
  settle(c, a, 0, true, 0);   // key 5 stored and valid
  queue.push_back(Q{Key{5, 5}, true, 10, 1, 2});   // hit
  queue.push_back(Q{Key{6, 6}, true, 20, 1, 3});   // fresh
  queue.push_back(Q{Key{0, 0}, false, 30, 1, 4});  // scratch
  queue.push_back(Q{Key{6, 6}, true, 20, 1, 5});   // deferred (same key as 3)
  CHECK(admit(c, queue, lim, fbytes, taken, a) == 3);
  CHECK(a.state[0] == 1 && a.fresh[1] && !a.keyed[2]);
  for (size_t k = 0; k < 3; ++k) settle(c, a, k, false, -5);
  CHECK(c.map.count(Key{5, 5}) == 1 && c.map.at(Key{5, 5}).valid && c.map.at(Key{5, 5}).pins == 0);
  CHECK(c.map.count(Key{6, 6}) == 0);
  CHECK(c.map.size() == 1 && c.used == 100);
  arena_ok(c);
  // the deferred request with key 6 is admitted fresh (state 0), not as a hit
  CHECK(admit(c, queue, lim, fbytes, taken, a) == 1);
  CHECK(taken[0].ticket == 5 && a.state[0] == 0 && a.fresh[0]);
  settle(c, a, 0, true, 0);
  CHECK(c.map.at(Key{6, 6}).valid);
  arena_ok(c);
}

// Reuse off: every request gets a scratch region, keys are ignored.
static void test_reuse_off() {
  Cache c;
  c.init(1000);
  std::deque<Q> queue;
  queue.push_back(Q{Key{9, 9}, true, 10, 1, 1});
  queue.push_back(Q{Key{9, 9}, true, 10, 1, 2});
  std::vector<Q> taken;
  Admitted a;
  const Limits lim{64, 1 << 20, 1 << 20, false};
  CHECK(admit(c, queue, lim, fbytes, taken, a) == 2);
  CHECK(!a.keyed[0] && !a.keyed[1] && a.state[0] == 0 && a.state[1] == 0);
  settle(c, a, 0, true, 0);
  settle(c, a, 1, true, 0);
  CHECK(c.map.empty() && c.used == 0);
  arena_ok(c);
}

int main() {
  test_arena_random();
  test_lru_victim();
  test_admission_and_completion();
  test_failed_launch();
  test_reuse_off();
  if (g_fail) {
    std::fprintf(stderr, "%d checks failed\n", g_fail);
    return 1;
  }
  std::printf("ok\n");
  return 0;
}
