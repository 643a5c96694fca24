// Host-side state of the serving runtime, in plain C++ (no HIP): the factor
// arena (first-fit free list with coalescing, LRU eviction of unpinned
// entries), admission of queued requests into a launch, and the factor
// bookkeeping when a launch completes or fails.  mhm_server.hip drives it
// from its worker thread under the server lock; on its own it builds into a
// CPU test under the address and undefined-behaviour sanitizers.
#pragma once

#include <cstddef>
#include <cstdint>
#include <deque>
#include <iterator>
#include <list>
#include <map>
#include <string>
#include <unordered_map>
#include <vector>

namespace mhm_srv {

inline int n_of(int s) { return (s + 1) * (s + 2) / 2; }

struct Key {
  uint64_t hi, lo;
  bool operator==(const Key& o) const { return hi == o.hi && lo == o.lo; }
};
struct KeyHash {
  size_t operator()(const Key& k) const { return k.hi * 0x9E3779B97F4A7C15ull ^ k.lo; }
};
// The factor region of an unkeyed request (or of any request with reuse
// off): private to that request and freed when it completes.
inline Key scratch_key(uint64_t ticket) { return Key{~0ull, ticket}; }

struct Entry {
  size_t off = 0, bytes = 0;
  int pins = 0;          // launches in flight that use the factor
  bool valid = false;    // a factor has been stored (set at completion)
  std::list<Key>::iterator lru;
};

struct Cache {
  size_t cap = 0;
  std::map<size_t, size_t> free_;   // offset -> bytes
  std::unordered_map<Key, Entry, KeyHash> map;
  std::list<Key> lru;               // front = most recently used
  size_t used = 0;
  uint64_t evictions = 0;

  void init(size_t bytes) {
    cap = bytes;
    used = 0;
    free_.clear();
    map.clear();
    lru.clear();
    if (bytes) free_[0] = bytes;
  }
  void release(size_t off, size_t bytes) {
    auto it = free_.emplace(off, bytes).first;
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
    used -= bytes;
  }
  bool take(size_t bytes, size_t& off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        off = it->first;
        const size_t rest = it->second - bytes;
        free_.erase(it);
        if (rest) free_[off + bytes] = rest;
        used += bytes;
        return true;
      }
    }
    return false;
  }
  void erase(const Key& k) {
    auto it = map.find(k);
    if (it == map.end()) return;
    release(it->second.off, it->second.bytes);
    lru.erase(it->second.lru);
    map.erase(it);
  }
  // room for `bytes`, evicting least recently used unpinned factors
  bool alloc(size_t bytes, size_t& off) {
    if (bytes == 0 || bytes > cap) return false;
    while (!take(bytes, off)) {
      auto victim = lru.end();
      for (auto it = lru.rbegin(); it != lru.rend(); ++it) {
        if (map.at(*it).pins == 0) {
          victim = std::prev(it.base());
          break;
        }
      }
      if (victim == lru.end()) return false;
      const Key k = *victim;
      erase(k);
      ++evictions;
    }
    return true;
  }
  // a new pinned entry at the front of the LRU order
  void insert(const Key& k, size_t off, size_t bytes) {
    Entry en;
    en.off = off;
    en.bytes = bytes;
    en.pins = 1;
    lru.push_front(k);
    en.lru = lru.begin();
    map[k] = en;
  }
  void touch(const Key& k) {
    Entry& e = map.at(k);
    lru.erase(e.lru);
    lru.push_front(k);
    e.lru = lru.begin();
  }
  // Consistency of the arena (for tests): free blocks inside the arena,
  // sorted, disjoint and coalesced; entries disjoint from them and from each
  // other; free plus used bytes make the capacity; the LRU list holds every
  // entry once.
  bool check(std::string* why = nullptr) const {
    auto bad = [&](const char* m) {
      if (why) *why = m;
      return false;
    };
    size_t free_bytes = 0, end = 0;
    bool first = true;
    for (const auto& kv : free_) {
      if (kv.second == 0 || kv.first + kv.second > cap) return bad("free block outside the arena");
      if (!first && kv.first <= end) return bad(kv.first < end ? "free blocks overlap" : "free blocks not coalesced");
      end = kv.first + kv.second;
      first = false;
      free_bytes += kv.second;
    }
    size_t used_bytes = 0;
    std::map<size_t, size_t> taken;
    for (const auto& kv : map) {
      const Entry& e = kv.second;
      if (e.pins < 0) return bad("negative pin count");
      if (e.bytes == 0 || e.off + e.bytes > cap) return bad("entry outside the arena");
      taken[e.off] = e.bytes;
      used_bytes += e.bytes;
      auto f = free_.upper_bound(e.off);
      if (f != free_.end() && f->first < e.off + e.bytes) return bad("entry overlaps a free block");
      if (f != free_.begin()) {
        --f;
        if (f->first + f->second > e.off) return bad("entry overlaps a free block");
      }
      if (!(*e.lru == kv.first)) return bad("entry's LRU position names another key");
    }
    size_t prev_end = 0;
    first = true;
    for (const auto& kv : taken) {
      if (!first && kv.first < prev_end) return bad("entries overlap");
      prev_end = kv.first + kv.second;
      first = false;
    }
    if (used_bytes != used) return bad("used bytes disagree with the entries");
    if (free_bytes + used != cap) return bad("free plus used bytes differ from the capacity");
    if (lru.size() != map.size()) return bad("LRU list and entry map differ in size");
    return true;
  }
};

// One launch's requests as admitted: per request, the factor state passed to
// the kernel (0 factor and store, 1 reuse), the factor's arena offset, the
// entry that holds it, and whether this launch created that entry.
struct Admitted {
  std::vector<int8_t> state;
  std::vector<size_t> foff;
  std::vector<Key> pinned;
  std::vector<uint8_t> keyed, fresh;
  int64_t hits = 0;
  void clear() {
    state.clear();
    foff.clear();
    pinned.clear();
    keyed.clear();
    fresh.clear();
    hits = 0;
  }
};

struct Limits {
  int max_batch;
  int64_t cap_tri, cap_rhs;   // sub-triangles and solution entries one launch holds
  bool reuse;
};

// Moves the queued requests that fit into `taken`, in arrival order, and
// pins (or allocates) their factors.  A request is left in the queue when its
// key is already being factored (by this launch or a running one: the next
// launch reuses the factor); admission stops at the first request whose
// factor finds no room after evicting every unpinned factor, or that would
// exceed the launch's capacity.  Q has fields key, keyed, s, l, ticket;
// factor_bytes(s) is the size of one factor.
template <class Q, class FactorBytes>
int admit(Cache& cache, std::deque<Q>& queue, const Limits& lim, FactorBytes factor_bytes, std::vector<Q>& taken,
          Admitted& out) {
  taken.clear();
  out.clear();
  int64_t tri = 0, rhs = 0;
  std::unordered_map<Key, int, KeyHash> in_batch;
  for (auto it = queue.begin(); it != queue.end() && (int)taken.size() < lim.max_batch;) {
    const Q& q = *it;
    const int n = n_of(q.s), r = 3 * (q.l + 1) + 1;
    if (tri + (int64_t)q.s * q.s > lim.cap_tri || rhs + (int64_t)n * r > lim.cap_rhs) break;
    const bool keyed = lim.reuse && q.keyed;
    const Key k = keyed ? q.key : scratch_key(q.ticket);
    int8_t st = 0;
    size_t off = 0;
    bool fresh = false;
    if (keyed) {
      auto e = cache.map.find(k);
      if (in_batch.count(k) || (e != cache.map.end() && !e->second.valid)) {
        ++it;   // being factored: a later launch reuses the factor
        continue;
      }
      if (e != cache.map.end()) {
        st = 1;
        off = e->second.off;
        e->second.pins++;
        cache.touch(k);
        out.hits++;
      } else {
        const size_t bytes = factor_bytes(q.s);
        if (!cache.alloc(bytes, off)) break;   // no memory: wait for running launches
        cache.insert(k, off, bytes);
        fresh = true;
        in_batch[k] = 1;
      }
    } else {
      const size_t bytes = factor_bytes(q.s);
      if (!cache.alloc(bytes, off)) break;
      cache.insert(k, off, bytes);
      fresh = true;
    }
    out.state.push_back(st);
    out.foff.push_back(off);
    out.pinned.push_back(k);
    out.keyed.push_back(keyed);
    out.fresh.push_back(fresh);
    tri += (int64_t)q.s * q.s;
    rhs += (int64_t)n * r;
    taken.push_back(std::move(*it));
    it = queue.erase(it);
  }
  return (int)taken.size();
}

// Factor bookkeeping for request k of a finished or failed launch: the
// entry is unpinned; a keyed factor this launch stored becomes valid when
// the launch ran and the element reported info 0.  Otherwise the entry is
// erased once no launch uses it - a scratch region, a factor the launch
// created but did not store (failed launch, failed element), or a reused
// factor whose element failed - so no later request ever reuses a factor
// that was never computed.  A reused factor of a failed launch is kept.
inline void settle(Cache& cache, const Admitted& a, size_t k, bool launch_ok, int info) {
  auto it = cache.map.find(a.pinned[k]);
  if (it == cache.map.end()) return;
  Entry& e = it->second;
  e.pins--;
  bool drop;
  if (!a.keyed[k]) drop = true;
  else if (!launch_ok) drop = a.fresh[k] != 0;
  else if (info == 0) {
    e.valid = true;
    drop = false;
  } else {
    drop = true;
  }
  if (drop && e.pins == 0) cache.erase(a.pinned[k]);
}

}  // namespace mhm_srv
