// Host-only checks of the device memory cache (lrx_cache.h) with a fake
// mapper that hands out address ranges without backing memory.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <vector>

#include "lrx_cache.h"

namespace {

struct FakeMapper {
  size_t capacity = (size_t)300 << 30;
  size_t in_use = 0;
  uintptr_t next = (uintptr_t)1 << 40;
  int maps = 0, unmaps = 0, quiesces = 0;
  std::map<uintptr_t, size_t> live;
  void* map(size_t bytes) {
    if (in_use + bytes > capacity) return nullptr;
    const uintptr_t p = next;
    next += (bytes + ((size_t)2 << 20) - 1) / ((size_t)2 << 20) * ((size_t)2 << 20) + ((size_t)2 << 20);
    live[p] = bytes;
    in_use += bytes;
    ++maps;
    return (void*)p;
  }
  void unmap(void* p) {
    auto it = live.find((uintptr_t)p);
    if (it == live.end()) { std::printf("FAIL unmap of an unmapped segment\n"); std::exit(1); }
    in_use -= it->second;
    live.erase(it);
    ++unmaps;
  }
  void quiesce() { ++quiesces; }
};

using Cache = lrx::BlockCache<FakeMapper>;
int failures = 0;
#define CHECK(c, ...) do { if (!(c)) { std::printf("FAIL line %d: ", __LINE__); std::printf(__VA_ARGS__); std::printf("\n"); ++failures; } } while (0)

// Structural invariants: blocks tile each segment, no two neighbouring free
// blocks, live blocks hold their requests, byte accounting matches.
void validate(Cache& C, const std::map<uintptr_t, size_t>& live_req) {
  size_t used = 0, mapped = 0;
  std::map<size_t, size_t> seg_size;
  std::map<size_t, std::pair<size_t, bool>> last;   // per segment: end offset, last block free
  size_t live_seen = 0;
  C.walk([&](size_t seg, size_t off, size_t size, bool free) {
    auto it = last.find(seg);
    const size_t expect = it == last.end() ? 0 : it->second.first;
    CHECK(off == expect, "segment %zu: block at %zu, expected %zu", seg, off, expect);
    if (it != last.end()) CHECK(!(free && it->second.second), "segment %zu: two free neighbours at %zu", seg, off);
    CHECK(size % Cache::kAlign == 0 && off % Cache::kAlign == 0, "block not aligned");
    last[seg] = {off + size, free};
    seg_size[seg] = off + size;
    if (!free) { used += size; ++live_seen; }
  });
  for (auto& s : seg_size) mapped += s.second;
  CHECK(used == C.used(), "used %zu != cache used %zu", used, C.used());
  CHECK(mapped == C.mapped(), "mapped %zu != cache mapped %zu", mapped, C.mapped());
  CHECK(mapped == C.mapper().in_use, "mapped %zu != mapper %zu", mapped, C.mapper().in_use);
  CHECK(live_seen == live_req.size(), "live blocks %zu != requests %zu", live_seen, live_req.size());
  // live requests are disjoint and aligned
  uintptr_t end = 0;
  for (auto& r : live_req) {
    CHECK(r.first % Cache::kAlign == 0, "pointer not aligned");
    CHECK(r.first >= end, "live blocks overlap");
    end = r.first + r.second;
  }
}

size_t draw_size(std::mt19937_64& g) {
  std::uniform_real_distribution<double> u(0.0, 1.0);
  if (u(g) < 0.7) return (size_t)std::exp(u(g) * std::log(4.0 * (1 << 20)));          // 1 B .. 4 MiB
  return (size_t)std::exp(std::log(64.0 * (1 << 20)) + u(g) * std::log(320.0));     // 64 MiB .. 20 GiB
}

void random_ops() {
  Cache C;
  std::mt19937_64 g(11081);
  std::map<uintptr_t, size_t> live;
  std::vector<uintptr_t> keys;
  for (int step = 0; step < 20000; ++step) {
    if (!live.empty() && (g() % 2 == 0 || C.mapped() > ((size_t)200 << 30))) {
      auto it = live.begin();
      std::advance(it, g() % live.size());
      CHECK(C.free((void*)it->first), "free of a live block failed");
      live.erase(it);
    } else {
      const size_t n = draw_size(g);
      void* p = C.alloc(n);
      CHECK(p != nullptr, "alloc of %zu failed", n);
      if (p) live[(uintptr_t)p] = n;
    }
    if (step % 97 == 0) validate(C, live);
  }
  validate(C, live);
  for (auto& r : live) C.free((void*)r.first);
  live.clear();
  validate(C, live);
  size_t blocks = 0;
  C.walk([&](size_t, size_t off, size_t, bool free) { ++blocks; CHECK(free && off == 0, "segment not whole after freeing all"); });
  CHECK(blocks == C.segments(), "%zu blocks in %zu segments after freeing all", blocks, C.segments());
  CHECK(C.trim(0) == 0 && C.mapper().in_use == 0 && C.mapper().live.empty(), "trim(0) left memory mapped");
  std::printf("random_ops ok: %d maps\n", C.mapper().maps);
}

void reuse_without_mapping() {
  Cache C;
  std::mt19937_64 g(7);
  std::vector<size_t> sizes;
  for (int i = 0; i < 60; ++i) sizes.push_back(draw_size(g));
  for (int rep = 0; rep < 3; ++rep) {
    std::vector<void*> ps;
    for (size_t s : sizes) ps.push_back(C.alloc(s));
    const int maps = C.mapper().maps;
    for (void* p : ps) C.free(p);
    if (rep == 0) continue;
    CHECK(C.mapper().maps == maps, "round %d mapped new segments", rep);
  }
  const int maps = C.mapper().maps;
  std::vector<void*> ps;
  for (size_t s : sizes) ps.push_back(C.alloc(s));
  CHECK(C.mapper().maps == maps, "repeated request sequence mapped new segments");
  for (void* p : ps) C.free(p);
  std::printf("reuse ok: %d maps for %zu requests x 4\n", C.mapper().maps, sizes.size());
}

void out_of_memory() {
  Cache C;
  C.mapper().capacity = (size_t)40 << 30;
  const size_t GiB = (size_t)1 << 30;
  void* a = C.alloc(10 * GiB);
  void* b = C.alloc(10 * GiB);
  void* c = C.alloc(10 * GiB);
  CHECK(a && b && c, "three 10 GiB blocks in 40 GiB");
  C.free(a);
  C.free(b);
  // 15 GiB does not fit in the free 10 GiB blocks nor in the 10 GiB unmapped:
  // the cache unmaps its idle segments and maps again
  void* d = C.alloc(15 * GiB);
  CHECK(d != nullptr, "15 GiB after unmapping idle segments");
  CHECK(C.mapper().quiesces == 1, "device quiesced once (%d)", C.mapper().quiesces);
  void* e = C.alloc(30 * GiB);
  CHECK(e == nullptr, "30 GiB cannot fit beside 25 GiB in use");
  std::map<uintptr_t, size_t> live{{(uintptr_t)c, 10 * GiB}, {(uintptr_t)d, 15 * GiB}};
  validate(C, live);
  CHECK(!C.free((void*)0x1234), "free of a foreign pointer");
  CHECK(C.free(c) && !C.free(c), "double free");
  C.free(d);
  CHECK(C.trim(0) == 0, "trim after out of memory");
  std::printf("out_of_memory ok\n");
}

void small_and_large_classes() {
  Cache C;
  void* big = C.alloc((size_t)1 << 30);
  C.free(big);
  const int maps = C.mapper().maps;
  void* small = C.alloc(1000);
  CHECK(C.mapper().maps == maps + 1, "a small request maps a small segment instead of cutting the large block");
  void* big2 = C.alloc((size_t)1 << 30);
  CHECK(big2 == big, "the large block is reused whole");
  C.free(small);
  C.free(big2);
  CHECK(C.trim((size_t)1 << 30) <= ((size_t)1 << 30), "trim keeps at most the requested bytes");
  std::printf("classes ok\n");
}

}  // namespace

int main() {
  random_ops();
  reuse_without_mapping();
  out_of_memory();
  small_and_large_classes();
  if (failures) {
    std::printf("%d failures\n", failures);
    return 1;
  }
  std::printf("ALL OK\n");
  return 0;
}
