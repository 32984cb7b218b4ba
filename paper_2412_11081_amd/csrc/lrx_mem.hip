// Device memory cache of the library, one per device, shared by every
// context of the process.
//
// Contexts that come and go (a serving stream) would otherwise hand device
// memory back to the driver and map it again for the next request; memory
// that comes back from the driver must be cleared first, and while it is
// cleared the runtime holds up every thread's allocations and launches.  The
// cache keeps what it has mapped until lrx_pool_trim: segments come from
// hipMalloc, requests are served best-fit from free blocks (split when the
// rest is worth keeping), and a freed block merges with its free neighbours
// in the same segment.  Callers free a block only once the work that used it
// has finished (the context synchronises its streams first).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <functional>
#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "lrx_internal.h"

namespace lrx {
namespace {

constexpr size_t kAlign = 512;                    // every block starts on 512 B
constexpr size_t kSmall = (size_t)64 << 20;       // requests below this share segments
constexpr size_t kSmallSegment = (size_t)256 << 20;
constexpr size_t kLargeRound = (size_t)2 << 20;   // large segments: whole 2 MiB pages
constexpr size_t kMinSplit = 4096;                // a rest below this stays with the block

struct Block {
  char* base;
  size_t size;
  bool free;
  bool small;      // in a shared segment of small blocks
  Block* prev;     // neighbours in the same segment (address order)
  Block* next;
};

struct Cache {
  std::mutex mu;
  std::multimap<size_t, Block*> idle[2];         // free blocks by size: [0] large, [1] small segments
  std::unordered_map<void*, Block*> live;        // blocks in use by address
  std::vector<Block*> segments;                  // first block of every segment
  size_t mapped = 0, used = 0;

  void add_idle(Block* b) { idle[b->small].emplace(b->size, b); }
  void drop_idle(Block* b) {
    auto r = idle[b->small].equal_range(b->size);
    for (auto it = r.first; it != r.second; ++it)
      if (it->second == b) {
        idle[b->small].erase(it);
        return;
      }
  }

  // Free whole segments (one free block spanning the segment), largest first,
  // until at most `keep` bytes stay mapped.  Caller holds mu; the device must
  // be idle.
  void release(size_t keep) {
    std::multimap<size_t, size_t, std::greater<size_t>> order;
    for (size_t k = 0; k < segments.size(); ++k) {
      Block* b = segments[k];
      if (b->free && !b->next) order.emplace(b->size, k);
    }
    std::vector<bool> gone(segments.size(), false);
    for (auto& e : order) {
      if (mapped <= keep) break;
      Block* b = segments[e.second];
      drop_idle(b);
      (void)hipFree(b->base);
      mapped -= b->size;
      delete b;
      gone[e.second] = true;
    }
    std::vector<Block*> rest;
    for (size_t k = 0; k < segments.size(); ++k)
      if (!gone[k]) rest.push_back(segments[k]);
    segments.swap(rest);
  }
};

std::mutex g_caches_mu;
std::map<int, Cache*> g_caches;   // never destroyed: contexts may outlive static destruction order

Cache& cache_of(int device) {
  std::lock_guard<std::mutex> lk(g_caches_mu);
  Cache*& c = g_caches[device];
  if (!c) c = new Cache();
  return *c;
}

}  // namespace

void* dev_alloc(int device, size_t bytes) {
  const size_t size = (std::max<size_t>(bytes, 1) + kAlign - 1) / kAlign * kAlign;
  Cache& C = cache_of(device);
  std::lock_guard<std::mutex> lk(C.mu);
  // small requests are served from small segments only, so that they do not
  // cut up the large blocks that whole-structure buffers need
  const bool small = size < kSmall;
  Block* b = nullptr;
  auto it = C.idle[small].lower_bound(size);
  if (it != C.idle[small].end()) {
    b = it->second;
    C.idle[small].erase(it);
  } else {
    const size_t seg = small ? kSmallSegment : (size + kLargeRound - 1) / kLargeRound * kLargeRound;
    void* p = nullptr;
    if (hipMalloc(&p, seg) != hipSuccess) {
      // out of device memory: hand back every idle segment and try once more
      (void)hipGetLastError();
      (void)hipDeviceSynchronize();
      C.release(0);
      if (hipMalloc(&p, seg) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
      }
    }
    b = new Block{(char*)p, seg, false, small, nullptr, nullptr};
    C.segments.push_back(b);
    C.mapped += seg;
  }
  if (b->size - size >= kMinSplit) {
    Block* rest = new Block{b->base + size, b->size - size, true, b->small, b, b->next};
    if (b->next) b->next->prev = rest;
    b->next = rest;
    b->size = size;
    C.add_idle(rest);
  }
  b->free = false;
  C.live[b->base] = b;
  C.used += b->size;
  return b->base;
}

void dev_free(int device, void* p) {
  if (!p) return;
  Cache& C = cache_of(device);
  std::lock_guard<std::mutex> lk(C.mu);
  auto it = C.live.find(p);
  if (it == C.live.end()) return;
  Block* b = it->second;
  C.live.erase(it);
  C.used -= b->size;
  b->free = true;
  if (b->next && b->next->free) {
    Block* n = b->next;
    C.drop_idle(n);
    b->size += n->size;
    b->next = n->next;
    if (n->next) n->next->prev = b;
    delete n;
  }
  if (b->prev && b->prev->free) {
    Block* q = b->prev;
    C.drop_idle(q);
    q->size += b->size;
    q->next = b->next;
    if (b->next) b->next->prev = q;
    delete b;
    b = q;
  }
  C.add_idle(b);
}

size_t dev_trim(int device, size_t keep) {
  Cache& C = cache_of(device);
  std::lock_guard<std::mutex> lk(C.mu);
  C.release(keep);
  return C.mapped;
}

void dev_cache_bytes(int device, size_t* mapped, size_t* used) {
  Cache& C = cache_of(device);
  std::lock_guard<std::mutex> lk(C.mu);
  if (mapped) *mapped = C.mapped;
  if (used) *used = C.used;
}

}  // namespace lrx
