// Best-fit cache of memory blocks carved from mapped segments.
//
// Segments come from a Mapper (map(bytes) -> pointer or nullptr, unmap(p),
// quiesce() before segments are unmapped to retry a failed map).  A request
// is rounded up to kAlign and served best-fit from the free blocks of its
// class: small requests (below kSmall) share segments of kSmallSegment bytes,
// large ones get segments of their own size rounded to kLargeRound, so small
// blocks never cut up the large free blocks that big buffers need.  A block
// is split when the rest is at least kMinSplit; a freed block merges with its
// free neighbours in the same segment, so a segment whose blocks are all free
// is one free block again and can be unmapped by trim().  The cache never
// touches the memory itself.  Not thread-safe: the caller holds a lock.
#pragma once
#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <functional>
#include <map>
#include <unordered_map>
#include <vector>

namespace lrx {

template <class Mapper>
class BlockCache {
 public:
  static constexpr size_t kAlign = 512;
  static constexpr size_t kSmall = (size_t)64 << 20;
  static constexpr size_t kSmallSegment = (size_t)256 << 20;
  static constexpr size_t kLargeRound = (size_t)2 << 20;
  static constexpr size_t kMinSplit = 4096;

  explicit BlockCache(Mapper m = Mapper()) : map_(m) {}
  // Unmaps every segment, blocks in use included.
  ~BlockCache() {
    for (Block* s : segs_) {
      for (Block* b = s->next; b;) {
        Block* n = b->next;
        delete b;
        b = n;
      }
      map_.unmap(s->base);
      delete s;
    }
  }
  BlockCache(const BlockCache&) = delete;
  BlockCache& operator=(const BlockCache&) = delete;

  Mapper& mapper() { return map_; }
  size_t mapped() const { return mapped_; }
  size_t used() const { return used_; }
  size_t segments() const { return segs_.size(); }

  void* alloc(size_t bytes) {
    const size_t size = (std::max<size_t>(bytes, 1) + kAlign - 1) / kAlign * kAlign;
    const bool small = size < kSmall;
    Block* b = nullptr;
    auto it = idle_[small].lower_bound(size);
    if (it != idle_[small].end()) {
      b = it->second;
      idle_[small].erase(it);
    } else {
      const size_t seg = small ? kSmallSegment : (size + kLargeRound - 1) / kLargeRound * kLargeRound;
      void* p = map_.map(seg);
      if (!p) {
        // out of memory: unmap every idle segment and try once more
        map_.quiesce();
        trim(0);
        p = map_.map(seg);
        if (!p) return nullptr;
      }
      b = new Block{(char*)p, seg, false, small, nullptr, nullptr};
      segs_.push_back(b);
      mapped_ += seg;
    }
    if (b->size - size >= kMinSplit) {
      Block* rest = new Block{b->base + size, b->size - size, true, b->small, b, b->next};
      if (b->next) b->next->prev = rest;
      b->next = rest;
      b->size = size;
      idle_[rest->small].emplace(rest->size, rest);
    }
    b->free = false;
    live_[b->base] = b;
    used_ += b->size;
    return b->base;
  }

  // Returns false for a pointer the cache did not hand out (or freed twice).
  bool free(void* p) {
    auto it = live_.find(p);
    if (it == live_.end()) return false;
    Block* b = it->second;
    live_.erase(it);
    used_ -= b->size;
    b->free = true;
    if (b->next && b->next->free) {
      Block* n = b->next;
      drop_idle(n);
      b->size += n->size;
      b->next = n->next;
      if (n->next) n->next->prev = b;
      delete n;
    }
    if (b->prev && b->prev->free) {
      Block* q = b->prev;
      drop_idle(q);
      q->size += b->size;
      q->next = b->next;
      if (b->next) b->next->prev = q;
      delete b;
      b = q;
    }
    idle_[b->small].emplace(b->size, b);
    return true;
  }

  // Unmap segments that are entirely free, largest first, until at most
  // `keep` bytes stay mapped; returns the bytes still mapped.
  size_t trim(size_t keep) {
    std::vector<size_t> order;
    for (size_t k = 0; k < segs_.size(); ++k)
      if (segs_[k]->free && !segs_[k]->next) order.push_back(k);
    std::stable_sort(order.begin(), order.end(),
                     [&](size_t x, size_t y) { return segs_[x]->size > segs_[y]->size; });
    std::vector<bool> gone(segs_.size(), false);
    for (size_t k : order) {
      if (mapped_ <= keep) break;
      Block* b = segs_[k];
      drop_idle(b);
      map_.unmap(b->base);
      mapped_ -= b->size;
      delete b;
      gone[k] = true;
    }
    std::vector<Block*> rest;
    for (size_t k = 0; k < segs_.size(); ++k)
      if (!gone[k]) rest.push_back(segs_[k]);
    segs_.swap(rest);
    return mapped_;
  }

  // Every block of every segment in address order as (segment, offset, size,
  // free): for checks of the cache's invariants.
  template <class F>
  void walk(F&& f) const {
    for (size_t k = 0; k < segs_.size(); ++k)
      for (const Block* b = segs_[k]; b; b = b->next) f(k, (size_t)(b->base - segs_[k]->base), b->size, b->free);
  }

 private:
  struct Block {
    char* base;
    size_t size;
    bool free;
    bool small;      // in a shared segment of small blocks
    Block* prev;     // neighbours in the same segment (address order)
    Block* next;
  };

  void drop_idle(Block* b) {
    auto r = idle_[b->small].equal_range(b->size);
    for (auto it = r.first; it != r.second; ++it)
      if (it->second == b) {
        idle_[b->small].erase(it);
        return;
      }
  }

  Mapper map_;
  std::multimap<size_t, Block*> idle_[2];         // free blocks by size: [0] large, [1] small segments
  std::unordered_map<void*, Block*> live_;        // blocks in use, by address
  std::vector<Block*> segs_;                      // first block of every segment
  size_t mapped_ = 0, used_ = 0;
};

}  // namespace lrx
