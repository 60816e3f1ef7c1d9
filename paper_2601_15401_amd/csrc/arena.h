// First-fit allocator over the offsets [0, size) of one device allocation,
// with coalescing of freed blocks.  Host-only bookkeeping: it never touches
// the memory it hands out, so it is also built and checked on its own (with
// the address and undefined-behaviour sanitizers) by a host program.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <iterator>
#include <map>

namespace mick {

class Arena {
 public:
  explicit Arena(size_t size = 0) : size_(size) {
    if (size) free_[0] = size;
  }
  // Offset of a block of `bytes` (callers pass multiples of 256), or
  // SIZE_MAX when no free block is large enough.
  size_t take(size_t bytes) {
    if (bytes == 0) return SIZE_MAX;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      const size_t off = it->first, rest = it->second - bytes;
      free_.erase(it);
      if (rest) free_[off + bytes] = rest;
      used_ += bytes;
      return off;
    }
    return SIZE_MAX;
  }
  // Returns a block obtained from take(); neighbouring free blocks merge.
  void give(size_t off, size_t bytes) {
    used_ -= bytes;
    auto nx = free_.lower_bound(off);
    if (nx != free_.end() && off + bytes == nx->first) {
      bytes += nx->second;
      nx = free_.erase(nx);
    }
    if (nx != free_.begin()) {
      auto pv = std::prev(nx);
      if (pv->first + pv->second == off) {
        pv->second += bytes;
        return;
      }
    }
    free_[off] = bytes;
  }
  size_t used() const { return used_; }
  size_t size() const { return size_; }
  // Free blocks, and the largest one (fragmentation diagnostics).
  size_t free_blocks() const { return free_.size(); }
  size_t largest_free() const {
    size_t m = 0;
    for (auto& f : free_) m = f.second > m ? f.second : m;
    return m;
  }

 private:
  size_t size_, used_ = 0;
  std::map<size_t, size_t> free_;  // offset -> length
};

}  // namespace mick
