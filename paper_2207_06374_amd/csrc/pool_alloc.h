// First-fit allocator of 256-byte aligned ranges in [0, capacity) of a
// caller-owned device pool (host bookkeeping only: no device memory is
// touched here).  Free ranges are kept sorted by offset and merged with
// their neighbours on release, so a fully drained pool is one free range
// again.  Plain C++ (no HIP), so the host tests can compile it alone.
#pragma once

#include <cstdint>
#include <iterator>
#include <map>

namespace trstmi {

class PoolAllocator {
 public:
  static constexpr uint64_t kAlign = 256;

  explicit PoolAllocator(uint64_t capacity = 0) { reset(capacity); }

  void reset(uint64_t capacity) {
    capacity_ = capacity / kAlign * kAlign;
    free_.clear();
    if (capacity_ > 0) free_[0] = capacity_;
    used_ = peak_ = 0;
  }

  static uint64_t round(uint64_t size) { return (size + kAlign - 1) / kAlign * kAlign; }

  // Offset of a free range of round(size) bytes (the lowest one that fits),
  // or false if none does.
  bool alloc(uint64_t size, uint64_t* offset) {
    const uint64_t need = round(size);
    if (need == 0) return false;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < need) continue;
      const uint64_t off = it->first, len = it->second;
      free_.erase(it);
      if (len > need) free_[off + need] = len - need;
      used_ += need;
      if (used_ > peak_) peak_ = used_;
      *offset = off;
      return true;
    }
    return false;
  }

  // Returns a range given out by alloc (same size as asked).
  void release(uint64_t offset, uint64_t size) {
    uint64_t off = offset, len = round(size);
    used_ -= len;
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + len == next->first) {  // merge with the range above
      len += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {  // merge with the range below
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += len;
        return;
      }
    }
    free_[off] = len;
  }

  uint64_t capacity() const { return capacity_; }
  uint64_t used() const { return used_; }
  uint64_t peak() const { return peak_; }
  const std::map<uint64_t, uint64_t>& free_ranges() const { return free_; }

 private:
  uint64_t capacity_ = 0, used_ = 0, peak_ = 0;
  std::map<uint64_t, uint64_t> free_;  // offset -> length
};

}  // namespace trstmi
