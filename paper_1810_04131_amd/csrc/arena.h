// Host bookkeeping of the serving arena (host code only; builds with a plain
// C++ compiler): first-fit ranges of a node arena and a device-memory budget.
#pragma once

#include <algorithm>
#include <cstdint>
#include <utility>
#include <vector>

namespace yq {

// Node ranges [0, capacity) handed out first fit.  Free ranges are kept sorted
// by offset and merged with their neighbours, so the first range that fits is
// the lowest-offset free run of at least the requested length.
class NodeArena {
 public:
  explicit NodeArena(int64_t capacity = 0) { reset(capacity); }
  void reset(int64_t capacity) {
    cap_ = capacity;
    free_.clear();
    if (capacity > 0) free_.push_back({0, capacity});
  }
  int64_t capacity() const { return cap_; }
  // Takes n > 0 nodes; false (and off unchanged) when no free run is long enough.
  bool take(int64_t n, int64_t& off) {
    if (n <= 0) return false;
    for (size_t k = 0; k < free_.size(); ++k) {
      auto& fr = free_[k];
      if (fr.second >= n) {
        off = fr.first;
        fr.first += n;
        fr.second -= n;
        if (fr.second == 0) free_.erase(free_.begin() + (std::ptrdiff_t)k);
        return true;
      }
    }
    return false;
  }
  // Returns a range that take() handed out.
  void give(int64_t off, int64_t n) {
    if (n <= 0) return;
    auto it = std::lower_bound(free_.begin(), free_.end(), std::make_pair(off, (int64_t)0));
    it = free_.insert(it, {off, n});
    // merge with the following and the preceding range
    const size_t k = (size_t)(it - free_.begin());
    if (k + 1 < free_.size() && free_[k].first + free_[k].second == free_[k + 1].first) {
      free_[k].second += free_[k + 1].second;
      free_.erase(free_.begin() + (std::ptrdiff_t)(k + 1));
    }
    if (k > 0 && free_[k - 1].first + free_[k - 1].second == free_[k].first) {
      free_[k - 1].second += free_[k].second;
      free_.erase(free_.begin() + (std::ptrdiff_t)k);
    }
  }
  int64_t free_total() const {
    int64_t t = 0;
    for (const auto& r : free_) t += r.second;
    return t;
  }
  const std::vector<std::pair<int64_t, int64_t>>& ranges() const { return free_; }

 private:
  int64_t cap_ = 0;
  std::vector<std::pair<int64_t, int64_t>> free_;   // (offset, length), sorted, merged
};

// Device-memory budget of admitted requests (bytes, by per-request estimates).
struct MemBudget {
  double limit = 0.0, used = 0.0;
  bool fits(double bytes) const { return used + bytes <= limit; }
  void take(double bytes) { used += bytes; }
  void give(double bytes) { used = std::max(0.0, used - bytes); }
};

}  // namespace yq
