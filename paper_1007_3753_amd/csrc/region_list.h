// A free list of device memory regions that are never returned to the
// runtime (uncached exchange memory must outlive every kernel that read it).
// Each plan takes its own region; a destroyed plan gives its region back and
// a later plan may take it again.  Host-only code (no HIP), so its logic is
// checked on the CPU.
#pragma once
#include <cstddef>
#include <functional>
#include <mutex>
#include <vector>

namespace l1 {

class RegionList {
 public:
  // A free region of at least `bytes` (the smallest that fits), else a new
  // one from `alloc` (which returns null on failure).  *got receives the
  // region's size (0 on failure).
  void* get(size_t bytes, const std::function<void*(size_t)>& alloc, size_t* got) {
    std::lock_guard<std::mutex> lock(mu_);
    int best = -1;
    for (int i = 0; i < (int)free_.size(); ++i)
      if (free_[i].bytes >= bytes && (best < 0 || free_[i].bytes < free_[best].bytes)) best = i;
    if (best >= 0) {
      const Region r = free_[best];
      free_.erase(free_.begin() + best);
      *got = r.bytes;
      return r.p;
    }
    void* p = alloc(bytes);
    *got = p ? bytes : 0;
    return p;
  }
  // Give a region back for reuse.
  void put(void* p, size_t bytes) {
    if (!p) return;
    std::lock_guard<std::mutex> lock(mu_);
    free_.push_back(Region{p, bytes});
  }
  size_t free_count() {
    std::lock_guard<std::mutex> lock(mu_);
    return free_.size();
  }

 private:
  struct Region {
    void* p;
    size_t bytes;
  };
  std::mutex mu_;
  std::vector<Region> free_;
};

}  // namespace l1
