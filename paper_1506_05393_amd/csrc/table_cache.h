// A small least-recently-used cache shared between threads (host code only,
// no HIP types): each sequence keeps the step tables of its last few
// (grid, readout count) keys in one.
//
// A lookup hands out a shared reference to the entry. An entry that is
// evicted (or dropped by clear()) while another call still holds it is
// released only when the last holder drops its reference, so a caller may use
// what it got for as long as it keeps the reference, whatever other threads
// look up meanwhile.
#pragma once

#include <cstddef>
#include <memory>
#include <mutex>
#include <utility>
#include <vector>

namespace mrf {

template <class Key, class T>
class LruCache {
 public:
  explicit LruCache(size_t capacity) : cap_(capacity > 0 ? capacity : 1) {}

  // The entry of `key`: found (and made the most recent), or built by
  // make(std::shared_ptr<T>*) -> int status (0 = success) under the cache's
  // lock, inserted, and the least recent entry evicted beyond the capacity.
  // On a failed build nothing is inserted and make's status is returned.
  template <class Make>
  int get(const Key& key, Make&& make, std::shared_ptr<const T>* out) {
    std::lock_guard<std::mutex> lk(mu_);
    for (size_t i = 0; i < items_.size(); ++i) {
      if (items_[i].first == key) {
        auto hit = items_[i];
        items_.erase(items_.begin() + (long)i);
        items_.push_back(hit);
        *out = hit.second;
        return 0;
      }
    }
    std::shared_ptr<T> made;
    const int rc = make(&made);
    if (rc != 0) return rc;
    if (items_.size() >= cap_) items_.erase(items_.begin());
    items_.emplace_back(key, made);
    *out = std::move(made);
    return 0;
  }

  // Drops the cache's own references (holders keep theirs).
  void clear() {
    std::lock_guard<std::mutex> lk(mu_);
    items_.clear();
  }

  size_t size() const {
    std::lock_guard<std::mutex> lk(mu_);
    return items_.size();
  }

 private:
  size_t cap_;
  mutable std::mutex mu_;
  std::vector<std::pair<Key, std::shared_ptr<T>>> items_;
};

}  // namespace mrf
