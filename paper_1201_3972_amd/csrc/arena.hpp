// arena.hpp -- first-fit allocator over the offsets of one device buffer (the
// serving engine's space for one-off frames).  Plain C++ with no HIP, so the
// host tests build it with g++ under the address and undefined-behaviour
// sanitizers.
#pragma once

#include <stddef.h>

#include <iterator>
#include <map>

namespace irf {
namespace host {

constexpr size_t kArenaAlign = 4096;

inline size_t round_up(size_t n) { return (n + kArenaAlign - 1) / kArenaAlign * kArenaAlign; }

// Blocks are rounded up to 4 KiB and taken from the lowest free offset that
// fits; a released block merges with free neighbours on both sides, so freeing
// everything restores one block of the whole capacity.
class Arena {
  public:
    void reset(size_t capacity) {
        free_.clear();
        used_ = 0;
        if (capacity) free_[0] = capacity;
    }
    size_t used() const { return used_; }
    size_t free_blocks() const { return free_.size(); }
    bool alloc(size_t bytes, size_t *off) {
        const size_t need = round_up(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= need) {
                *off = it->first;
                used_ += need;
                const size_t rest = it->second - need, start = it->first + need;
                free_.erase(it);
                if (rest) free_[start] = rest;
                return true;
            }
        }
        return false;
    }
    // `off` and `bytes` must be those of a block alloc() returned and not yet released.
    void release(size_t off, size_t bytes) {
        size_t start = off, size = round_up(bytes);
        used_ -= size;
        auto next = free_.lower_bound(start);
        if (next != free_.end() && start + size == next->first) {
            size += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == start) {
                prev->second += size;
                return;
            }
        }
        free_[start] = size;
    }

  private:
    std::map<size_t, size_t> free_;  // offset -> size
    size_t used_ = 0;
};

}  // namespace host
}  // namespace irf
