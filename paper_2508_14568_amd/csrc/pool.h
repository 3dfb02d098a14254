// First-fit allocator of device arena space (offsets only: nothing is
// dereferenced), shared by the serving engines.
#pragma once

#include <cstddef>
#include <iterator>
#include <map>

namespace lvs {

// First-fit allocator over a byte range of the arena (offsets, 256-aligned).
class Pool {
public:
    // The range is used in whole 256-byte units, so that a request of at most
    // total() bytes always fits an empty pool.
    void init(size_t bytes) {
        free_.clear();
        bytes &= ~size_t(255);
        if (bytes) free_[0] = bytes;
        total_ = bytes;
    }
    bool alloc(size_t bytes, size_t* off) {
        bytes = unit(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes;
            const size_t at = it->first + bytes;
            free_.erase(it);
            if (rest) free_[at] = rest;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = unit(bytes);
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
    }
    size_t total() const { return total_; }

private:
    static size_t unit(size_t x) { return (x + 255) & ~size_t(255); }
    std::map<size_t, size_t> free_;
    size_t total_ = 0;
};

}  // namespace lvs
