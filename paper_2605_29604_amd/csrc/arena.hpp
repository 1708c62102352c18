// First-fit allocator of 256-byte aligned regions of a caller-owned device arena
// (host bookkeeping of offsets only; plain C++, no device calls).  Frees coalesce
// with their free neighbours.
#pragma once
#include <algorithm>
#include <cstddef>
#include <iterator>
#include <map>

namespace tcmis {

inline size_t round256(size_t x) { return (x + 255) & ~(size_t)255; }

class Arena {
public:
    void init(size_t bytes) {
        free_.clear();
        bytes &= ~(size_t)255;
        if (bytes) free_[0] = bytes;
        cap_ = bytes;
        used_ = 0;
    }
    bool alloc(size_t bytes, size_t* off) {
        bytes = round256(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes, next = it->first + bytes;
            free_.erase(it);
            if (rest) free_[next] = rest;
            used_ += bytes;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = round256(bytes);
        used_ -= bytes;
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
    size_t capacity() const { return cap_; }
    size_t used() const { return used_; }
    size_t largest_free() const {
        size_t m = 0;
        for (const auto& f : free_) m = std::max(m, f.second);
        return m;
    }

private:
    std::map<size_t, size_t> free_;
    size_t cap_ = 0, used_ = 0;
};

}  // namespace tcmis
