// First-fit allocator over the byte range [0, size): the serving admission
// budget (host only; offsets into an arena or a caller buffer).
#pragma once

#include <stdint.h>

#include <iterator>
#include <map>

namespace zinc {

// Free ranges are kept by offset and merged with their neighbours on release;
// sizes are rounded up to kAlign bytes.
class Arena {
public:
    static constexpr uint64_t kAlign = 256;

    explicit Arena(uint64_t size = 0) : size_(size) {
        if (size) free_[0] = size;
    }
    bool alloc(uint64_t bytes, uint64_t* off) {
        bytes = (bytes + kAlign - 1) & ~(kAlign - 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const uint64_t rest = it->second - bytes, start = it->first + bytes;
            free_.erase(it);
            if (rest) free_[start] = rest;
            used_ += bytes;
            return true;
        }
        return false;
    }
    void release(uint64_t off, uint64_t bytes) {
        bytes = (bytes + kAlign - 1) & ~(kAlign - 1);
        used_ -= bytes;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + bytes == next->first) {
            bytes += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += bytes;
                return;
            }
        }
        free_[off] = bytes;
    }
    uint64_t size() const { return size_; }
    uint64_t used() const { return used_; }

private:
    uint64_t size_ = 0, used_ = 0;
    std::map<uint64_t, uint64_t> free_;
};

}  // namespace zinc
