// Host bookkeeping of a caller-owned workspace: first-fit allocation of
// 256-byte aligned pieces of the offset range [0, size), with neighbouring
// free pieces merged on release.  Pure host C++ (no HIP), so the same code is
// compiled into the library and into a CPU test under the address and
// undefined-behaviour sanitizers.
//
// The workspace knows offsets only; the library adds the caller's device base
// address.  need() is the figure reported after a failed allocation: the end
// of the highest live piece plus the request, a size at which that request
// (with the same pieces live) would have been served.  A call that fails
// releases what it took, so a caller can grow its buffer to need() and call
// again; later requests of the same call may then ask for more.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <map>

namespace mcd {

class WsAlloc {
  public:
    static constexpr size_t kAlign = 256;
    static constexpr size_t kFail = ~size_t(0);

    explicit WsAlloc(size_t size) : size_(size / kAlign * kAlign) {
        if (size_ > 0) free_[0] = size_;
    }

    size_t size() const { return size_; }
    size_t in_use() const { return in_use_; }
    size_t high_water() const { return high_; }
    size_t need() const { return need_; }
    // highest end offset any piece has reached (the bytes a workspace must
    // have to replay the same sequence of takes and releases)
    size_t extent() const { return ext_; }
    size_t pieces() const { return used_.size(); }

    static size_t round(size_t bytes) {
        const size_t b = std::max<size_t>(bytes, 1);
        return (b + kAlign - 1) / kAlign * kAlign;
    }

    // Offset of a new piece of at least `bytes`, or kFail (need() updated).
    size_t alloc(size_t bytes) {
        const size_t len = round(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < len) continue;
            const size_t off = it->first, rest = it->second - len;
            free_.erase(it);
            if (rest > 0) free_[off + len] = rest;
            used_[off] = len;
            in_use_ += len;
            ext_ = std::max(ext_, off + len);
            high_ = std::max(high_, in_use_);
            return off;
        }
        // enough for this request: after the highest live piece
        const size_t top = used_.empty() ? 0 : used_.rbegin()->first + used_.rbegin()->second;
        need_ = std::max(need_, top + len);
        return kFail;
    }

    // Releases the piece at `off`; false if `off` is not a live piece.
    bool release(size_t off) {
        auto u = used_.find(off);
        if (u == used_.end()) return false;
        size_t start = off, len = u->second;
        used_.erase(u);
        in_use_ -= len;
        auto next = free_.lower_bound(start);
        if (next != free_.end() && next->first == start + len) {
            len += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == start) {
                start = prev->first;
                len += prev->second;
                free_.erase(prev);
            }
        }
        free_[start] = len;
        return true;
    }

    // Largest piece that could be taken now.
    size_t largest_free() const {
        size_t m = 0;
        for (auto &f : free_) m = std::max(m, f.second);
        return m;
    }

    void clear_need() { need_ = 0; }

    // Restarts the extent at the end of the highest live piece, so that
    // extent() measures one call from here on (a workspace reused by many
    // calls keeps the largest end any of them reached otherwise).
    void restart_extent() {
        ext_ = used_.empty() ? 0 : used_.rbegin()->first + used_.rbegin()->second;
    }
    void set_need(size_t b) { need_ = std::max(need_, b); }

    // Extends the range to `nsize` bytes (a copy used to replay takes
    // beyond the caller's size, for size answers).
    void grow_to(size_t nsize) {
        nsize = nsize / kAlign * kAlign;
        if (nsize <= size_) return;
        size_t start = size_, len = nsize - size_;
        if (!free_.empty()) {
            auto last = std::prev(free_.end());
            if (last->first + last->second == size_) {
                start = last->first;
                len += last->second;
                free_.erase(last);
            }
        }
        free_[start] = len;
        size_ = nsize;
    }

  private:
    size_t size_;
    size_t in_use_ = 0, high_ = 0, need_ = 0, ext_ = 0;
    std::map<size_t, size_t> free_;   // offset -> length, disjoint, merged
    std::map<size_t, size_t> used_;   // offset -> length of live pieces
};

}  // namespace mcd
