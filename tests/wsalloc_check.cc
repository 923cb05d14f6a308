// Host check of the workspace bookkeeping (mcd_wsalloc.h), built by
// tests/test_wsalloc.py with g++ under the address and undefined-behaviour
// sanitizers.  Random takes and releases against a brute-force model of the
// range: pieces stay aligned, inside the range and disjoint; the byte
// counts, the extent and the need figure match their definitions; releasing
// everything leaves one free range; a stack-ordered sequence fits a range of
// exactly its extent.
#include <stdio.h>
#include <stdlib.h>

#include <map>
#include <random>
#include <vector>

#include "mcd_wsalloc.h"

using mcd::WsAlloc;

static int fail(const char *what, long a, long b) {
    fprintf(stderr, "FAIL %s: %ld %ld\n", what, a, b);
    return 1;
}

int main() {
    std::mt19937_64 rng(12345);
    for (int trial = 0; trial < 200; trial++) {
        const size_t size = (size_t)(1 + rng() % 4096) * WsAlloc::kAlign + rng() % 255;
        WsAlloc w(size);
        if (w.size() != size / WsAlloc::kAlign * WsAlloc::kAlign) return fail("size", w.size(), size);
        std::map<size_t, size_t> live;   // offset -> rounded length
        size_t ext = 0;
        for (int op = 0; op < 400; op++) {
            if (live.empty() || rng() % 3 != 0) {
                const size_t req = 1 + rng() % (size / 6 + 1);
                const size_t off = w.alloc(req);
                const size_t len = WsAlloc::round(req);
                if (off == WsAlloc::kFail) {
                    // no free gap of len bytes may exist
                    size_t prev = 0;
                    for (auto &p : live) {
                        if (p.first - prev >= len) return fail("missed gap", (long)prev, (long)len);
                        prev = p.first + p.second;
                    }
                    if (w.size() - prev >= len) return fail("missed tail", (long)prev, (long)len);
                    const size_t top = live.empty() ? 0 : live.rbegin()->first + live.rbegin()->second;
                    if (w.need() < top + len) return fail("need", (long)w.need(), (long)(top + len));
                    continue;
                }
                if (off % WsAlloc::kAlign) return fail("align", (long)off, 0);
                if (off + len > w.size()) return fail("range", (long)(off + len), (long)w.size());
                auto nx = live.lower_bound(off);
                if (nx != live.end() && nx->first < off + len) return fail("overlap next", (long)off, (long)nx->first);
                if (nx != live.begin()) {
                    auto pv = std::prev(nx);
                    if (pv->first + pv->second > off) return fail("overlap prev", (long)off, (long)pv->first);
                }
                // first fit: no earlier gap of len bytes
                size_t prev = 0;
                for (auto &p : live) {
                    if (p.first >= off) break;
                    if (p.first - prev >= len) return fail("not first fit", (long)prev, (long)off);
                    prev = p.first + p.second;
                }
                live[off] = len;
                ext = std::max(ext, off + len);
            } else {
                auto it = live.begin();
                std::advance(it, rng() % live.size());
                if (!w.release(it->first)) return fail("release", (long)it->first, 0);
                if (w.release(it->first)) return fail("double release", (long)it->first, 0);
                live.erase(it);
            }
            size_t used = 0;
            for (auto &p : live) used += p.second;
            if (used != w.in_use()) return fail("in_use", (long)used, (long)w.in_use());
            if (w.pieces() != live.size()) return fail("pieces", (long)w.pieces(), (long)live.size());
            if (w.extent() != ext) return fail("extent", (long)w.extent(), (long)ext);
        }
        if (w.release(size + 4096)) return fail("foreign release", 0, 0);
        for (auto &p : live) w.release(p.first);
        if (w.in_use() != 0 || w.largest_free() != w.size()) return fail("coalesce", (long)w.largest_free(), (long)w.size());
    }
    // a stack-ordered sequence replayed on a range of exactly its extent
    for (int trial = 0; trial < 100; trial++) {
        WsAlloc big(size_t(1) << 40);
        std::vector<std::pair<size_t, size_t>> seq;   // (is_take, size or index)
        std::vector<size_t> stack;
        std::vector<size_t> sizes;
        for (int k = 0; k < 60; k++) {
            if (stack.empty() || rng() % 3) {
                const size_t b = 1 + rng() % 100000;
                sizes.push_back(b);
                stack.push_back(big.alloc(b));
            } else {
                big.release(stack.back());
                stack.pop_back();
                sizes.push_back(0);
            }
        }
        WsAlloc exact(big.extent());
        std::vector<size_t> st2;
        for (size_t b : sizes) {
            if (b) {
                const size_t o = exact.alloc(b);
                if (o == WsAlloc::kFail) return fail("replay", (long)b, (long)big.extent());
                st2.push_back(o);
            } else {
                exact.release(st2.back());
                st2.pop_back();
            }
        }
        // the copy grown without bound keeps the live pieces
        WsAlloc g = exact;
        g.grow_to(exact.size() * 2 + 4096);
        if (g.in_use() != exact.in_use() || g.size() != (exact.size() * 2 + 4096) / 256 * 256)
            return fail("grow", (long)g.in_use(), (long)exact.in_use());
        if (g.alloc(exact.size()) == WsAlloc::kFail) return fail("grown range", 0, 0);
    }
    // restart_extent: the extent of a second use of the same range
    {
        WsAlloc w(size_t(1) << 30);
        const size_t a = w.alloc(1 << 20), b = w.alloc(8 << 20);
        w.release(b);
        if (w.extent() != (size_t)(9 << 20)) return fail("extent before", (long)w.extent(), 0);
        w.restart_extent();
        if (w.extent() != (size_t)(1 << 20)) return fail("restart", (long)w.extent(), 0);
        w.alloc(4096);
        if (w.extent() != (size_t)(1 << 20) + 4096) return fail("after restart", (long)w.extent(), 0);
        (void)a;
    }
    printf("ok\n");
    return 0;
}
