// Host bookkeeping of the serving arena (no HIP calls): the first-fit block
// list of the device region and the pinned staging ring.  The library pairs
// each staging slot with a HIP event; a host test drives both structures
// through random sequences and checks that live blocks and slots never
// overlap and stay inside their regions.
#pragma once

#include <cstddef>
#include <deque>
#include <iterator>
#include <map>

namespace dnnmg {

constexpr size_t arena_round(size_t x) { return (x + 255) & ~size_t(255); }

// Free blocks of a region [0, bytes) in 256-byte units, adjacent blocks
// merged; allocation takes the first block that fits.
struct BlockList {
    std::map<size_t, size_t> free_blocks;   // offset -> size
    size_t bytes = 0, used = 0;

    void init(size_t region)
    {
        bytes = region & ~size_t(255);
        used = 0;
        free_blocks.clear();
        if (bytes) free_blocks[0] = bytes;
    }
    bool take(size_t want, size_t *off)
    {
        want = arena_round(want);
        for (auto it = free_blocks.begin(); it != free_blocks.end(); ++it) {
            if (it->second < want) continue;
            *off = it->first;
            const size_t rest = it->second - want, roff = it->first + want;
            free_blocks.erase(it);
            if (rest) free_blocks[roff] = rest;
            used += want;
            return true;
        }
        return false;
    }
    void give(size_t off, size_t size)
    {
        size = arena_round(size);
        used -= size;
        auto it = free_blocks.emplace(off, size).first;
        auto next = std::next(it);
        if (next != free_blocks.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_blocks.erase(next);
        }
        if (it != free_blocks.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_blocks.erase(it);
            }
        }
    }
    size_t largest() const
    {
        size_t m = 0;
        for (const auto &b : free_blocks) m = m > b.second ? m : b.second;
        return m;
    }
};

// A ring of contiguous slots over [0, bytes): slots are placed at the head and
// released oldest first; a slot never wraps (an unused end of the ring is
// added to the newest slot).  head == tail means empty when no slot is live
// and full otherwise.
struct StageRing {
    struct Slot { size_t off, size; };
    std::deque<Slot> slots;                 // live slots, oldest first
    size_t bytes = 0, head = 0, tail = 0;

    void init(size_t region)
    {
        bytes = arena_round(region);
        head = tail = 0;
        slots.clear();
    }
    // Where a slot of `want` bytes goes now; false if the oldest slot must be
    // released first (or want exceeds the ring).
    bool place(size_t want, size_t *off)
    {
        want = arena_round(want);
        if (want > bytes || want == 0) return false;
        if (slots.empty()) { head = tail = 0; *off = 0; return true; }
        if (head > tail) {                   // free: [head, end), then [0, tail)
            if (bytes - head >= want) { *off = head; return true; }
            if (tail >= want) {
                slots.back().size += bytes - head;
                head = 0;
                *off = 0;
                return true;
            }
            return false;
        }
        if (head < tail && tail - head >= want) { *off = head; return true; }
        return false;                        // full, or too little room before the tail
    }
    // Make the slot returned by place() live.
    void push(size_t off, size_t want)
    {
        want = arena_round(want);
        slots.push_back({off, want});
        head = off + want == bytes ? 0 : off + want;
    }
    void pop_oldest()
    {
        const Slot s = slots.front();
        slots.pop_front();
        tail = s.off + s.size == bytes ? 0 : s.off + s.size;
        if (slots.empty()) head = tail = 0;
    }
};

}  // namespace dnnmg
