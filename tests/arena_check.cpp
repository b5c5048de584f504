// Host test of the serving arena's bookkeeping (paper_2008_11520_amd/csrc/
// arena.h): random sequences of block allocations and releases, and of
// staging-ring slot placements and releases.  Live blocks (and live slots)
// must never overlap and must stay inside their region; releasing everything
// must give back one free block of the whole region; the ring must accept a
// slot of any size up to its own once it is empty.  Exits non-zero on a
// violation.
#include "arena.h"

#include <cstdio>
#include <random>
#include <vector>

using namespace dnnmg;

static int fails = 0;
#define CHECK(c, ...) do { if (!(c)) { if (fails++ < 10) { std::printf("FAIL: " __VA_ARGS__); std::printf("\n"); } } } while (0)

struct Span { size_t off, size; };

static bool disjoint(const std::vector<Span> &v)
{
    for (size_t i = 0; i < v.size(); ++i)
        for (size_t j = i + 1; j < v.size(); ++j)
            if (v[i].off < v[j].off + v[j].size && v[j].off < v[i].off + v[i].size) return false;
    return true;
}

int main()
{
    std::mt19937_64 g(7);
    // ---- block list
    for (int trial = 0; trial < 200; ++trial) {
        BlockList b;
        const size_t region = 256 * (1 + g() % 4000);
        b.init(region);
        std::vector<Span> live;
        for (int op = 0; op < 400; ++op) {
            if (live.empty() || g() % 3) {
                const size_t want = 1 + g() % (region / 4 + 1);
                size_t off = 0;
                const size_t largest = b.largest();
                const bool ok = b.take(want, &off);
                CHECK(ok == (arena_round(want) <= largest), "take %zu with largest free %zu: %d", want, largest, ok);
                if (ok) {
                    live.push_back({off, arena_round(want)});
                    CHECK(off % 256 == 0 && off + arena_round(want) <= b.bytes, "block [%zu, +%zu) outside", off, want);
                }
            } else {
                const size_t k = g() % live.size();
                b.give(live[k].off, live[k].size);
                live.erase(live.begin() + k);
            }
            size_t sum = 0;
            for (auto &s : live) sum += s.size;
            CHECK(sum == b.used, "used %zu, live blocks sum to %zu", b.used, sum);
            CHECK(disjoint(live), "live blocks overlap (trial %d op %d)", trial, op);
            // free blocks: disjoint from each other and from live blocks, together the rest
            size_t fsum = 0;
            std::vector<Span> all = live;
            for (auto &f : b.free_blocks) { fsum += f.second; all.push_back({f.first, f.second}); }
            CHECK(fsum + b.used == b.bytes && disjoint(all), "free list inconsistent (trial %d op %d)", trial, op);
        }
        for (auto &s : live) b.give(s.off, s.size);
        CHECK(b.free_blocks.size() == 1 && b.free_blocks.begin()->second == b.bytes && b.used == 0,
              "released arena is not one free block");
    }
    std::printf("block list: 200 random sequences of 400 operations consistent\n");
    // ---- staging ring
    for (int trial = 0; trial < 200; ++trial) {
        StageRing r;
        r.init(256 * (1 + g() % 64));
        std::vector<Span> live;   // in ring order (oldest first)
        for (int op = 0; op < 400; ++op) {
            if (!r.slots.empty() && g() % 3 == 0) {
                r.pop_oldest();
                live.erase(live.begin());
            } else {
                const size_t want = 1 + g() % r.bytes;
                size_t off = 0;
                if (r.place(want, &off)) {
                    CHECK(off % 256 == 0 && off + arena_round(want) <= r.bytes, "slot [%zu, +%zu) outside %zu", off,
                          want, r.bytes);
                    // place() may have lengthened the newest slot to the ring's end
                    if (!live.empty()) live.back().size = r.slots.back().size;
                    r.push(off, want);
                    live.push_back({off, arena_round(want)});
                    CHECK(disjoint(live), "live slots overlap (trial %d op %d)", trial, op);
                } else {
                    CHECK(!r.slots.empty(), "empty ring refused %zu of %zu bytes", want, r.bytes);
                }
            }
            CHECK(live.size() == r.slots.size(), "slot count");
            for (size_t k = 0; k < live.size(); ++k)
                CHECK(live[k].off == r.slots[k].off, "slot %zu offset", k);
        }
        while (!r.slots.empty()) r.pop_oldest();
        size_t off = 1;
        CHECK(r.place(r.bytes, &off) && off == 0, "an empty ring refuses a slot of its own size");
    }
    std::printf("staging ring: 200 random sequences of 400 operations consistent\n");
    if (fails) { std::printf("%d violations\n", fails); return 1; }
    std::printf("arena bookkeeping consistent\n");
    return 0;
}
