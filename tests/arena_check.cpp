// Randomised check of the serving loop's first-fit arena (csrc/arena.h), run
// on the host by tests/test_arena.py. Against a byte-granule model of the
// arena it checks, after every operation: live blocks are disjoint and inside
// the arena, the free list is sorted, disjoint, coalesced and covers exactly
// the bytes no live block holds, and alloc returns the lowest offset whose
// free run fits (first fit) or fails only when no free run fits.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "arena.h"

using gw::Arena;

static int fails = 0;
#define CHECK(c)                                                         \
    do {                                                                 \
        if (!(c)) {                                                      \
            std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
            if (++fails > 20) std::exit(1);                              \
        }                                                                \
    } while (0)

struct Live {
    size_t off, bytes;
};

// granule map: true where a live block sits
static void check_state(const Arena &a, const std::vector<Live> &live) {
    const size_t G = Arena::kGranule, ng = a.size / G;
    std::vector<char> used(ng, 0);
    for (const Live &l : live) {
        const size_t b = Arena::granules(l.bytes ? l.bytes : 1);
        CHECK(l.off % G == 0 && l.off + b <= a.size);
        for (size_t g = l.off / G; g < (l.off + b) / G && g < ng; ++g) {
            CHECK(!used[g]);   // disjoint
            used[g] = 1;
        }
    }
    size_t prev_end = 0;
    bool first = true;
    size_t covered = 0;
    for (const auto &f : a.free_) {
        CHECK(f.second > 0 && f.first % G == 0 && f.second % G == 0 && f.first + f.second <= a.size);
        if (!first) CHECK(f.first > prev_end);   // sorted, disjoint and not touching (coalesced)
        for (size_t g = f.first / G; g < (f.first + f.second) / G && g < ng; ++g) CHECK(!used[g]);
        covered += f.second;
        prev_end = f.first + f.second;
        first = false;
    }
    size_t n_used = 0;
    for (char u : used) n_used += u;
    CHECK(covered + n_used * G == a.size);   // every granule is free or live
    CHECK(a.free_bytes() == covered);
}

// the first-fit answer from the model: lowest offset of a free run of >= need bytes
static bool model_first_fit(const Arena &a, const std::vector<Live> &live, size_t need, size_t *off) {
    const size_t G = Arena::kGranule, ng = a.size / G, k = Arena::granules(need ? need : 1) / G;
    std::vector<char> used(ng, 0);
    for (const Live &l : live)
        for (size_t g = l.off / G; g < (l.off + Arena::granules(l.bytes ? l.bytes : 1)) / G; ++g) used[g] = 1;
    size_t run = 0;
    for (size_t g = 0; g < ng; ++g) {
        run = used[g] ? 0 : run + 1;
        if (run == k) {
            // the run may start inside a longer free block; first fit takes the
            // block's start, which is the run's start when the run begins there
            size_t s = g + 1 - k;
            while (s > 0 && !used[s - 1]) --s;
            *off = s * G;
            return true;
        }
    }
    return false;
}

int main() {
    std::mt19937_64 rng(12345);
    long ops = 0;
    for (int trial = 0; trial < 200; ++trial) {
        Arena a;
        const size_t size = (size_t)(rng() % 64 + 1) * Arena::kGranule + (trial % 3 == 0 ? 100 : 0);
        a.init(nullptr, size);
        CHECK(a.size % Arena::kGranule == 0 && a.size <= size && a.size + Arena::kGranule > size);
        std::vector<Live> live;
        check_state(a, live);
        for (int step = 0; step < 400; ++step, ++ops) {
            if (live.empty() || rng() % 100 < 55) {
                const size_t want = rng() % 5 == 0 ? 0 : rng() % (a.size / 3 + 1);
                size_t expect = 0, got = 777;
                const bool fits = model_first_fit(a, live, want, &expect);
                const bool ok = a.alloc(want, &got);
                CHECK(ok == fits);
                if (ok) {
                    CHECK(got == expect);
                    live.push_back({got, want});
                } else {
                    CHECK(got == 777);
                }
            } else {
                const size_t k = rng() % live.size();
                a.release(live[k].off, live[k].bytes);
                live.erase(live.begin() + k);
            }
            check_state(a, live);
        }
        while (!live.empty()) {
            a.release(live.back().off, live.back().bytes);
            live.pop_back();
        }
        check_state(a, live);
        CHECK(a.free_.size() == (a.size ? 1u : 0u) && a.free_bytes() == a.size);   // one block again
    }
    std::printf("arena: %ld operations, %d failed checks\n", ops, fails);
    return fails ? 1 : 0;
}
