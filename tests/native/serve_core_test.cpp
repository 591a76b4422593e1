// Host tests of the serving runtime's admission core (serve_core.hpp):
// arena allocation and coalescing, FIFO admission by footprint and slots.
// Built and run by tests/test_serve_core.py with g++ (no GPU).
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "serve_core.hpp"

using trig::serve::Admission;
using trig::serve::Arena;

static int failures = 0;
#define CHECK(c)                                                     \
    do {                                                             \
        if (!(c)) {                                                  \
            std::printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #c); \
            ++failures;                                              \
        }                                                            \
    } while (0)

static void test_arena_basics() {
    Arena a(4096, 256);
    size_t b0 = a.alloc(100), b1 = a.alloc(256), b2 = a.alloc(1000);
    CHECK(b0 == 0 && b1 == 256 && b2 == 512);
    CHECK(a.in_use() == 256 + 256 + 1024);
    CHECK(a.alloc(4096) == Arena::kFail);
    CHECK(a.release(b1));
    CHECK(!a.release(b1));  // double free rejected
    CHECK(a.alloc(256) == 256);  // first fit reuses the hole
    CHECK(a.release(b0) && a.release(256) && a.release(b2));
    CHECK(a.in_use() == 0 && a.largest_free() == 4096 && a.live_blocks() == 0);  // fully coalesced
    CHECK(a.alloc(0) == 0);  // zero bytes still takes one unit
}

static void test_arena_random_coalescing() {
    std::mt19937 rng(7);
    Arena a(1 << 20, 256);
    std::vector<size_t> live;
    for (int it = 0; it < 20000; ++it) {
        if (live.empty() || (rng() % 3)) {
            size_t n = 1 + rng() % 20000;
            size_t off = a.alloc(n);
            if (off != Arena::kFail) {
                CHECK(off % 256 == 0 && off + a.round(n) <= a.capacity());
                live.push_back(off);
            }
        } else {
            size_t k = rng() % live.size();
            CHECK(a.release(live[k]));
            live.erase(live.begin() + k);
        }
    }
    for (size_t off : live) CHECK(a.release(off));
    CHECK(a.in_use() == 0 && a.largest_free() == a.capacity());
}

static void test_admission_fifo_and_slots() {
    Admission adm(10240, 2);  // capacity is rounded down to the alignment
    CHECK(adm.admissible(10240) && !adm.admissible(10241));
    CHECK(!Admission(10000, 1).admissible(10000));
    adm.enqueue(1, 4000);
    adm.enqueue(2, 4000);
    adm.enqueue(3, 100);
    uint64_t t;
    size_t o1, o2, o3;
    CHECK(adm.admit_next(t, o1) && t == 1);
    CHECK(adm.admit_next(t, o2) && t == 2);
    CHECK(!adm.admit_next(t, o3));  // no free slot although memory fits
    adm.complete(o1);
    CHECK(adm.admit_next(t, o3) && t == 3);
    adm.complete(o2);
    adm.complete(o3);
    CHECK(adm.free_slots() == 2 && adm.arena().in_use() == 0);
}

static void test_admission_memory_blocks_fifo() {
    Admission adm(8192, 8);
    adm.enqueue(1, 6000);
    adm.enqueue(2, 6000);  // does not fit while 1 runs
    adm.enqueue(3, 512);   // would fit, but FIFO: waits behind 2
    uint64_t t;
    size_t o1, o2;
    CHECK(adm.admit_next(t, o1) && t == 1);
    CHECK(!adm.admit_next(t, o2));
    CHECK(adm.queued() == 2);
    adm.complete(o1);
    CHECK(adm.admit_next(t, o2) && t == 2);
    CHECK(adm.cancel(3) && !adm.cancel(3) && adm.queued() == 0);
}

static void test_footprint() {
    using trig::serve::slice_footprint;
    CHECK(slice_footprint(0, 0, 0) > 0);
    size_t f = slice_footprint(1000, 90000, 4096);
    CHECK(f >= 4 * 3001 + 8 * 90000 + 4 * 1000 + 1000 + 4 * 1000 + 4096);
    CHECK(f % 256 == 0);
}

int main() {
    test_arena_basics();
    test_arena_random_coalescing();
    test_admission_fifo_and_slots();
    test_admission_memory_blocks_fifo();
    test_footprint();
    if (failures) {
        std::printf("%d failures\n", failures);
        return 1;
    }
    std::printf("serve_core: all checks passed\n");
    return 0;
}
