// host_checks.cpp -- host-side checks built with g++ under the address and
// undefined-behaviour sanitizers (tests/test_native_cpu.py):
//   * every sorting network of netgen.hpp sorts, and every merge network
//     merges, all 0-1 inputs (the 0-1 principle: then they sort any input);
//   * the serving arena (arena.hpp) against a page-bitmap model under random
//     allocations and releases, with coalescing back to one free block;
//   * the argument checks of host_common.hpp at their boundaries.
// Prints "ok" and returns 0 when everything holds.
#include <stdint.h>
#include <stdio.h>

#include <random>
#include <vector>

#include "../../paper_1201_3972_amd/csrc/arena.hpp"
#include "../../paper_1201_3972_amd/csrc/host_common.hpp"
#include "../../paper_1201_3972_amd/csrc/netgen.hpp"

static int failures = 0;
#define CHECK(c)                                                       \
    do {                                                               \
        if (!(c)) {                                                    \
            fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
            ++failures;                                                \
        }                                                              \
    } while (0)

template <int N>
static void check_sort_network() {
    const auto &net = irf::net::network<N>;
    for (uint32_t bits = 0; bits < (1u << N); ++bits) {
        int v[N];
        for (int i = 0; i < N; ++i) v[i] = (bits >> i) & 1;
        for (int c = 0; c < irf::net::Network<N>::size; ++c) {
            const int i = net.lo[c], j = net.hi[c];
            CHECK(0 <= i && i < j && j < N);
            if (v[i] > v[j]) {
                const int t = v[i];
                v[i] = v[j];
                v[j] = t;
            }
        }
        for (int i = 1; i < N; ++i)
            if (v[i - 1] > v[i]) {
                fprintf(stderr, "network %d leaves input %u unsorted\n", N, bits);
                ++failures;
                return;
            }
    }
}

template <int P>
static void check_merge_network() {
    const auto &net = irf::net::merge_network<P>;
    // two sorted 0-1 halves: a zeros then ones in [0,P), b zeros then ones in [P,2P)
    for (int a = 0; a <= P; ++a)
        for (int b = 0; b <= P; ++b) {
            std::vector<int> v(2 * P);
            for (int i = 0; i < P; ++i) {
                v[i] = i >= a;
                v[P + i] = i >= b;
            }
            for (int c = 0; c < irf::net::MergeNetwork<P>::size; ++c) {
                const int i = net.lo[c], j = net.hi[c];
                CHECK(0 <= i && i < j && j < 2 * P);
                if (v[i] > v[j]) std::swap(v[i], v[j]);
            }
            for (int i = 1; i < 2 * P; ++i) CHECK(v[i - 1] <= v[i]);
        }
}

template <int... N>
static void check_sort_networks(std::integer_sequence<int, N...>) {
    (check_sort_network<N + 1>(), ...);
}

static void check_arena() {
    using irf::host::Arena;
    using irf::host::round_up;
    const size_t page = irf::host::kArenaAlign, pages = 257;
    CHECK(round_up(0) == 0 && round_up(1) == page && round_up(page) == page && round_up(page + 1) == 2 * page);
    Arena a;
    a.reset(pages * page);
    CHECK(a.used() == 0 && a.free_blocks() == 1);
    // exhaustion: one page at a time until nothing fits
    std::vector<size_t> offs;
    size_t off = 0;
    while (a.alloc(1, &off)) offs.push_back(off);
    CHECK(offs.size() == pages && a.used() == pages * page && a.free_blocks() == 0);
    for (size_t i = 0; i < offs.size(); ++i) CHECK(offs[i] == i * page);  // first fit, in order
    // free every other page, then the rest: everything merges back
    for (size_t i = 0; i < offs.size(); i += 2) a.release(offs[i], 1);
    CHECK(a.free_blocks() == (pages + 1) / 2);
    CHECK(!a.alloc(2 * page, &off));  // fragmented: no two adjacent free pages
    for (size_t i = 1; i < offs.size(); i += 2) a.release(offs[i], page);
    CHECK(a.used() == 0 && a.free_blocks() == 1);
    CHECK(a.alloc(pages * page, &off) && off == 0);
    a.release(0, pages * page);
    // random allocations and releases against a page bitmap
    std::mt19937 rng(12013972);
    std::vector<char> busy(pages, 0);
    struct Block { size_t off, bytes; };
    std::vector<Block> live;
    for (int step = 0; step < 20000; ++step) {
        if (live.empty() || rng() % 3 != 0) {
            const size_t bytes = 1 + rng() % (9 * page);
            const size_t np = round_up(bytes) / page;
            // the model's first fit
            size_t want = SIZE_MAX;
            for (size_t p = 0; p + np <= pages && want == SIZE_MAX; ++p) {
                bool fits = true;
                for (size_t q = p; q < p + np; ++q) fits = fits && !busy[q];
                if (fits) want = p;
            }
            size_t got = 0;
            const bool ok = a.alloc(bytes, &got);
            CHECK(ok == (want != SIZE_MAX));
            if (ok) {
                CHECK(got == want * page);
                for (size_t q = want; q < want + np; ++q) busy[q] = 1;
                live.push_back({got, bytes});
            }
        } else {
            const size_t i = rng() % live.size();
            const Block b = live[i];
            a.release(b.off, b.bytes);
            for (size_t q = b.off / page; q < (b.off + round_up(b.bytes)) / page; ++q) busy[q] = 0;
            live[i] = live.back();
            live.pop_back();
        }
        size_t used = 0;
        for (size_t q = 0; q < pages; ++q) used += busy[q] ? page : 0;
        CHECK(a.used() == used);
    }
    for (const Block &b : live) a.release(b.off, b.bytes);
    CHECK(a.used() == 0 && a.free_blocks() == 1);
}

static void check_validation() {
    using namespace irf::host;
    CHECK(check_common(1, 1, 1, IRF_U8, 3) == IRF_OK);
    CHECK(check_common(IRF_MAX_DIM, IRF_MAX_DIM, 1, IRF_U16, IRF_MAX_WINDOW) == IRF_OK);
    CHECK(check_common(0, 1, 1, IRF_U8, 3) == IRF_ERR_DIMS);
    CHECK(check_common(IRF_MAX_DIM + 1, 1, 1, IRF_U8, 3) == IRF_ERR_DIMS);
    CHECK(check_common(1, 1, 0, IRF_U8, 3) == IRF_ERR_DIMS);
    CHECK(check_common(1, 1, 1, (irf_dtype)3, 3) == IRF_ERR_DTYPE);
    CHECK(check_common(1, 1, 1, IRF_U8, 4) == IRF_ERR_WINDOW);
    CHECK(check_common(1, 1, 1, IRF_U8, IRF_MAX_WINDOW + 2) == IRF_ERR_WINDOW);
    CHECK(check_batch_frame(8, 8, IRF_U8, IRF_MAX_BATCH_WINDOW) == IRF_OK);
    CHECK(check_batch_frame(8, 8, IRF_U8, IRF_MAX_BATCH_WINDOW + 2) == IRF_ERR_WINDOW);
    // pitches: at least one row, below 2^24; spans below 4 GiB; strides at least one frame
    CHECK(check_layout(640, 0, 320, 240, 1, 2) == IRF_OK);
    CHECK(check_layout(639, 0, 320, 240, 1, 2) == IRF_ERR_PITCH);
    CHECK(check_layout(kMaxPitch, 0, 1, 2, 1, 1) == IRF_OK);
    CHECK(check_layout(kMaxPitch + 1, 0, 1, 2, 1, 1) == IRF_ERR_PITCH);
    CHECK(check_layout(kMaxPitch, 0, 1, 257, 1, 1) == IRF_OK);   // span 256 * (2^24 - 1) + 1 < 2^32
    CHECK(check_layout(kMaxPitch, 0, 1, 258, 1, 1) == IRF_ERR_PITCH);
    CHECK(check_layout(640, 640 * 240, 320, 240, 4, 2) == IRF_OK);
    CHECK(check_layout(640, 640 * 240 - 1, 320, 240, 4, 2) == IRF_ERR_PITCH);
    // spans: last byte included, one past excluded
    const Span s = span_of(reinterpret_cast<void *>(uintptr_t(1) << 32), 640, 0, 320, 240, 1, 2);
    CHECK(s.hi - s.lo == 640u * 239u + 640u);
    CHECK(overlap(s, Span{s.hi - 1, s.hi + 10}));
    CHECK(!overlap(s, Span{s.hi, s.hi + 10}));
    CHECK(!overlap(s, Span{s.lo - 10, s.lo}));
    CHECK(is16(reinterpret_cast<void *>(uintptr_t(64))) && !is16(reinterpret_cast<void *>(uintptr_t(72))));
}

int main() {
    check_sort_networks(std::make_integer_sequence<int, 16>{});
    check_merge_network<1>();
    check_merge_network<2>();
    check_merge_network<4>();
    check_merge_network<8>();
    check_merge_network<16>();
    check_merge_network<32>();
    check_merge_network<64>();
    check_arena();
    check_validation();
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("ok\n");
    return 0;
}
