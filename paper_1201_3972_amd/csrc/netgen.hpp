// netgen.hpp -- compile-time comparator networks used by the median selection.
//
// Pure constexpr C++ (no HIP), so the host tests can compile it with g++ and
// check the networks exhaustively (0-1 principle) without a GPU.
//
// Batcher's odd-even merge sort, written for any n: the network for the next
// power of two with every comparator that touches an index >= n removed.  Those
// comparators would only ever meet +infinity padding, so the pruned network still
// sorts n inputs.  (K. E. Batcher, "Sorting networks and their applications",
// AFIPS 1968; the index form follows Knuth, TAOCP vol. 3, 5.3.4.)
#pragma once

namespace irf {
namespace net {

constexpr int imin(int a, int b) { return a < b ? a : b; }

// Calls f(i, j) for every comparator (i < j) of the n-input network, in order.
template <typename F>
constexpr void odd_even_merge(int n, F &&f) {
    for (int p = 1; p < n; p += p)
        for (int k = p; k >= 1; k /= 2)
            for (int j = k % p; j + k <= n - 1; j += 2 * k)
                for (int i = 0; i <= imin(k - 1, n - j - k - 1); ++i)
                    if ((i + j) / (2 * p) == (i + j + k) / (2 * p)) f(i + j, i + j + k);
}

constexpr int count_comparators(int n) {
    int c = 0;
    odd_even_merge(n, [&](int, int) { ++c; });
    return c;
}

template <int N>
struct Network {
    static constexpr int size = count_comparators(N);
    int lo[size > 0 ? size : 1];
    int hi[size > 0 ? size : 1];
    constexpr Network() : lo(), hi() {
        int c = 0;
        odd_even_merge(N, [&](int i, int j) {
            lo[c] = i;
            hi[c] = j;
            ++c;
        });
    }
};

template <int N>
inline constexpr Network<N> network{};

// The last stage of the odd-even merge sort on 2P inputs: it merges two sorted
// halves [0, P) and [P, 2P) into one sorted sequence (Batcher's merge).
template <typename F>
constexpr void odd_even_merge_stage(int P, F &&f) {
    const int n = 2 * P, p = P;
    for (int k = p; k >= 1; k /= 2)
        for (int j = k % p; j + k <= n - 1; j += 2 * k)
            for (int i = 0; i <= imin(k - 1, n - j - k - 1); ++i)
                if ((i + j) / (2 * p) == (i + j + k) / (2 * p)) f(i + j, i + j + k);
}

constexpr int count_merge_comparators(int P) {
    int c = 0;
    odd_even_merge_stage(P, [&](int, int) { ++c; });
    return c;
}

template <int P>
struct MergeNetwork {
    static constexpr int size = count_merge_comparators(P);
    int lo[size > 0 ? size : 1];
    int hi[size > 0 ? size : 1];
    constexpr MergeNetwork() : lo(), hi() {
        int c = 0;
        odd_even_merge_stage(P, [&](int i, int j) {
            lo[c] = i;
            hi[c] = j;
            ++c;
        });
    }
};

template <int P>
inline constexpr MergeNetwork<P> merge_network{};

constexpr int pow2_at_least(int n) {
    int p = 1;
    while (p < n) p *= 2;
    return p;
}

}  // namespace net
}  // namespace irf
