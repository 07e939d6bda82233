// lpa_sortnet.h -- Batcher's odd-even merge sorting network, built at
// compile time, for sorting a short row's labels in one lane's registers.
//
// Every compare-exchange (a, b) of the network has a < b and leaves the
// smaller key at a.  Restricting the network for 2^k inputs to the pairs
// with b < D sorts D inputs: positions D .. 2^k - 1 can be taken to hold
// +infinity, and a compare-exchange with +infinity at b changes nothing.
// Plain C++17: the host test compiles this header with g++.
#pragma once

#include <cstdint>

namespace lpa {

constexpr int kSortNetMax = 32;    // largest network: 32 inputs

// The internal CSR's column (and weight) arrays hold this many readable
// entries past their last arc, so a lane may read kSortNetMax arcs from any
// row start without a bound check (what it reads past its row is masked).
constexpr int kLaneArcPad = kSortNetMax;
constexpr int kSortNetPairs = 192;  // Batcher's network for 32 inputs has 191

struct SortNet {
    uint8_t a[kSortNetPairs];
    uint8_t b[kSortNetPairs];
    int n;
};

// The compare-exchanges of Batcher's odd-even merge sort for N = 2^k inputs
// (merges of sorted runs of length p = 1, 2, 4, ...; within a merge, the
// comparisons at distance k = p, p/2, ..., 1), keeping those with b < D.
constexpr SortNet sort_net(int N, int D) {
    SortNet r{};
    r.n = 0;
    for (int p = 1; p < N; p <<= 1)
        for (int k = p; k >= 1; k >>= 1)
            for (int j = k % p; j + k < N; j += 2 * k)
                for (int i = 0; i < k && i + j + k < N; ++i)
                    if ((i + j) / (2 * p) == (i + j + k) / (2 * p) && i + j + k < D) {
                        r.a[r.n] = (uint8_t)(i + j);
                        r.b[r.n] = (uint8_t)(i + j + k);
                        ++r.n;
                    }
    return r;
}

// The smallest power of two >= d (d >= 1).
constexpr int sort_net_size(int d) {
    int n = 1;
    while (n < d) n <<= 1;
    return n;
}

// The network that sorts D inputs (D <= kSortNetMax).
template <int D>
struct SortNetFor {
    static_assert(D >= 1 && D <= kSortNetMax, "network size");
    static constexpr SortNet net = sort_net(sort_net_size(D), D);
};

}  // namespace lpa
