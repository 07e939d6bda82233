// lpa_rows.h -- walking a caller's CSR without binning (the modularity and
// COPRA kernels that read it as stored).
#pragma once

#include "lpa_device.h"

namespace lpa {

// The first kHeadArcs arcs of a row are taken with the row, the rest in
// chunks of kHeadArcs arcs spread over the grid, so that no wavefront walks
// a hub alone.
constexpr uint64_t kHeadArcs = 4096;

// The row holding arc k < m: the largest r < n with rp[r] <= k (row_ptr
// assumed monotone; on a malformed one the result is still a row < n).
__device__ __forceinline__ uint32_t row_of_arc(const Graph &g, uint64_t k) {
    uint32_t lo = 0, hi = g.n;
    while (hi - lo > 1) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if (g.rp[mid] <= k)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

}  // namespace lpa
