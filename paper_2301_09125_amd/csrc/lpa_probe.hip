// lpa_probe.hip -- calibration of the roofline the vote kernels are held to.
//
// Every vote round reads, per arc, its column (streamed) and the label of
// the column's vertex (a 4-byte gather at an address the column decides).
// gather_probe_k performs exactly that access pattern and nothing else: a
// wavefront streams 512 indices (8 per lane, 64 apart, every load issued
// unconditionally) and gathers the 512 table entries they name, so its rate
// over an index stream with a given footprint and skew is the ceiling of any
// kernel that gathers one label per arc from such a stream.

#include "lpa_internal.h"

namespace lpa {

__global__ __launch_bounds__(256) void gather_probe_k(const uint32_t *__restrict__ idx, uint64_t m,
                                                      const uint32_t *__restrict__ table, uint32_t table_n,
                                                      uint32_t *__restrict__ out) {
    const uint64_t lane = threadIdx.x & 63;
    const uint64_t wave = ((uint64_t)blockIdx.x * 256 + threadIdx.x) >> 6;
    const uint64_t nw = ((uint64_t)gridDim.x * 256) >> 6;
    uint32_t acc = 0;
    for (uint64_t base = wave * 512; base < m; base += nw * 512) {
        uint32_t u[8], x[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const uint64_t k = base + lane + 64 * j;
            u[j] = idx[k < m ? k : 0];
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) x[j] = table[min(u[j], table_n - 1)];  // clamped: never out of bounds
#pragma unroll
        for (int j = 0; j < 8; ++j) acc += (base + lane + 64 * j < m) ? x[j] : 0u;
    }
    out[(uint64_t)blockIdx.x * 256 + threadIdx.x] = acc;  // keeps the gathers
}

hipError_t launch_gather_probe(const uint32_t *idx, uint64_t m, const uint32_t *table, uint32_t table_n,
                               uint32_t *out, uint32_t grid, hipStream_t s) {
    gather_probe_k<<<grid, 256, 0, s>>>(idx, m, table, table_n, out);
    return hipGetLastError();
}

}  // namespace lpa
