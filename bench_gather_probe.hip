// bench_gather_probe.hip -- bench-only calibration library (libgather_probe.so),
// built and loaded by `bench.py --gather-ceiling`; not part of liblpa.so.
//
// A vote round reads, per arc, its column (streamed) and the label of the
// column's vertex (a 4-byte gather at an address the column decides).
// gather_probe_k performs exactly that access pattern and nothing else: a
// wavefront streams 512 indices (8 per lane, 64 apart, every load issued
// unconditionally) and gathers the 512 table entries they name, so its rate
// over an index stream with a given footprint and skew is the ceiling of any
// kernel that gathers one label per arc from such a stream.

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

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

}  // namespace

// Gathers per second (*rate) of table[idx[k]], k < m, over `reps` timed
// passes (one untimed pass first) on `stream` (a hipStream_t, NULL = the null
// stream) of the current device.  idx: device u32[m]; table: device
// u32[table_n] (indices at or above table_n read the last entry).  Returns 0,
// -1 for a NULL pointer or a zero size, or the HIP error code.
extern "C" int gather_probe_rate(const uint32_t *idx, uint64_t m, const uint32_t *table, uint32_t table_n,
                                 uint32_t reps, void *stream, double *rate) {
    if (!idx || !table || !rate || m == 0 || table_n == 0 || reps == 0) return -1;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    int dev = 0, ncu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return (int)e;
    const uint32_t grid = (uint32_t)(ncu > 0 ? ncu : 256) * 16;
    uint32_t *out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    e = hipMalloc(&out, (size_t)grid * 256 * sizeof(uint32_t));
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) {
        gather_probe_k<<<grid, 256, 0, s>>>(idx, m, table, table_n, out);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (uint32_t r = 0; r < reps && e == hipSuccess; ++r) {
        gather_probe_k<<<grid, 256, 0, s>>>(idx, m, table, table_n, out);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (out) (void)hipFree(out);
    if (e != hipSuccess) return (int)e;
    *rate = ms > 0.f ? (double)m * reps / ((double)ms * 1e-3) : 0.0;
    return 0;
}
