// lpa_noalloc.hip -- modularity (Section 1) without any allocation, for
// callers that cannot allocate device or pinned memory (code between HIP
// graph captures, serving loops, harnesses that forbid hipMalloc).
//
// The scratch lives in one file-scope device array of fixed size.  Each GPU
// that loads the library holds its own copy until the process ends; its
// address on a device is looked up once (lpa_init calls noalloc_attach with
// that device current) and only that address is handed to kernels and
// copies.  Every call on a GPU shares that GPU's copy and finds the previous
// call's contents there: the community sums, the two totals and the error
// word are cleared by a fill kernel at the start of each call, the rest is
// fully overwritten.  Calls that overlap on one GPU (two streams, two
// threads) race on it.
//
// The sums are the same exact integers as lpa_modularity's; the kernels read
// the CSR as the caller stores it (no binning, no relabelled copy), one
// wavefront per 64 rows with long rows summed by the whole wavefront.

#include <cstring>
#include <mutex>

#include "lpa.h"
#include "lpa_internal.h"

namespace lpa {

typedef unsigned long long u64;

// Layout of the scratch, in u64 words: K (community sums) for up to
// kNoAllocMaxN labels, the two totals, the error word, the five result
// words, then the sum-of-squares partials of kNoAllocParts blocks.
constexpr uint32_t kNoAllocMaxN = LPA_NOALLOC_MAX_N;
constexpr uint32_t kNoAllocParts = 1024;
constexpr size_t kOffSums = kNoAllocMaxN;
constexpr size_t kOffErr = kOffSums + 2;
constexpr size_t kOffOut = kOffSums + 8;
constexpr size_t kOffParts = kOffSums + 16;
constexpr size_t kScratchWords = kOffParts + 2 * (size_t)kNoAllocParts;

static __device__ __align__(256) unsigned long long scratch[kScratchWords];

constexpr int kMaxDevices = 64;
static unsigned long long *g_scratch[kMaxDevices];
static std::mutex g_scratch_mu;

hipError_t noalloc_attach(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch[device]) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[device] = static_cast<unsigned long long *>(p);
    return hipSuccess;
}

static lpa_status na_status(hipError_t e) {
    return e == hipSuccess ? LPA_OK : e == hipErrorOutOfMemory ? LPA_ENOMEM : LPA_EDEVICE;
}

}  // namespace lpa

using namespace lpa;

#define NA_TRY(expr)                                 \
    do {                                             \
        const hipError_t _e = (expr);                \
        if (_e != hipSuccess) return na_status(_e); \
    } while (0)

extern "C" lpa_status lpa_modularity_noalloc(lpa_ctx *c, const lpa_csr *g, const uint32_t *labels, double *q_out,
                                             uint64_t *terms) {
    if (!c || !q_out || !g) return LPA_EINVAL;
    if (!g->row_ptr || (g->m > 0 && !g->col) || (g->n == 0 && g->m != 0)) return LPA_EINVAL;
    if (g->n && !labels) return LPA_EINVAL;
    if (g->n > kNoAllocMaxN) return LPA_ETOOLARGE;
    *q_out = 0.0;
    if (terms) std::memset(terms, 0, 4 * sizeof(uint64_t));
    if (g->n == 0) return LPA_OK;
    const int dev = ctx_device(c);
    if (dev < 0 || dev >= kMaxDevices) return LPA_EDEVICE;
    NA_TRY(hipSetDevice(dev));
    NA_TRY(noalloc_attach(dev));  // done by lpa_init; a no-op unless that lookup failed
    unsigned long long *S;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        S = g_scratch[dev];
    }
    if (!S) return LPA_EDEVICE;
    const hipStream_t s = ctx_stream(c);
    const uint32_t n = g->n;
    u64 *K = S, *sums = S + kOffSums, *out = S + kOffOut, *parts = S + kOffParts;
    uint32_t *err = reinterpret_cast<uint32_t *>(S + kOffErr);
    NA_TRY(launch_modularity_any(Graph{g->row_ptr, g->col, g->w, n, g->m}, labels, K, sums, err, parts,
                                 kNoAllocParts, out, s));
    u64 res[5];
    NA_TRY(hipMemcpyAsync(res, out, sizeof(res), hipMemcpyDeviceToHost, s));
    NA_TRY(hipStreamSynchronize(s));
    const uint32_t errbits = (uint32_t)res[4];
    if (errbits) return LPA_EINVAL;  // a malformed row_ptr, a col value or a label >= n
    const unsigned __int128 sk2 = ((unsigned __int128)res[1] << 64) | (unsigned __int128)res[0];
    const u64 two_m = res[2], sigma_in = res[3];
    double q = 0.0;
    if (two_m > 0) {
        const double W = (double)two_m;
        q = (double)sigma_in / W - (double)sk2 / (W * W);
    }
    *q_out = q;
    if (terms) {
        terms[0] = two_m;
        terms[1] = sigma_in;
        terms[2] = (u64)sk2;
        terms[3] = (u64)(sk2 >> 64);
    }
    return LPA_OK;
}
