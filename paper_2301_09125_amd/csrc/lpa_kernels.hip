// lpa_kernels.hip -- gfx950 kernels of the RAK label-propagation library.
//
// Method (arXiv 2301.09125, Section 3.2): in every round each vertex adopts
// the label with the largest total edge weight among its neighbours (plus a
// self weight on its own label, the Section 3.1.2 self-loop), ties going to
// the lowest label; rounds are synchronous (read L_old, write L_new).
//
// A vote is the max over candidate labels of the 64-bit key
//     (tally << 32) | ~label,
// which orders by tally first and, among equal tallies, prefers the lowest
// label.  Tallies are u32 (the runtime rejects weighted degrees >= 2^32), all
// accumulation is integer, so results do not depend on the order in which
// atomics land: the labels are deterministic.
//
// Degree bins (chosen once per run):
//   vote_thread_k  1 <= d <= 8     one lane, registers, pairwise tally
//   vote_group_k   d <= 32         16-lane group, LDS open-addressing table
//   vote_wave_k    d <= 256        one wavefront, LDS table
//   vote_hub_k     d > 256         256-thread block per chunk of <= 2048 arcs,
//                                  LDS table; longer rows flush their chunk
//                                  tallies into a global slab (hub_reduce_k,
//                                  hub_final_k finish the vote)
// Hashtable slots are u64 (label << 32 | tally); EMPTY has the label field all
// ones, a value no label takes (labels < n <= 2^32 - 2).  A label is claimed
// with one 64-bit CAS carrying its first weight, later hits add to the low
// half, so a slot never holds a label without its weight.
//
// Every vertex's own current label is tallied in registers and reduced
// across lanes instead of going through the table: in late rounds most
// neighbours share it, and that would serialise the table's atomics.

#include "lpa_internal.h"

namespace lpa {

#define EMPTY_SLOT 0xFFFFFFFF00000000ull

typedef unsigned long long u64;

// lowbias32 integer hash (C. Wellons, "Prospecting for Hash Functions", 2018)
__device__ __forceinline__ uint32_t hmix(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

// Make this wavefront's LDS writes visible to its other lanes.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ u64 umax64(u64 a, u64 b) { return a > b ? a : b; }

// slot (label << 32 | tally)  ->  vote key (tally << 32 | ~label)
__device__ __forceinline__ u64 slot_key(u64 x) { return (x << 32) | (uint32_t)~(uint32_t)(x >> 32); }

__device__ __forceinline__ u64 own_key(uint32_t own, u64 tally) {
    return (tally << 32) | (uint32_t)~own;
}

__device__ __forceinline__ uint32_t next_pow2(uint32_t x) {
    return x <= 1 ? 1u : 1u << (32 - __clz(x - 1));
}

// Read arc k: returns L_old[col[k]] and its weight; an out-of-range column
// raises ERR_COL and is read as vertex 0 so no access leaves the arrays.
__device__ __forceinline__ uint32_t arc_label(const RoundArgs &a, uint64_t k, uint32_t &wv) {
    uint32_t u = a.g.col[k];
    if (u >= a.g.n) {
        atomicOr(a.err, ERR_COL);
        u = 0;
    }
    wv = a.g.w ? a.g.w[k] : 1u;
    return a.L_old[u];
}

// Insert (lab, wv) into an LDS table of mask+1 slots with linear probing.
// The caller guarantees more slots than distinct labels.
__device__ __forceinline__ void lds_insert(u64 *T, uint32_t mask, uint32_t lab, uint32_t wv) {
    uint32_t h = hmix(lab) & mask;
    const u64 desired = ((u64)lab << 32) | wv;
    for (;;) {
        u64 prev = atomicCAS(&T[h], EMPTY_SLOT, desired);
        if (prev == EMPTY_SLOT) return;
        if ((uint32_t)(prev >> 32) == lab) {
            atomicAdd(&T[h], (u64)wv);
            return;
        }
        h = (h + 1) & mask;
    }
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}
__device__ __forceinline__ u64 wave_max64(u64 x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x = umax64(x, __shfl_xor(x, off, 64));
    return x;
}

// ---------------------------------------------------------------- fills --

__global__ void iota2_k(uint32_t *a, uint32_t *b, uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        a[i] = i;
        if (b) b[i] = i;
    }
}
__global__ void fill64_k(u64 *p, u64 v, uint64_t count) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void fill32_k(uint32_t *p, uint32_t v, uint64_t count) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void copy32_k(uint32_t *dst, const uint32_t *src, uint64_t count) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}
__global__ void check_labels_k(const uint32_t *labels, uint32_t n, uint32_t *err) {
    bool bad = false;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        bad |= labels[i] >= n;
    if (bad) atomicOr(err, ERR_LABEL);
}

static inline unsigned grid_for(uint64_t count, unsigned per_block, unsigned cap) {
    uint64_t g = (count + per_block - 1) / per_block;
    if (g < 1) g = 1;
    return (unsigned)(g < cap ? g : cap);
}

hipError_t launch_fill_u32_iota(uint32_t *a, uint32_t *b, uint32_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    iota2_k<<<grid_for(n, 256, 8192), 256, 0, s>>>(a, b, n);
    return hipGetLastError();
}
hipError_t launch_fill_u64(u64 *p, u64 v, uint64_t count, hipStream_t s) {
    if (count == 0) return hipSuccess;
    fill64_k<<<grid_for(count, 256, 8192), 256, 0, s>>>(p, v, count);
    return hipGetLastError();
}
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, uint64_t count, hipStream_t s) {
    if (count == 0) return hipSuccess;
    fill32_k<<<grid_for(count, 256, 8192), 256, 0, s>>>(p, v, count);
    return hipGetLastError();
}
hipError_t launch_copy_u32(uint32_t *dst, const uint32_t *src, uint64_t count, hipStream_t s) {
    if (count == 0) return hipSuccess;
    copy32_k<<<grid_for(count, 256, 8192), 256, 0, s>>>(dst, src, count);
    return hipGetLastError();
}
hipError_t launch_check_labels(const uint32_t *labels, uint32_t n, uint32_t *err, hipStream_t s) {
    if (n == 0) return hipSuccess;
    check_labels_k<<<grid_for(n, 256, 4096), 256, 0, s>>>(labels, n, err);
    return hipGetLastError();
}

// -------------------------------------------------------------- binning --

__device__ __forceinline__ int bin_of(uint64_t d, uint32_t tmax, uint32_t gmax, uint32_t wmax) {
    return d == 0 ? BIN_ZERO : d <= tmax ? BIN_THREAD : d <= gmax ? BIN_GROUP : d <= wmax ? BIN_WAVE : BIN_HUB;
}

// Bin of vertex v, or -1 when its row_ptr entries are malformed.
__device__ __forceinline__ int vertex_bin(const Graph &g, uint32_t v, uint32_t tmax, uint32_t gmax,
                                          uint32_t wmax, uint64_t &d, bool &bad) {
    uint64_t a = g.rp[v], b = g.rp[v + 1];
    bad = (b < a) || (b > g.m) || (v == 0 && a != 0) || (v + 1 == g.n && b != g.m);
    d = bad ? 0 : b - a;
    return bad ? -1 : bin_of(d, tmax, gmax, wmax);
}

__global__ __launch_bounds__(256) void bin_count_k(Graph g, uint32_t tmax, uint32_t gmax, uint32_t wmax,
                                                   uint32_t *blk_counts, u64 *blk_arcs, uint32_t nblk,
                                                   uint32_t *err) {
    __shared__ uint32_t cnt[NBINS];
    __shared__ u64 arcs[NBINS];
    if (threadIdx.x < NBINS) {
        cnt[threadIdx.x] = 0;
        arcs[threadIdx.x] = 0;
    }
    __syncthreads();
    const uint32_t v = blockIdx.x * 256 + threadIdx.x;
    int bin = -1;
    uint64_t d = 0;
    if (v < g.n) {
        bool bad;
        bin = vertex_bin(g, v, tmax, gmax, wmax, d, bad);
        if (bad) atomicOr(err, ERR_ROWPTR);
    }
#pragma unroll
    for (int b = 0; b < NBINS; ++b) {
        u64 mask = __ballot(bin == b);
        if ((threadIdx.x & 63) == 0 && mask) atomicAdd(&cnt[b], (uint32_t)__popcll(mask));
    }
    if (bin > 0) atomicAdd(&arcs[bin], (u64)d);
    __syncthreads();
    if (threadIdx.x < NBINS) {
        blk_counts[threadIdx.x * nblk + blockIdx.x] = cnt[threadIdx.x];
        blk_arcs[threadIdx.x * nblk + blockIdx.x] = arcs[threadIdx.x];
    }
}

// One 1024-thread block: turn per-block counts into global offsets of a
// single array holding the bins back to back (bin 0 first).
__global__ __launch_bounds__(1024) void bin_scan_k(uint32_t *blk_counts, const u64 *blk_arcs, uint32_t nblk,
                                                   uint32_t *totals, u64 *arc_totals) {
    __shared__ uint32_t sh[1024];
    __shared__ u64 sa[1024];
    const uint32_t t = threadIdx.x;
    const uint32_t per = (nblk + 1023) / 1024;
    const uint32_t lo = min(t * per, nblk), hi = min(lo + per, nblk);
    uint32_t base = 0;
    for (int bin = 0; bin < NBINS; ++bin) {
        uint32_t *c = blk_counts + (size_t)bin * nblk;
        const u64 *ar = blk_arcs + (size_t)bin * nblk;
        uint32_t s = 0;
        u64 as = 0;
        for (uint32_t i = lo; i < hi; ++i) {
            s += c[i];
            as += ar[i];
        }
        sh[t] = s;
        sa[t] = as;
        __syncthreads();
        for (uint32_t off = 1; off < 1024; off <<= 1) {
            uint32_t x = t >= off ? sh[t - off] : 0;
            u64 y = (t & (2 * off - 1)) == 0 && t + off < 1024 ? sa[t + off] : 0;
            __syncthreads();
            sh[t] += x;
            sa[t] += y;
            __syncthreads();
        }
        uint32_t run = base + sh[t] - s;
        for (uint32_t i = lo; i < hi; ++i) {
            uint32_t x = c[i];
            c[i] = run;
            run += x;
        }
        const uint32_t total = sh[1023];
        if (t == 0) {
            totals[bin] = total;
            arc_totals[bin] = sa[0];
        }
        base += total;
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void bin_scatter_k(Graph g, uint32_t tmax, uint32_t gmax, uint32_t wmax,
                                                     const uint32_t *blk_offsets, uint32_t nblk,
                                                     uint32_t *order) {
    __shared__ uint32_t wcnt[4][NBINS];
    const uint32_t v = blockIdx.x * 256 + threadIdx.x;
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int bin = -1;
    if (v < g.n) {
        uint64_t d;
        bool bad;
        bin = vertex_bin(g, v, tmax, gmax, wmax, d, bad);
    }
    uint32_t rank = 0;
#pragma unroll
    for (int b = 0; b < NBINS; ++b) {
        u64 mask = __ballot(bin == b);
        if (lane == 0) wcnt[wave][b] = (uint32_t)__popcll(mask);
        if (bin == b) rank = (uint32_t)__popcll(mask & ((1ull << lane) - 1));
    }
    __syncthreads();
    if (bin > 0) {
        uint32_t off = blk_offsets[(size_t)bin * nblk + blockIdx.x];
        for (uint32_t w = 0; w < wave; ++w) off += wcnt[w][bin];
        order[off + rank] = v;
    }
}

__global__ void gather_rows_k(const uint64_t *rp, const uint32_t *verts, uint32_t count, uint64_t *out) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
        uint32_t v = verts[i];
        out[2 * i] = rp[v];
        out[2 * i + 1] = rp[v + 1];
    }
}

hipError_t launch_bin_count(const Graph &g, uint32_t tmax, uint32_t gmax, uint32_t wmax, uint32_t *blk_counts,
                            u64 *blk_arcs, uint32_t nblk, uint32_t *err, hipStream_t s) {
    bin_count_k<<<nblk, 256, 0, s>>>(g, tmax, gmax, wmax, blk_counts, blk_arcs, nblk, err);
    return hipGetLastError();
}
hipError_t launch_bin_scan(uint32_t *blk_counts, const u64 *blk_arcs, uint32_t nblk, uint32_t *totals,
                           u64 *arc_totals, hipStream_t s) {
    bin_scan_k<<<1, 1024, 0, s>>>(blk_counts, blk_arcs, nblk, totals, arc_totals);
    return hipGetLastError();
}
hipError_t launch_bin_scatter(const Graph &g, uint32_t tmax, uint32_t gmax, uint32_t wmax,
                              const uint32_t *blk_offsets, uint32_t nblk, uint32_t *order, hipStream_t s) {
    bin_scatter_k<<<nblk, 256, 0, s>>>(g, tmax, gmax, wmax, blk_offsets, nblk, order);
    return hipGetLastError();
}
hipError_t launch_gather_rows(const uint64_t *rp, const uint32_t *verts, uint32_t count, uint64_t *out,
                              hipStream_t s) {
    if (count == 0) return hipSuccess;
    gather_rows_k<<<grid_for(count, 256, 4096), 256, 0, s>>>(rp, verts, count, out);
    return hipGetLastError();
}

// ---------------------------------------------------------- vote: lanes --

// One lane per vertex, degree 1..kThreadMaxCap: the row sits in registers
// and every neighbour label is tallied against every other (upper triangle).
__global__ __launch_bounds__(256) void vote_thread_k(RoundArgs a, const uint32_t *__restrict__ list, uint32_t cnt) {
    constexpr int D = kThreadMaxCap;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t stride = gridDim.x * 256;
    u64 wchg = 0;
    for (uint32_t base = blockIdx.x * 256 + (threadIdx.x & ~63u); base < cnt; base += stride) {
        const uint32_t i = base + lane;
        bool ch = false;
        if (i < cnt) {
            const uint32_t v = list[i];
            const uint64_t b = a.g.rp[v];
            const uint32_t d = (uint32_t)(a.g.rp[v + 1] - b);
            const uint32_t own = a.L_old[v];
            uint32_t lab[D], wt[D], tl[D];
            uint64_t rs = a.sw;
#pragma unroll
            for (int j = 0; j < D; ++j) {
                lab[j] = 0xFFFFFFFFu;  // never a label: matches only other padding
                wt[j] = 0;
                if (j < (int)d) {
                    lab[j] = arc_label(a, b + j, wt[j]);
                    rs += wt[j];
                }
            }
#pragma unroll
            for (int j = 0; j < D; ++j) tl[j] = wt[j] + (lab[j] == own ? a.sw : 0u);
#pragma unroll
            for (int j = 0; j < D; ++j)
#pragma unroll
                for (int k = j + 1; k < D; ++k)
                    if (lab[j] == lab[k]) {
                        tl[j] += wt[k];
                        tl[k] += wt[j];
                    }
            u64 best = a.sw ? own_key(own, a.sw) : 0ull;
#pragma unroll
            for (int j = 0; j < D; ++j)
                if (j < (int)d) best = umax64(best, ((u64)tl[j] << 32) | (uint32_t)~lab[j]);
            const uint32_t nl = best ? ~(uint32_t)best : own;
            a.L_new[v] = nl;
            ch = nl != own;
            if (a.check && rs > 0xFFFFFFFFull) atomicOr(a.err, ERR_WOVF);
        }
        wchg += __popcll(__ballot(ch));
    }
    if (lane == 0 && wchg) atomicAdd(a.changed, wchg);
}

// G lanes per vertex (G divides 64) with a CAP-slot LDS table per group.
// Each wavefront walks its own vertices; no block-wide barrier is needed
// because a group's table is only touched by lanes of its wavefront.
template <int G, int CAP>
__global__ __launch_bounds__(256) void vote_group_k(RoundArgs a, const uint32_t *__restrict__ list, uint32_t cnt) {
    constexpr int GPB = 256 / G;  // groups per block
    constexpr int GPW = 64 / G;   // groups per wavefront
    __shared__ u64 table[GPB * CAP];
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t gl = threadIdx.x & (G - 1);
    u64 *T = table + (threadIdx.x / G) * CAP;
    for (uint32_t s = gl; s < CAP; s += G) T[s] = EMPTY_SLOT;
    wave_sync();
    u64 wchg = 0;
    const uint32_t stride = gridDim.x * GPB;
    for (uint32_t base = blockIdx.x * GPB + (threadIdx.x >> 6) * GPW; base < cnt; base += stride) {
        const uint32_t idx = base + lane / G;
        const bool act = idx < cnt;
        uint32_t v = 0, own = 0;
        uint64_t b = 0, e = 0;
        if (act) {
            v = list[idx];
            b = a.g.rp[v];
            e = a.g.rp[v + 1];
            own = a.L_old[v];
        }
        uint32_t S = next_pow2(2u * (uint32_t)(e - b));
        S = S < (uint32_t)G ? (uint32_t)G : (S > (uint32_t)CAP ? (uint32_t)CAP : S);
        const uint32_t mask = S - 1;
        uint32_t own_w = 0, own_hit = 0;
        uint64_t rs = 0;
        for (uint64_t k = b + gl; k < e; k += G) {
            uint32_t wv;
            const uint32_t lab = arc_label(a, k, wv);
            rs += wv;
            if (lab == own) {
                own_w += wv;
                own_hit = 1;
            } else {
                lds_insert(T, mask, lab, wv);
            }
        }
        wave_sync();
        u64 best = 0;
        for (uint32_t s = gl; s < S; s += G) {
            const u64 x = T[s];
            if (x != EMPTY_SLOT) {
                best = umax64(best, slot_key(x));
                T[s] = EMPTY_SLOT;
            }
        }
#pragma unroll
        for (int off = G / 2; off > 0; off >>= 1) {
            best = umax64(best, __shfl_xor(best, off, 64));
            own_w += __shfl_xor(own_w, off, 64);
            own_hit |= __shfl_xor(own_hit, off, 64);
            rs += __shfl_xor(rs, off, 64);
        }
        bool ch = false;
        if (act && gl == 0) {
            if (own_hit || a.sw) best = umax64(best, own_key(own, (u64)own_w + a.sw));
            const uint32_t nl = best ? ~(uint32_t)best : own;
            a.L_new[v] = nl;
            ch = nl != own;
            if (a.check && rs + a.sw > 0xFFFFFFFFull) atomicOr(a.err, ERR_WOVF);
        }
        wchg += __popcll(__ballot(ch));
        wave_sync();
    }
    if (lane == 0 && wchg) atomicAdd(a.changed, wchg);
}

hipError_t launch_vote_thread(const RoundArgs &a, const uint32_t *list, uint32_t cnt, int grid_cap,
                              hipStream_t s) {
    if (cnt == 0) return hipSuccess;
    vote_thread_k<<<grid_for(cnt, 256, grid_cap), 256, 0, s>>>(a, list, cnt);
    return hipGetLastError();
}
hipError_t launch_vote_group(const RoundArgs &a, const uint32_t *list, uint32_t cnt, int grid_cap,
                             hipStream_t s) {
    if (cnt == 0) return hipSuccess;
    vote_group_k<kGroupLanes, kGroupSlots>
        <<<grid_for(cnt, 256 / kGroupLanes, grid_cap), 256, 0, s>>>(a, list, cnt);
    return hipGetLastError();
}
hipError_t launch_vote_wave(const RoundArgs &a, const uint32_t *list, uint32_t cnt, int grid_cap,
                            hipStream_t s) {
    if (cnt == 0) return hipSuccess;
    vote_group_k<64, kWaveSlots><<<grid_for(cnt, 4, grid_cap), 256, 0, s>>>(a, list, cnt);
    return hipGetLastError();
}

// ----------------------------------------------------------- vote: hubs --

// Block-wide reductions for 256 threads (4 wavefronts).
struct BlockRed {
    u64 mx[4];
    u64 sum[4];
    u64 sum2[4];
    uint32_t orv[4];
};

__device__ __forceinline__ void block_reduce(BlockRed &R, u64 &mx, u64 &sum, u64 &sum2, uint32_t &orv) {
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    mx = wave_max64(mx);
    sum = wave_sum(sum);
    sum2 = wave_sum(sum2);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) orv |= __shfl_xor(orv, off, 64);
    if (lane == 0) {
        R.mx[wave] = mx;
        R.sum[wave] = sum;
        R.sum2[wave] = sum2;
        R.orv[wave] = orv;
    }
    __syncthreads();
    mx = umax64(umax64(R.mx[0], R.mx[1]), umax64(R.mx[2], R.mx[3]));
    sum = R.sum[0] + R.sum[1] + R.sum[2] + R.sum[3];
    sum2 = R.sum2[0] + R.sum2[1] + R.sum2[2] + R.sum2[3];
    orv = R.orv[0] | R.orv[1] | R.orv[2] | R.orv[3];
}

// Merge (lab, cnt) into hub row h's global slab; a newly claimed slot is
// recorded in the row's touched list so phase 2 visits only used slots.
__device__ __forceinline__ void slab_insert(u64 *S, uint32_t mask, uint32_t *tlist, uint32_t *tcount,
                                            uint32_t lab, uint32_t cnt) {
    uint32_t h = hmix(lab) & mask;
    const u64 desired = ((u64)lab << 32) | cnt;
    for (;;) {
        u64 prev = atomicCAS(&S[h], EMPTY_SLOT, desired);
        if (prev == EMPTY_SLOT) {
            uint32_t pos = atomicAdd(tcount, 1u);
            tlist[pos] = h;
            return;
        }
        if ((uint32_t)(prev >> 32) == lab) {
            atomicAdd(&S[h], (u64)cnt);
            return;
        }
        h = (h + 1) & mask;
    }
}

__global__ __launch_bounds__(256) void vote_hub_k(RoundArgs a, const HubItem *__restrict__ items, uint32_t count,
                                                  uint32_t cap_slots, HubState hs) {
    __shared__ u64 T[kChunkSlotsMax];
    __shared__ BlockRed R;
    for (uint32_t s = threadIdx.x; s < cap_slots; s += 256) T[s] = EMPTY_SLOT;
    __syncthreads();
    u64 bchg = 0;
    for (uint32_t it = blockIdx.x; it < count; it += gridDim.x) {
        const HubItem item = items[it];
        const uint32_t own = a.L_old[item.v];
        uint32_t S = next_pow2(2u * (uint32_t)(item.b1 - item.b0));
        S = S < 64u ? 64u : (S > cap_slots ? cap_slots : S);
        const uint32_t mask = S - 1;
        u64 own_w = 0, rs = 0;
        uint32_t own_hit = 0;
        for (uint64_t k = item.b0 + threadIdx.x; k < item.b1; k += 256) {
            uint32_t wv;
            const uint32_t lab = arc_label(a, k, wv);
            rs += wv;
            if (lab == own) {
                own_w += wv;
                own_hit = 1;
            } else {
                lds_insert(T, mask, lab, wv);
            }
        }
        __syncthreads();
        u64 best = 0;
        if (item.hub == kNoHub) {
            for (uint32_t s = threadIdx.x; s < S; s += 256) {
                const u64 x = T[s];
                if (x != EMPTY_SLOT) {
                    best = umax64(best, slot_key(x));
                    T[s] = EMPTY_SLOT;
                }
            }
            block_reduce(R, best, own_w, rs, own_hit);
            if (threadIdx.x == 0) {
                if (own_hit || a.sw) best = umax64(best, own_key(own, own_w + a.sw));
                const uint32_t nl = best ? ~(uint32_t)best : own;
                a.L_new[item.v] = nl;
                bchg += nl != own;
                if (a.check && rs + a.sw > 0xFFFFFFFFull) atomicOr(a.err, ERR_WOVF);
            }
        } else {
            const uint32_t h = item.hub;
            u64 *slab = hs.slab + hs.slab_off[h];
            const uint32_t smask = hs.slab_mask[h];
            uint32_t *tlist = hs.touched + hs.touched_off[h];
            for (uint32_t s = threadIdx.x; s < S; s += 256) {
                const u64 x = T[s];
                if (x != EMPTY_SLOT) {
                    slab_insert(slab, smask, tlist, &hs.tcount[h], (uint32_t)(x >> 32), (uint32_t)x);
                    T[s] = EMPTY_SLOT;
                }
            }
            block_reduce(R, best, own_w, rs, own_hit);
            if (threadIdx.x == 0) {
                if (own_w) atomicAdd(&hs.own_sum[h], own_w);
                if (own_hit) atomicOr(&hs.own_seen[h], 1u);
                if (a.check) atomicAdd(&hs.rowsum[h], rs);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0 && bchg) atomicAdd(a.changed, bchg);
}

// Phase 2: max key over the slots claimed by a multi-chunk row, clearing
// them for the next round.
__global__ __launch_bounds__(256) void hub_reduce_k(HubState hs, const ReduceItem *__restrict__ items,
                                                    uint32_t count) {
    __shared__ BlockRed R;
    for (uint32_t it = blockIdx.x; it < count; it += gridDim.x) {
        const ReduceItem r = items[it];
        const uint32_t t1 = min(r.t1, hs.tcount[r.hub]);
        if (r.t0 >= t1) continue;  // uniform over the block
        u64 *slab = hs.slab + hs.slab_off[r.hub];
        const uint32_t *tlist = hs.touched + hs.touched_off[r.hub];
        u64 best = 0, z0 = 0, z1 = 0;
        uint32_t z2 = 0;
        for (uint32_t p = r.t0 + threadIdx.x; p < t1; p += 256) {
            const uint32_t s = tlist[p];
            best = umax64(best, slot_key(slab[s]));
            slab[s] = EMPTY_SLOT;
        }
        block_reduce(R, best, z0, z1, z2);
        if (threadIdx.x == 0 && best) atomicMax(&hs.best[r.hub], best);
        __syncthreads();
    }
}

// Phase 3: one lane per multi-chunk row picks the winner and resets the
// row's state for the next round.
__global__ __launch_bounds__(256) void hub_final_k(RoundArgs a, HubState hs, uint32_t count) {
    const uint32_t lane = threadIdx.x & 63;
    u64 wchg = 0;
    for (uint32_t base = blockIdx.x * 256 + (threadIdx.x & ~63u); base < count; base += gridDim.x * 256) {
        const uint32_t i = base + lane;
        bool ch = false;
        if (i < count) {
            const uint32_t v = hs.vertex[i];
            const uint32_t own = a.L_old[v];
            u64 best = hs.best[i];
            if (hs.own_seen[i] || a.sw) best = umax64(best, own_key(own, hs.own_sum[i] + a.sw));
            const uint32_t nl = best ? ~(uint32_t)best : own;
            a.L_new[v] = nl;
            ch = nl != own;
            if (a.check && hs.rowsum[i] + a.sw > 0xFFFFFFFFull) atomicOr(a.err, ERR_WOVF);
            hs.best[i] = 0;
            hs.own_sum[i] = 0;
            hs.own_seen[i] = 0;
            hs.tcount[i] = 0;
            hs.rowsum[i] = 0;
        }
        wchg += __popcll(__ballot(ch));
    }
    if (lane == 0 && wchg) atomicAdd(a.changed, wchg);
}

hipError_t launch_vote_hub(const RoundArgs &a, const HubItem *items, uint32_t count, uint32_t chunk,
                           const HubState &hs, hipStream_t s) {
    if (count == 0) return hipSuccess;
    uint32_t cap = 2 * chunk;
    if (cap > (uint32_t)kChunkSlotsMax) return hipErrorInvalidValue;
    vote_hub_k<<<grid_for(count, 1, 2048), 256, 0, s>>>(a, items, count, cap, hs);
    return hipGetLastError();
}
hipError_t launch_hub_reduce(const HubState &hs, const ReduceItem *items, uint32_t count, hipStream_t s) {
    if (count == 0) return hipSuccess;
    hub_reduce_k<<<grid_for(count, 1, 4096), 256, 0, s>>>(hs, items, count);
    return hipGetLastError();
}
hipError_t launch_hub_final(const RoundArgs &a, const HubState &hs, uint32_t count, hipStream_t s) {
    if (count == 0) return hipSuccess;
    hub_final_k<<<grid_for(count, 256, 1024), 256, 0, s>>>(a, hs, count);
    return hipGetLastError();
}

// ----------------------------------------------------------- modularity --
//
// Q = Sigma_in / 2m - sum_c K_c^2 / (2m)^2 (Section 1).  Integer sums: 2m and
// Sigma_in in u64, K_c in u64 atomics, sum K_c^2 as u128 partials.

__device__ __forceinline__ uint32_t mod_arc(const ModArgs &a, uint64_t k, uint32_t lv, u64 &kv) {
    uint32_t u = a.g.col[k];
    if (u >= a.g.n) {
        atomicOr(a.err, ERR_COL);
        u = 0;
    }
    const uint32_t wv = a.g.w ? a.g.w[k] : 1u;
    kv += wv;
    return a.labels[u] == lv ? wv : 0u;
}

// K[lv] += kv with one atomic for all lanes of the wavefront that share the
// first active lane's label (the common case once labels have merged).
__device__ __forceinline__ void add_community(u64 *K, bool act, uint32_t lv, u64 kv) {
    const u64 actmask = __ballot(act);
    if (!actmask) return;
    const int lead = __ffsll((long long)actmask) - 1;
    const uint32_t ll = __shfl(lv, lead, 64);
    const bool same = act && lv == ll;
    const u64 part = wave_sum(same ? kv : 0ull);
    if ((int)(threadIdx.x & 63) == lead && part) atomicAdd(&K[ll], part);
    if (act && !same && kv) atomicAdd(&K[lv], kv);
}

__global__ __launch_bounds__(256) void mod_small_k(ModArgs a, const uint32_t *__restrict__ list, uint32_t cnt) {
    __shared__ BlockRed R;
    u64 tw = 0, sin = 0;
    for (uint32_t base = blockIdx.x * 256 + (threadIdx.x & ~63u); base < cnt; base += gridDim.x * 256) {
        const uint32_t i = base + (threadIdx.x & 63);
        const bool act = i < cnt;
        u64 kv = 0;
        uint32_t lv = 0;
        if (act) {
            const uint32_t v = list[i];
            lv = a.labels[v];
            for (uint64_t k = a.g.rp[v]; k < a.g.rp[v + 1]; ++k) sin += mod_arc(a, k, lv, kv);
        }
        tw += kv;
        add_community(a.K, act, lv, kv);
    }
    u64 z = 0;
    uint32_t zo = 0;
    block_reduce(R, z, tw, sin, zo);
    if (threadIdx.x == 0) {
        if (tw) atomicAdd(&a.sums[0], tw);
        if (sin) atomicAdd(&a.sums[1], sin);
    }
}

__global__ __launch_bounds__(256) void mod_wave_k(ModArgs a, const uint32_t *__restrict__ list, uint32_t cnt) {
    __shared__ BlockRed R;
    const uint32_t lane = threadIdx.x & 63;
    u64 tw = 0, sin = 0;
    for (uint32_t i = blockIdx.x * 4 + (threadIdx.x >> 6); i < cnt; i += gridDim.x * 4) {
        const uint32_t v = list[i];
        const uint32_t lv = a.labels[v];
        u64 kv = 0;
        for (uint64_t k = a.g.rp[v] + lane; k < a.g.rp[v + 1]; k += 64) sin += mod_arc(a, k, lv, kv);
        kv = wave_sum(kv);
        tw += lane == 0 ? kv : 0;
        if (lane == 0 && kv) atomicAdd(&a.K[lv], kv);
    }
    u64 z = 0;
    uint32_t zo = 0;
    block_reduce(R, z, tw, sin, zo);
    if (threadIdx.x == 0) {
        if (tw) atomicAdd(&a.sums[0], tw);
        if (sin) atomicAdd(&a.sums[1], sin);
    }
}

__global__ __launch_bounds__(256) void mod_hub_k(ModArgs a, const HubItem *__restrict__ items, uint32_t count) {
    __shared__ BlockRed R;
    u64 tw = 0, sin = 0;
    for (uint32_t it = blockIdx.x; it < count; it += gridDim.x) {
        const HubItem item = items[it];
        const uint32_t lv = a.labels[item.v];
        u64 kv = 0, s = 0, z = 0;
        uint32_t zo = 0;
        for (uint64_t k = item.b0 + threadIdx.x; k < item.b1; k += 256) s += mod_arc(a, k, lv, kv);
        block_reduce(R, z, kv, s, zo);
        if (threadIdx.x == 0) {
            tw += kv;
            sin += s;
            if (kv) atomicAdd(&a.K[lv], kv);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (tw) atomicAdd(&a.sums[0], tw);
        if (sin) atomicAdd(&a.sums[1], sin);
    }
}

// Per-block u128 partial sums of K_c^2, written as (lo, hi) pairs.
__global__ __launch_bounds__(256) void mod_sumsq_k(const u64 *__restrict__ K, uint32_t n, u64 *partials) {
    __shared__ unsigned __int128 sh[256];
    unsigned __int128 acc = 0;
    for (uint32_t c = blockIdx.x * 256 + threadIdx.x; c < n; c += gridDim.x * 256) {
        const u64 k = K[c];
        acc += (unsigned __int128)k * k;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (uint32_t off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = (u64)sh[0];
        partials[2 * blockIdx.x + 1] = (u64)(sh[0] >> 64);
    }
}

hipError_t launch_mod_small(const ModArgs &a, const uint32_t *list, uint32_t cnt, hipStream_t s) {
    if (cnt == 0) return hipSuccess;
    mod_small_k<<<grid_for(cnt, 256, 2048), 256, 0, s>>>(a, list, cnt);
    return hipGetLastError();
}
hipError_t launch_mod_wave(const ModArgs &a, const uint32_t *list, uint32_t cnt, hipStream_t s) {
    if (cnt == 0) return hipSuccess;
    mod_wave_k<<<grid_for(cnt, 4, 2048), 256, 0, s>>>(a, list, cnt);
    return hipGetLastError();
}
hipError_t launch_mod_hub(const ModArgs &a, const HubItem *items, uint32_t count, hipStream_t s) {
    if (count == 0) return hipSuccess;
    mod_hub_k<<<grid_for(count, 1, 2048), 256, 0, s>>>(a, items, count);
    return hipGetLastError();
}
hipError_t launch_mod_sumsq(const u64 *K, uint32_t n, u64 *partials, uint32_t nparts, hipStream_t s) {
    mod_sumsq_k<<<nparts, 256, 0, s>>>(K, n, partials);
    return hipGetLastError();
}

}  // namespace lpa
