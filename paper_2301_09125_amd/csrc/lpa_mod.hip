// lpa_mod.hip -- modularity (arXiv 2301.09125, Section 1) on the internal
// graph:  Q = Sigma_in / 2m - sum_c K_c^2 / (2m)^2.
//
// Integer sums throughout: 2m and Sigma_in in u64, K_c (summed weighted
// degree of community c, indexed by the label value) in u64, sum K_c^2 as
// u128 block partials added on the host; only the final expression is FP64.
// K_c contributions are first merged per block in an LDS table so that a
// large community costs one global atomic per block, not one per vertex.
//
// Incremental form (labels_prev set): the last round of a plain run already
// summed, over every row, the weight of the arcs whose neighbour held the
// row's own label, i.e. Sigma_in of the labels L' of the round before.  Only
// arcs with an endpoint that changed label in the last round can change
// their term, so the kernels below read the arcs of the changed rows only
// and add, per such arc (v, u, w), w * ([L(v) = L(u)] - [L'(v) = L'(u)]),
// once if u changed too and twice if it did not (the reverse arc (u, v) of
// a symmetric graph carries the same term and is not visited).  K_c still
// takes every vertex, and for unit weights its degree needs no arc at all.

#include "lpa_rows.h"

namespace lpa {

// Grid cap of the row and item loops (grid stride): 16 blocks per CU on a
// 256-CU chip, two or more rounds of the 7 to 8 blocks that fit per CU, so a
// partly filled last round is a small share of the launch.
constexpr unsigned kModGrid = 4096;

constexpr uint32_t kModSlots = 1024;
constexpr uint32_t kEmpty32 = 0xFFFFFFFFu;

struct ModTable {
    uint32_t key[kModSlots];
    u64 val[kModSlots];
    BlockRed R;
};

__device__ __forceinline__ void mod_table_init(ModTable &M) {
    for (uint32_t s = threadIdx.x; s < kModSlots; s += 256) {
        M.key[s] = kEmpty32;
        M.val[s] = 0;
    }
    __syncthreads();
}

__device__ __forceinline__ void mod_table_add(ModTable &M, u64 *K, uint32_t lab, u64 kv) {
    uint32_t h = hmix(lab) & (kModSlots - 1);
    for (int p = 0; p < 16; ++p) {
        const uint32_t prev = atomicCAS(&M.key[h], kEmpty32, lab);
        if (prev == kEmpty32 || prev == lab) {
            atomicAdd(&M.val[h], kv);
            return;
        }
        h = (h + 1) & (kModSlots - 1);
    }
    atomicAdd(&K[lab], kv);  // table crowded: go straight to memory
}

// Per-wavefront peel of the first active lane's label, then the LDS table.
__device__ __forceinline__ void add_community(ModTable &M, u64 *K, bool act, uint32_t lv, u64 kv) {
    const u64 actmask = __ballot(act);
    if (!actmask) return;
    const int lead = __ffsll((long long)actmask) - 1;
    const uint32_t ll = (uint32_t)__builtin_amdgcn_readlane((int)lv, lead);
    const bool same = act && lv == ll;
    const u64 part = wave_sum(same ? kv : 0ull);
    if ((int)(threadIdx.x & 63) == lead && part) mod_table_add(M, K, ll, part);
    if (act && !same && kv) mod_table_add(M, K, lv, kv);
}

__device__ __forceinline__ void mod_finish(const ModArgs &a, ModTable &M, u64 tw, u64 sin) {
    __syncthreads();
    for (uint32_t s = threadIdx.x; s < kModSlots; s += 256)
        if (M.key[s] != kEmpty32 && M.val[s]) atomicAdd(&a.K[M.key[s]], M.val[s]);
    u64 z = 0;
    uint32_t zo = 0;
    block_reduce(M.R, z, tw, sin, zo);
    if (threadIdx.x == 0) {
        if (tw) atomicAdd(&a.sums[0], tw);
        if (sin) atomicAdd(&a.sums[1], sin);
    }
}

// Weighted degree and same-label weight of arcs k0 + j*STRIDE (j < A, < e).
// Every lane issues every load (arcs past the row read arc k0 and are
// masked), so the label gathers are in flight together: loads behind
// per-lane branches are waited for one at a time.  k0 < e for lane 0.
template <int A, int STRIDE>
__device__ __forceinline__ void mod_arcs(const ModArgs &a, uint64_t k0, uint64_t e, uint32_t lv, u64 &kv,
                                         u64 &sin) {
    uint32_t u[A], wv[A];
    uint32_t valid = 0;
    const uint64_t k_first = k0 - (threadIdx.x & 63) * (STRIDE == 1 ? 0 : 1);  // an arc of the row
#pragma unroll
    for (int j = 0; j < A; ++j) {
        const uint64_t k = k0 + (uint64_t)j * STRIDE;
        const bool in = k < e;
        valid |= (uint32_t)in << j;
        const uint32_t x = a.g.col[in ? k : k_first];
        u[j] = in ? x : 0u;
    }
    if (a.g.w) {
#pragma unroll
        for (int j = 0; j < A; ++j) {
            const uint64_t k = k0 + (uint64_t)j * STRIDE;
            const uint32_t x = a.g.w[(valid >> j & 1u) ? k : k_first];
            wv[j] = (valid >> j & 1u) ? x : 0u;
        }
    } else {
#pragma unroll
        for (int j = 0; j < A; ++j) wv[j] = valid >> j & 1u;
    }
    bool bad = false;
#pragma unroll
    for (int j = 0; j < A; ++j) {
        bad |= u[j] >= a.g.n;
        u[j] = u[j] >= a.g.n ? 0u : u[j];
    }
    if (bad) atomicOr(a.err, ERR_COL);
    uint32_t lab[A];
#pragma unroll
    for (int j = 0; j < A; ++j) lab[j] = a.labels[u[j]];
#pragma unroll
    for (int j = 0; j < A; ++j) {
        kv += wv[j];
        if ((valid >> j & 1u) && lab[j] == lv) sin += wv[j];
    }
}

// Incremental form: weighted degree of arcs k0 + j*STRIDE (j < A, < e) and,
// for a changed row (lv = its label now, pv = before), the change of its
// arcs' Sigma_in terms, added to d modulo 2^64.
template <int A, int STRIDE>
__device__ __forceinline__ void mod_delta_arcs(const ModArgs &a, uint64_t k0, uint64_t e, bool changed, uint32_t lv,
                                               uint32_t pv, u64 &kv, u64 &d) {
    uint32_t u[A], wv[A];
    uint32_t valid = 0;
    const uint64_t k_first = k0 - (threadIdx.x & 63) * (STRIDE == 1 ? 0 : 1);  // an arc of the row
#pragma unroll
    for (int j = 0; j < A; ++j) {
        const uint64_t k = k0 + (uint64_t)j * STRIDE;
        valid |= (uint32_t)(k < e) << j;
    }
    if (a.g.w) {
#pragma unroll
        for (int j = 0; j < A; ++j) {
            const uint64_t k = k0 + (uint64_t)j * STRIDE;
            const uint32_t x = a.g.w[(valid >> j & 1u) ? k : k_first];
            wv[j] = (valid >> j & 1u) ? x : 0u;
        }
    } else {
#pragma unroll
        for (int j = 0; j < A; ++j) wv[j] = valid >> j & 1u;
    }
#pragma unroll
    for (int j = 0; j < A; ++j) kv += wv[j];
    if (!changed) return;
#pragma unroll
    for (int j = 0; j < A; ++j) {
        const uint64_t k = k0 + (uint64_t)j * STRIDE;
        const uint32_t x = a.g.col[(valid >> j & 1u) ? k : k_first];
        u[j] = (valid >> j & 1u) && x < a.g.n ? x : 0u;
    }
    uint32_t ln[A], lp[A];
#pragma unroll
    for (int j = 0; j < A; ++j) {
        ln[j] = a.labels[u[j]];
        lp[j] = a.labels_prev[u[j]];
    }
#pragma unroll
    for (int j = 0; j < A; ++j) {
        const bool now = ln[j] == lv, before = lp[j] == pv;
        if ((valid >> j & 1u) && now != before) {
            const u64 t = (u64)wv[j] * (ln[j] != lp[j] ? 1u : 2u);
            d += now ? t : (u64)0 - t;
        }
    }
}

// Incremental form, one lane per row (rows of at most 32 arcs).
__global__ __launch_bounds__(256) void mod_delta_thread_k(ModArgs a, uint32_t lo, uint32_t cnt) {
    __shared__ ModTable M;
    mod_table_init(M);
    u64 tw = 0, d = 0;
    for (uint32_t base = blockIdx.x * 256 + (threadIdx.x & ~63u); base < cnt; base += gridDim.x * 256) {
        const uint32_t i = base + (threadIdx.x & 63);
        const bool act = i < cnt;
        u64 kv = 0;
        uint32_t lv = 0;
        if (act) {
            const uint32_t v = lo + i;
            lv = a.labels[v];
            const uint32_t pv = a.labels_prev[v];
            const uint64_t b = a.g.rp[v], e = a.g.rp[v + 1];
            if (lv == pv && !a.g.w)
                kv = e - b;  // unit weights, label kept: no arc to read
            else
                for (uint64_t k = b; k < e; k += 8) mod_delta_arcs<8, 1>(a, k, e, lv != pv, lv, pv, kv, d);
        }
        tw += kv;
        add_community(M, a.K, act, lv, kv);
    }
    mod_finish(a, M, tw, d);
}

// Incremental form, rows of at most 512 arcs, 64 rows per wavefront step:
// a row whose label stayed (unit weights) only adds its degree, one lane
// each; the other rows' arcs are read by the whole wavefront, one row after
// another.
__global__ __launch_bounds__(256) void mod_delta_wave_k(ModArgs a, uint32_t lo, uint32_t cnt) {
    __shared__ ModTable M;
    mod_table_init(M);
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    u64 tw = 0, d = 0;
    for (uint32_t base = (blockIdx.x * 4 + wave) * 64; base < cnt; base += gridDim.x * 4 * 64) {
        const uint32_t i = base + lane;
        const bool act = i < cnt;
        const uint32_t v = lo + (act ? i : 0u);  // row lo exists: cnt > 0
        const uint32_t lv = a.labels[v], pv = a.labels_prev[v];
        const uint64_t b = a.g.rp[v], e = a.g.rp[v + 1];
        const bool quick = act && lv == pv && !a.g.w;
        const u64 kq = quick ? (u64)(e - b) : 0ull;
        tw += kq;
        add_community(M, a.K, quick, lv, kq);
        u64 slow = __ballot(act && !quick);
        while (slow) {
            const int j = __ffsll((long long)slow) - 1;
            slow &= slow - 1;
            const uint32_t lj = (uint32_t)__shfl((int)lv, j, 64), pj = (uint32_t)__shfl((int)pv, j, 64);
            const uint64_t bj = __shfl(b, j, 64), ej = __shfl(e, j, 64);
            u64 kv = 0;
            mod_delta_arcs<kWaveArcs / 64, 64>(a, bj + lane, ej, lj != pj, lj, pj, kv, d);
            kv = wave_sum(kv);
            tw += lane == 0 ? kv : 0;
            add_community(M, a.K, lane == 0, lj, kv);
        }
    }
    mod_finish(a, M, tw, d);
}

// Incremental form, segments of long rows, 64 segments per wavefront step
// as above.
__global__ __launch_bounds__(256) void mod_delta_hub_k(ModArgs a, const HubItem *__restrict__ items,
                                                       uint32_t count) {
    __shared__ ModTable M;
    mod_table_init(M);
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    u64 tw = 0, d = 0;
    for (uint32_t base = (blockIdx.x * 4 + wave) * 64; base < count; base += gridDim.x * 4 * 64) {
        const uint32_t it = base + lane;
        const bool act = it < count;
        const HubItem item = items[act ? it : 0u];  // item 0 exists: count > 0
        const uint32_t lv = a.labels[item.r], pv = a.labels_prev[item.r];
        const bool quick = act && lv == pv && !a.g.w;
        const u64 kq = quick ? (u64)(item.b1 - item.b0) : 0ull;
        tw += kq;
        add_community(M, a.K, quick, lv, kq);
        u64 slow = __ballot(act && !quick);
        while (slow) {
            const int j = __ffsll((long long)slow) - 1;
            slow &= slow - 1;
            const uint32_t lj = (uint32_t)__shfl((int)lv, j, 64), pj = (uint32_t)__shfl((int)pv, j, 64);
            const uint64_t bj = __shfl(item.b0, j, 64), ej = __shfl(item.b1, j, 64);
            u64 kv = 0;
            mod_delta_arcs<kWaveArcs / 64, 64>(a, bj + lane, ej, lj != pj, lj, pj, kv, d);
            kv = wave_sum(kv);
            tw += lane == 0 ? kv : 0;
            add_community(M, a.K, lane == 0, lj, kv);
        }
    }
    mod_finish(a, M, tw, d);
}

// One lane per row (rows of at most 32 arcs).
__global__ __launch_bounds__(256) void mod_thread_k(ModArgs a, uint32_t lo, uint32_t cnt) {
    __shared__ ModTable M;
    mod_table_init(M);
    u64 tw = 0, sin = 0;
    for (uint32_t base = blockIdx.x * 256 + (threadIdx.x & ~63u); base < cnt; base += gridDim.x * 256) {
        const uint32_t i = base + (threadIdx.x & 63);
        const bool act = i < cnt;
        u64 kv = 0;
        uint32_t lv = 0;
        if (act) {
            const uint32_t v = lo + i;
            lv = a.labels[v];
            const uint64_t e = a.g.rp[v + 1];
            for (uint64_t k = a.g.rp[v]; k < e; k += 8) mod_arcs<8, 1>(a, k, e, lv, kv, sin);
        }
        tw += kv;
        add_community(M, a.K, act, lv, kv);
    }
    mod_finish(a, M, tw, sin);
}

// One wavefront per row (rows of at most 512 arcs).
__global__ __launch_bounds__(256) void mod_wave_k(ModArgs a, uint32_t lo, uint32_t cnt) {
    __shared__ ModTable M;
    mod_table_init(M);
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    u64 tw = 0, sin = 0;
    for (uint32_t i = blockIdx.x * 4 + wave; i < cnt; i += gridDim.x * 4) {
        const uint32_t v = lo + i;
        const uint32_t lv = a.labels[v];
        u64 kv = 0;
        mod_arcs<kWaveArcs / 64, 64>(a, a.g.rp[v] + lane, a.g.rp[v + 1], lv, kv, sin);
        kv = wave_sum(kv);
        tw += lane == 0 ? kv : 0;
        add_community(M, a.K, lane == 0, lv, kv);
    }
    mod_finish(a, M, tw, sin);
}

// One wavefront per segment of a long row.
__global__ __launch_bounds__(256) void mod_hub_k(ModArgs a, const HubItem *__restrict__ items, uint32_t count) {
    __shared__ ModTable M;
    mod_table_init(M);
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    u64 tw = 0, sin = 0;
    for (uint32_t it = blockIdx.x * 4 + wave; it < count; it += gridDim.x * 4) {
        const HubItem item = items[it];
        const uint32_t lv = a.labels[item.r];
        u64 kv = 0;
        mod_arcs<kWaveArcs / 64, 64>(a, item.b0 + lane, item.b1, lv, kv, sin);
        kv = wave_sum(kv);
        tw += lane == 0 ? kv : 0;
        add_community(M, a.K, lane == 0, lv, kv);
    }
    mod_finish(a, M, tw, sin);
}

// Any row length, on a CSR as the caller stores it (no binning): each
// wavefront takes 64 rows; rows of at most 32 arcs are summed one lane
// each, longer rows by the whole wavefront in 512-arc steps, one row after
// another, up to their first kHeadArcs arcs (mod_tail_k sums the rest, so
// no wavefront walks a hub alone).  The row bounds and labels are checked here (a bad row is
// skipped and flagged, a bad label counts as label 0 and is flagged), so no
// access leaves the arrays whatever the input.
__global__ __launch_bounds__(256) void mod_any_k(ModArgs a) {
    __shared__ ModTable M;
    mod_table_init(M);
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t n = a.g.n;
    if (blockIdx.x == 0 && threadIdx.x == 0 && (a.g.rp[0] != 0 || a.g.rp[n] != a.g.m)) atomicOr(a.err, ERR_ROWPTR);
    u64 tw = 0, sin = 0;
    for (uint32_t base = (blockIdx.x * 4 + wave) * 64; base < n; base += gridDim.x * 4 * 64) {
        const uint32_t i = base + lane;
        const bool act = i < n;
        const uint32_t v = act ? i : 0u;
        const uint64_t b = a.g.rp[v], e = a.g.rp[v + 1];
        uint32_t lv = a.labels[v];
        const bool badrow = act && (b > e || e > a.g.m);
        const bool badlab = act && lv >= n;
        if (badrow) atomicOr(a.err, ERR_ROWPTR);
        if (badlab) atomicOr(a.err, ERR_LABEL);
        lv = badlab ? 0u : lv;
        const bool ok = act && !badrow;
        const bool one = ok && e - b <= 32;
        u64 kv = 0;
        if (one)
            for (uint64_t k = b; k < e; k += 8) mod_arcs<8, 1>(a, k, e, lv, kv, sin);
        tw += kv;
        add_community(M, a.K, one, lv, kv);
        u64 longm = __ballot(ok && !one);
        while (longm) {
            const int j = __ffsll((long long)longm) - 1;
            longm &= longm - 1;
            const uint32_t lj = (uint32_t)__shfl((int)lv, j, 64);
            const uint64_t bj = __shfl(b, j, 64), ej = __shfl(e, j, 64);
            // the first kHeadArcs arcs here, the rest in mod_tail_k
            const uint64_t eh = ej - bj > kHeadArcs ? bj + kHeadArcs : ej;
            u64 kw = 0;
            for (uint64_t k0 = bj; k0 < eh; k0 += kWaveArcs)
                mod_arcs<kWaveArcs / 64, 64>(a, k0 + lane, eh, lj, kw, sin);
            kw = wave_sum(kw);
            tw += lane == 0 ? kw : 0;
            add_community(M, a.K, lane == 0, lj, kw);
        }
    }
    mod_finish(a, M, tw, sin);
}

// The arcs of rows beyond their first kHeadArcs (mod_any_k took those), in
// chunks of kHeadArcs arcs: a chunk meets the tail of at most one row (a
// row that starts inside the chunk has its tail beyond it), found by a
// binary search over row_ptr.  K of the row's label, 2m and Sigma_in take
// the chunk's part with one device atomic each.
__global__ __launch_bounds__(256) void mod_tail_k(ModArgs a) {
    __shared__ BlockRed R;
    __shared__ uint32_t srow;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = threadIdx.x >> 6;
    const u64 m = a.g.m;
    const u64 nchunks = (m + kHeadArcs - 1) / kHeadArcs;
    u64 tw = 0, sin = 0;
    for (u64 c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const u64 c0 = c * kHeadArcs, c1 = c0 + kHeadArcs < m ? c0 + kHeadArcs : m;
        __syncthreads();  // every wave has read the previous chunk's srow
        if (threadIdx.x == 0) srow = row_of_arc(a.g, c0);
        __syncthreads();
        const uint32_t r = srow;
        const uint64_t b = a.g.rp[r], e = a.g.rp[r + 1] < m ? a.g.rp[r + 1] : m;
        const uint64_t t0 = c0 > b + kHeadArcs ? c0 : b + kHeadArcs, t1 = c1 < e ? c1 : e;
        if (t0 >= t1) continue;  // uniform: the chunk meets no tail
        uint32_t lv = a.labels[r];
        lv = lv >= a.g.n ? 0u : lv;  // flagged by mod_any_k
        u64 kv = 0;
        for (uint64_t k0 = t0 + wave * kWaveArcs; k0 < t1; k0 += 4 * kWaveArcs)
            mod_arcs<kWaveArcs / 64, 64>(a, k0 + lane, t1, lv, kv, sin);
        u64 z = 0, z2 = 0;
        uint32_t zo = 0;
        block_reduce(R, z, kv, z2, zo);
        if (threadIdx.x == 0 && kv) {
            atomicAdd(&a.K[lv], kv);
            tw += kv;
        }
    }
    sin = wave_sum(sin);
    if (lane == 0) {
        if (sin) atomicAdd(&a.sums[1], sin);
        if (wave == 0 && tw) atomicAdd(&a.sums[0], tw);
    }
}

// One block: the u128 sum of the partials of mod_sumsq_k, with the two sums
// and the error word, into out[0..4] = {sum K^2 low, high, 2m, Sigma_in,
// error bits}.
__global__ __launch_bounds__(256) void mod_final_k(const u64 *__restrict__ partials, uint32_t nparts,
                                                   const u64 *__restrict__ sums, const uint32_t *__restrict__ err,
                                                   u64 *out) {
    __shared__ unsigned __int128 sh[256];
    unsigned __int128 acc = 0;
    for (uint32_t i = threadIdx.x; i < nparts; i += 256)
        acc += ((unsigned __int128)partials[2 * i + 1] << 64) | (unsigned __int128)partials[2 * i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (uint32_t off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = (u64)sh[0];
        out[1] = (u64)(sh[0] >> 64);
        out[2] = sums[0];
        out[3] = sums[1];
        out[4] = *err;
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

hipError_t launch_mod_rows(const ModArgs &a, uint32_t lo, uint32_t cnt, int per_wave, hipStream_t s) {
    if (cnt == 0) return hipSuccess;
    if (a.labels_prev) {
        if (per_wave)
            mod_delta_wave_k<<<grid_for(cnt, 256, kModGrid), 256, 0, s>>>(a, lo, cnt);
        else
            mod_delta_thread_k<<<grid_for(cnt, 256, kModGrid), 256, 0, s>>>(a, lo, cnt);
    } else if (per_wave) {
        mod_wave_k<<<grid_for(cnt, 4, kModGrid), 256, 0, s>>>(a, lo, cnt);
    } else {
        mod_thread_k<<<grid_for(cnt, 256, kModGrid), 256, 0, s>>>(a, lo, cnt);
    }
    return hipGetLastError();
}
hipError_t launch_mod_hub(const ModArgs &a, const HubItem *items, uint32_t count, hipStream_t s) {
    if (count == 0) return hipSuccess;
    if (a.labels_prev)
        mod_delta_hub_k<<<grid_for(count, 256, kModGrid), 256, 0, s>>>(a, items, count);
    else
        mod_hub_k<<<grid_for(count, 4, kModGrid), 256, 0, s>>>(a, items, count);
    return hipGetLastError();
}
hipError_t launch_mod_any(const ModArgs &a, hipStream_t s) {
    if (a.g.n == 0) return hipSuccess;
    mod_any_k<<<grid_for(a.g.n, 256, kModGrid), 256, 0, s>>>(a);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && a.g.m > kHeadArcs) {
        mod_tail_k<<<grid_for(a.g.m, kHeadArcs, kModGrid), 256, 0, s>>>(a);
        e = hipGetLastError();
    }
    return e;
}
hipError_t launch_mod_final(const u64 *partials, uint32_t nparts, const u64 *sums, const uint32_t *err, u64 *out,
                            hipStream_t s) {
    mod_final_k<<<1, 256, 0, s>>>(partials, nparts, sums, err, out);
    return hipGetLastError();
}
hipError_t launch_modularity_any(const Graph &g, const uint32_t *labels, u64 *K, u64 *sums, uint32_t *err,
                                 u64 *partials, uint32_t nparts, u64 *out, hipStream_t s) {
    hipError_t e = launch_fill_u64(K, 0, g.n, s);
    if (e == hipSuccess) e = launch_fill_u64(sums, 0, 3, s);  // the two totals and the error word
    ModArgs ma;
    ma.g = g;
    ma.labels = labels;
    ma.K = K;
    ma.sums = sums;
    ma.err = err;
    ma.labels_prev = nullptr;
    if (e == hipSuccess) e = launch_mod_any(ma, s);
    if (e == hipSuccess) e = launch_mod_sumsq(K, g.n, partials, nparts, s);
    if (e == hipSuccess) e = launch_mod_final(partials, nparts, sums, err, out, s);
    return e;
}
hipError_t launch_mod_sumsq(const u64 *K, uint32_t n, u64 *partials, uint32_t nparts, hipStream_t s) {
    mod_sumsq_k<<<nparts, 256, 0, s>>>(K, n, partials);
    return hipGetLastError();
}

}  // namespace lpa
