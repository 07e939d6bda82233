// lpa_copra.hip -- COPRA (arXiv 2301.09125, Section 3.3): label propagation
// where every vertex holds up to max_labels (label, belonging coefficient)
// pairs.  Each round a vertex collects its neighbours' pairs, each scaled by
// the connecting edge weight, keeps the labels whose share of the collected
// weight reaches 1/max_labels (or, if none does, its best label alone) and
// normalises what it kept.  The run stops as RAK does, on the vertices whose
// best label changed.
//
// Exact arithmetic: coefficients are integers in units of 2^-16 (65536 =
// belonging 1).  The tally of label c at v is sum over arcs (v,u,w) of
// w * b_u(c), below 2^48 because weighted degrees stay below 2^32; the
// collected total is weighted_degree(v) * 2^16.  Label c is kept iff its
// tally is positive and tally * max_labels >= total.  New coefficients are
// floor(tally * 2^16 / kept_sum), and what the floors leave out of 2^16 goes
// to the best label (largest tally; ties to the lowest label, or to the
// highest lowbias32(label ^ k) with the hashed rule).  A vertex that
// collects nothing (no arcs) is its own community.  Kept labels are stored
// in increasing label order.
//
// State: one record per vertex (count, best label, then up to V (label,
// coefficient) pairs; a power-of-two number of words up to 128 bytes, so a
// neighbour's state is one line), double-buffered.  The rounds read the
// caller's CSR directly (original ids, no relabelled copy):
//   copra_group_k  rows with deg * V <= 32: 16 lanes per row, a 64-slot
//                  LDS table;
//   copra_wave_k   rows with deg * V <= 512: one wavefront per row, an LDS
//                  table of next_pow2(2 * deg * V) slots (<= 256 for the
//                  rows of deg * V <= 128, which run with a quarter of the
//                  LDS and so four times the blocks per CU; <= 1024);
//   copra_block_k  the other rows: one block per row, an LDS table of
//                  2048 or 4096 slots; a row whose distinct labels would fill more than
//                  3/4 of it is listed for
//   copra_gpiece_k, copra_gscan_k, copra_gdone_k  the listed rows, with a
//                  table in device memory of next_pow2(2 * min(deg * V, n))
//                  slots (at least twice the row's distinct labels) each:
//                  pieces of the row pre-sum their entries in LDS and add
//                  them to it, slices of the table are scanned in parallel
//                  for the decision, one wavefront per row writes the state.
// Rows without arcs are in no list: they stay alone, and both buffers hold
// that state from the start.  Semi-synchronous rounds: two half-rounds, a
// vertex votes in the half its SplitMix64 draw for the round names and
// copies its state in the other.

#include "lpa_copra.h"
#include "lpa_rows.h"

namespace lpa {

constexpr uint32_t kOne = 65536u;
constexpr uint32_t kCopraWaveSlots = 1024;      // rows of deg * V <= 512
constexpr uint32_t kCopraWaveSlotsSmall = 256;  // rows of deg * V <= 128 (a quarter of the LDS)
constexpr uint32_t kCopraBlockSlots = 4096;
constexpr uint32_t kEmptyKey = 0xFFFFFFFFu;
constexpr uint32_t kSliceSlots = kCopraSliceSlots;

__device__ __forceinline__ bool copra_votes(const CopraArgs &a, uint32_t v) {
    if (!a.half) return true;
    const u64 c = (((u64)a.t << 32) | v) << 1;
    return (uint32_t)(splitmix64_at(a.seed, c) >> 63) == a.half - 1;
}

__device__ __forceinline__ Tie copra_tie(const CopraArgs &a, uint32_t v) {
    Tie t{a.tie, 0u};
    if (a.tie) t.k = (uint32_t)splitmix64_at(a.seed, ((((u64)a.t << 32) | v) << 1) | 1u);
    return t;
}

// Insert (lab, x) into a table of mask+1 slots (LDS or device memory) with
// linear probing, giving up after mask+1 probes: 1 = claimed a new slot,
// 0 = added to the label's slot, -1 = no free slot (nothing added).
__device__ __forceinline__ int copra_insert_bounded(uint32_t *key, u64 *tal, uint32_t mask, uint32_t lab, u64 x) {
    uint32_t h = hmix(lab) & mask;
    for (uint32_t p = 0; p <= mask; ++p) {
        const uint32_t prev = atomicCAS(&key[h], kEmptyKey, lab);
        if (prev == kEmptyKey || prev == lab) {
            atomicAdd(&tal[h], x);
            return prev == kEmptyKey ? 1 : 0;
        }
        h = (h + 1) & mask;
    }
    return -1;
}

// Copy vertex v's state unchanged (the other half of a semi-synchronous round).
__device__ __forceinline__ void copra_copy(const CopraArgs &a, uint32_t v, uint32_t lane, uint32_t lanes) {
    for (uint32_t i = lane; i < a.V; i += lanes) {
        a.out[(u64)v * a.stride + 2 + 2 * i] = a.in[(u64)v * a.stride + 2 + 2 * i];
        a.out[(u64)v * a.stride + 3 + 2 * i] = a.in[(u64)v * a.stride + 3 + 2 * i];
    }
    if (lane == 0) {
        a.out[(u64)v * a.stride] = a.in[(u64)v * a.stride];
        a.out[(u64)v * a.stride + 1] = a.in[(u64)v * a.stride + 1];
    }
}

// A vertex with nothing to collect: its own community.
__device__ __forceinline__ void copra_alone(const CopraArgs &a, uint32_t v, uint32_t lab) {
    a.out[(u64)v * a.stride + 2] = lab;
    a.out[(u64)v * a.stride + 3] = kOne;
    a.out[(u64)v * a.stride] = 1;
    a.out[(u64)v * a.stride + 1] = lab;
}

// Write the kept labels klab[0..kn) (coefficients before the remainder in
// kcoef) in increasing label order, the remainder to `best`.  Lanes 0..63 of
// one wavefront call this; kn <= V <= 64.
__device__ __forceinline__ void copra_store(const CopraArgs &a, uint32_t v, uint32_t lane, const uint32_t *klab,
                                            const uint32_t *kcoef, uint32_t kn, uint32_t best) {
    const bool mine = lane < kn;
    const uint32_t l = mine ? klab[lane] : 0u;
    uint32_t c = mine ? kcoef[lane] : 0u;
    const uint32_t given = wave_sum(c);
    uint32_t rank = 0;
    for (uint32_t j = 0; j < kn; ++j) rank += klab[j] < l;
    if (mine && l == best) c += kOne - given;
    if (mine) {
        a.out[(u64)v * a.stride + 2 + 2 * rank] = l;
        a.out[(u64)v * a.stride + 3 + 2 * rank] = c;
    }
    if (lane == 0) {
        a.out[(u64)v * a.stride] = kn;
        a.out[(u64)v * a.stride + 1] = best;
    }
}

// 16 lanes per row, four rows per wavefront, rows with deg * V <= 32 (listed
// in `rows`): a 64-slot LDS table per row, reductions over each 16-lane row
// of the wavefront.
constexpr uint32_t kCopraGroupSlots = 64;
__global__ __launch_bounds__(256) void copra_group_k(CopraArgs a, const uint32_t *__restrict__ rows, uint32_t count) {
    __shared__ uint32_t skey[16][kCopraGroupSlots];
    __shared__ u64 stal[16][kCopraGroupSlots];
    __shared__ uint32_t sklab[16][32], skcoef[16][32], skn[16];
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t gl = lane & 15;
    const uint32_t grp = threadIdx.x >> 4;  // 0..15 in the block
    uint32_t *key = skey[grp];
    u64 *tal = stal[grp];
    const uint32_t V = a.V;
    u64 chg = 0;
    // every lane of a wavefront runs the same number of steps (the bound is
    // per wavefront), so the wavefront-wide LDS syncs line up
    for (uint32_t base = (blockIdx.x * 4 + (threadIdx.x >> 6)) * 4; base < count; base += gridDim.x * 16) {
        const uint32_t idx = base + (lane >> 4);
        const bool act = idx < count;
        const uint32_t v = act ? rows[idx] : 0u;
        const bool on = act && copra_votes(a, v);
        if (act && !on) copra_copy(a, v, gl, 16);
        const uint64_t b = on ? a.g.rp[v] : 0, e = on ? a.g.rp[v + 1] : 0;
        const Tie tie = copra_tie(a, v);
        for (uint32_t s = gl; s < kCopraGroupSlots; s += 16) {
            key[s] = kEmptyKey;
            tal[s] = 0;
        }
        if (gl == 0) skn[grp] = 0;
        wave_sync();
        u64 tw = 0;
        for (uint32_t j = 0; j < 2; ++j) {  // deg <= 32
            const uint64_t k = b + gl + 16 * j;
            const bool in = k < e;
            const uint32_t u = in ? a.g.col[k] : 0u;
            const uint32_t we = in ? (a.g.w ? a.g.w[k] : 1u) : 0u;
            const uint32_t c = in ? a.in[(u64)u * a.stride] : 0u;
            tw += we;
            for (uint32_t i = 0; i < c; ++i)
                if (copra_insert_bounded(key, tal, kCopraGroupSlots - 1, a.in[(u64)u * a.stride + 2 + 2 * i],
                                         (u64)we * a.in[(u64)u * a.stride + 3 + 2 * i]) < 0)
                    atomicOr(a.err, ERR_TABLE);  // cannot happen: at most 32 entries
        }
        wave_sync();
        const u64 total = row_sum64(tw) * kOne;
        u64 m1 = 0;
        for (uint32_t s = gl; s < kCopraGroupSlots; s += 16)
            if (key[s] != kEmptyKey) m1 = umax64(m1, tal[s] + 1);
        m1 = row_max64(m1);
        u64 bc = 0, ksum = 0, kcnt = 0;
        for (uint32_t s = gl; s < kCopraGroupSlots; s += 16) {
            const uint32_t l = key[s];
            if (l == kEmptyKey) continue;
            const u64 t = tal[s];
            if (t + 1 == m1) bc = umax64(bc, tie_code(tie, l));
            if (t > 0 && t * V >= total) {
                ksum += t;
                ++kcnt;
            }
        }
        bc = row_max64(bc);
        ksum = row_sum64(ksum);
        kcnt = row_sum64(kcnt);
        const uint32_t best = tie_label(tie, (uint32_t)bc);
        for (uint32_t s = gl; s < kCopraGroupSlots; s += 16) {
            const uint32_t l = key[s];
            if (l == kEmptyKey) continue;
            const u64 t = tal[s];
            if (on && t > 0 && t * V >= total) {
                const uint32_t j = atomicAdd(&skn[grp], 1u);
                sklab[grp][j] = l;
                skcoef[grp][j] = (uint32_t)(t * kOne / ksum);
            }
        }
        wave_sync();
        // kept labels (at most 32) in increasing order, the remainder to best
        const uint32_t kn = (uint32_t)kcnt;
        uint32_t given = 0;
        for (uint32_t j = gl; j < kn; j += 16) given += skcoef[grp][j];
        given = row_sum32(given);
        if (on && kn == 0 && gl == 0) copra_alone(a, v, best);
        if (on && kn > 0) {
            for (uint32_t j = gl; j < kn; j += 16) {
                const uint32_t l = sklab[grp][j];
                uint32_t c = skcoef[grp][j];
                uint32_t rank = 0;
                for (uint32_t q = 0; q < kn; ++q) rank += sklab[grp][q] < l;
                if (l == best) c += kOne - given;
                a.out[(u64)v * a.stride + 2 + 2 * rank] = l;
                a.out[(u64)v * a.stride + 3 + 2 * rank] = c;
            }
            if (gl == 0) {
                a.out[(u64)v * a.stride] = kn;
                a.out[(u64)v * a.stride + 1] = best;
            }
        }
        if (on && gl == 0) chg += a.in[(u64)v * a.stride + 1] != best;
        wave_sync();  // the tables are cleared for the next rows
    }
    block_count(chg, a.changed);
}

// One wavefront per row, rows with 32 < deg * V <= SLOTS / 2 (listed in
// `rows`), tables of up to SLOTS slots.
template <uint32_t SLOTS>
__global__ __launch_bounds__(256) void copra_wave_k(CopraArgs a, const uint32_t *__restrict__ rows, uint32_t count) {
    __shared__ uint32_t skey[4][SLOTS];
    __shared__ u64 stal[4][SLOTS];
    __shared__ uint32_t sklab[4][64], skcoef[4][64], skn[4];
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    uint32_t *key = skey[wave];
    u64 *tal = stal[wave];
    const uint32_t V = a.V;
    u64 chg = 0;
    for (uint32_t it = blockIdx.x * 4 + wave; it < count; it += gridDim.x * 4) {
        const uint32_t v = rows[it];
        const uint64_t b = a.g.rp[v], e = a.g.rp[v + 1];
        const uint64_t deg = e - b;
        if (!copra_votes(a, v)) {
            copra_copy(a, v, lane, 64);
            continue;
        }
        const uint32_t old_best = a.in[(u64)v * a.stride + 1];
        const Tie tie = copra_tie(a, v);
        const uint32_t S = next_pow2((uint32_t)(2 * deg * V));
        for (uint32_t s = lane; s < S; s += 64) {
            key[s] = kEmptyKey;
            tal[s] = 0;
        }
        if (lane == 0) skn[wave] = 0;
        wave_sync();
        u64 tw = 0;
        for (uint64_t k0 = b; k0 < e; k0 += 64) {
            const uint64_t k = k0 + lane;
            const bool in = k < e;
            const uint32_t u = in ? a.g.col[k] : 0u;
            const uint32_t we = in ? (a.g.w ? a.g.w[k] : 1u) : 0u;
            const uint32_t c = in ? a.in[(u64)u * a.stride] : 0u;
            tw += we;
            for (uint32_t i = 0; i < c; ++i)
                if (copra_insert_bounded(key, tal, S - 1, a.in[(u64)u * a.stride + 2 + 2 * i],
                                         (u64)we * a.in[(u64)u * a.stride + 3 + 2 * i]) < 0)
                    atomicOr(a.err, ERR_TABLE);  // cannot happen: distinct labels <= deg * V <= S / 2
        }
        wave_sync();
        const u64 total = wave_sum(tw) * kOne;
        u64 m1 = 0;  // largest tally + 1 over the occupied slots
        for (uint32_t s = lane; s < S; s += 64)
            if (key[s] != kEmptyKey) m1 = umax64(m1, tal[s] + 1);
        m1 = wave_max64(m1);
        u64 bc = 0;  // largest tie code among the heaviest labels
        u64 ksum = 0, kcnt = 0;
        for (uint32_t s = lane; s < S; s += 64) {
            const uint32_t l = key[s];
            if (l == kEmptyKey) continue;
            const u64 t = tal[s];
            if (t + 1 == m1) bc = umax64(bc, tie_code(tie, l));
            if (t > 0 && t * V >= total) {
                ksum += t;
                ++kcnt;
            }
        }
        bc = wave_max64(bc);
        ksum = wave_sum(ksum);
        kcnt = wave_sum(kcnt);
        const uint32_t best = tie_label(tie, (uint32_t)bc);
        if (kcnt == 0) {
            if (lane == 0) copra_alone(a, v, best);
        } else {
            for (uint32_t s = lane; s < S; s += 64) {
                const uint32_t l = key[s];
                if (l == kEmptyKey) continue;
                const u64 t = tal[s];
                if (t > 0 && t * V >= total) {
                    const uint32_t j = atomicAdd(&skn[wave], 1u);
                    sklab[wave][j] = l;
                    skcoef[wave][j] = (uint32_t)(t * kOne / ksum);
                }
            }
            wave_sync();
            copra_store(a, v, lane, sklab[wave], skcoef[wave], (uint32_t)kcnt, best);
        }
        if (lane == 0) chg += old_best != best;
        wave_sync();  // the table is cleared for the next row
    }
    block_count(chg, a.changed);
}

// The vote of row v from its filled LDS table of S slots, by a 256-thread
// block; reductions and kept lists in LDS.
__device__ __forceinline__ uint32_t copra_finish_block(const CopraArgs &a, uint32_t v, Tie tie, const uint32_t *key,
                                                       const u64 *tal, uint32_t S, u64 total, BlockRed *red,
                                                       uint32_t *klab, uint32_t *kcoef, uint32_t *kn) {
    const uint32_t V = a.V;
    u64 m1 = 0, z1 = 0, z2 = 0;
    uint32_t zo = 0;
    for (uint32_t s = threadIdx.x; s < S; s += 256)
        if (key[s] != kEmptyKey) m1 = umax64(m1, tal[s] + 1);
    block_reduce(red[0], m1, z1, z2, zo);
    u64 bc = 0, ksum = 0, kcnt = 0;
    for (uint32_t s = threadIdx.x; s < S; s += 256) {
        const uint32_t l = key[s];
        if (l == kEmptyKey) continue;
        const u64 t = tal[s];
        if (t + 1 == m1) bc = umax64(bc, tie_code(tie, l));
        if (t > 0 && t * V >= total) {
            ksum += t;
            ++kcnt;
        }
    }
    zo = 0;
    block_reduce(red[1], bc, ksum, kcnt, zo);
    const uint32_t best = tie_label(tie, (uint32_t)bc);
    if (kcnt == 0) {
        if (threadIdx.x == 0) copra_alone(a, v, best);
        return best;
    }
    for (uint32_t s = threadIdx.x; s < S; s += 256) {
        const uint32_t l = key[s];
        if (l == kEmptyKey) continue;
        const u64 t = tal[s];
        if (t > 0 && t * V >= total) {
            const uint32_t j = atomicAdd(kn, 1u);
            klab[j] = l;
            kcoef[j] = (uint32_t)(t * kOne / ksum);
        }
    }
    __syncthreads();
    if (threadIdx.x < 64) copra_store(a, v, threadIdx.x, klab, kcoef, (uint32_t)kcnt, best);
    return best;
}

// The first vote of row v while every vertex is still alone with belonging
// 1 and v lists each neighbour once: tally(u) = w(v,u) * 2^16.  A
// 256-thread block; kn zeroed by the caller.
__device__ __forceinline__ uint32_t copra_first_block(const CopraArgs &a, uint32_t v, Tie tie, BlockRed *red,
                                                      uint32_t *klab, uint32_t *kcoef, uint32_t *kn) {
    const uint32_t V = a.V;
    const uint64_t b = a.g.rp[v], e = a.g.rp[v + 1];
    u64 bk = 0, tw = 0, z = 0;
    uint32_t zo = 0;
    for (uint64_t k = b + threadIdx.x; k < e; k += 256) {
        const uint32_t we = a.g.w ? a.g.w[k] : 1u;
        tw += we;
        bk = umax64(bk, ((u64)we << 32) | tie_code(tie, a.g.col[k]));
    }
    block_reduce(red[0], bk, tw, z, zo);
    const uint32_t best = tie_label(tie, (uint32_t)bk);
    u64 ksum = 0, kcnt = 0;
    for (uint64_t k = b + threadIdx.x; k < e; k += 256) {
        const uint32_t we = a.g.w ? a.g.w[k] : 1u;
        if (we > 0 && (u64)we * V >= tw) {
            ksum += (u64)we * kOne;
            ++kcnt;
        }
    }
    u64 z2 = 0;
    zo = 0;
    block_reduce(red[1], z2, ksum, kcnt, zo);
    if (kcnt == 0) {
        if (threadIdx.x == 0) copra_alone(a, v, best);
        return best;
    }
    for (uint64_t k = b + threadIdx.x; k < e; k += 256) {
        const uint32_t we = a.g.w ? a.g.w[k] : 1u;
        if (we > 0 && (u64)we * V >= tw) {
            const uint32_t j = atomicAdd(kn, 1u);
            klab[j] = a.g.col[k];
            kcoef[j] = (uint32_t)(((u64)we << 32) / ksum);  // (w * 2^16) * 2^16 / kept_sum
        }
    }
    __syncthreads();
    if (threadIdx.x < 64) copra_store(a, v, threadIdx.x, klab, kcoef, (uint32_t)kcnt, best);
    return best;
}

// One block per row of deg * V > 512 (rows listed in `rows`), an LDS table
// of 2048 slots when deg * V <= 1024 (never more than 3/4 full) and of 4096
// otherwise; rows with too many distinct labels are listed for the global
// table.  While a row is finished, the bounds and the first 256 column ids
// of the block's next row are already on their way.
__global__ __launch_bounds__(256) void copra_block_k(CopraArgs a, const uint32_t *__restrict__ rows, uint32_t count) {
    __shared__ uint32_t key[kCopraBlockSlots];
    __shared__ u64 tal[kCopraBlockSlots];
    __shared__ BlockRed red[3];
    __shared__ uint32_t klab[64], kcoef[64], kn, claimed, full;
    const uint32_t V = a.V;
    u64 chg = 0;
    // the row prefetched by the previous turn (kNone: none)
    uint32_t pv = kNone, pu = 0, pw = 0;
    uint64_t pb = 0, pe = 0;
    for (uint32_t it = blockIdx.x; it < count; it += gridDim.x) {
        const uint32_t v = rows[it];
        const bool have = pv == v;
        pv = kNone;
        if (!copra_votes(a, v)) {
            copra_copy(a, v, threadIdx.x, 256);
            continue;
        }
        const Tie tie = copra_tie(a, v);
        if (a.first && a.distinct[v]) {
            // every neighbour still alone and listed once: label u's tally is
            // w(v,u) * 2^16, so the row is decided without a table
            if (threadIdx.x == 0) kn = 0;
            const uint32_t best = copra_first_block(a, v, tie, red, klab, kcoef, &kn);
            if (threadIdx.x == 0) chg += a.in[(u64)v * a.stride + 1] != best;
            __syncthreads();
            continue;
        }
        const uint64_t b = have ? pb : a.g.rp[v], e = have ? pe : a.g.rp[v + 1];
        const uint32_t S = (e - b) * V <= kCopraBlockSlots / 4 ? kCopraBlockSlots / 2 : kCopraBlockSlots;
        const uint32_t fill = S / 4 * 3;
        for (uint32_t s = threadIdx.x; s < S; s += 256) {
            key[s] = kEmptyKey;
            tal[s] = 0;
        }
        if (threadIdx.x == 0) {
            kn = 0;
            claimed = 0;
            full = 0;
        }
        // the next row's bounds
        const uint32_t vn = it + gridDim.x < count ? rows[it + gridDim.x] : kNone;
        uint64_t nb = 0, ne = 0;
        if (vn != kNone) {
            nb = a.g.rp[vn];
            ne = a.g.rp[vn + 1];
        }
        __syncthreads();
        u64 tw = 0;
        for (uint64_t k = b + threadIdx.x; k < e; k += 256) {
            const bool first = have && k == b + threadIdx.x;
            const uint32_t we = first ? pw : (a.g.w ? a.g.w[k] : 1u);
            tw += we;
            if (__atomic_load_n(&full, __ATOMIC_RELAXED)) continue;
            const uint32_t u = first ? pu : a.g.col[k];
            const uint32_t c = a.in[(u64)u * a.stride];
            for (uint32_t i = 0; i < c; ++i) {
                // the table is given up once 3/4 of it is claimed (or a probe
                // finds no slot): the row then goes to the device-memory table
                if (__atomic_load_n(&full, __ATOMIC_RELAXED)) break;
                const int r = copra_insert_bounded(key, tal, S - 1, a.in[(u64)u * a.stride + 2 + 2 * i],
                                                   (u64)we * a.in[(u64)u * a.stride + 3 + 2 * i]);
                if (r < 0 || (r > 0 && atomicAdd(&claimed, 1u) + 1 >= fill)) {
                    __atomic_store_n(&full, 1u, __ATOMIC_RELAXED);
                    break;
                }
            }
        }
        // the next row's first column ids and weights, read while this one
        // is finished
        if (vn != kNone) {
            const uint64_t k = nb + threadIdx.x;
            pu = k < ne ? a.g.col[k] : 0u;
            pw = k < ne ? (a.g.w ? a.g.w[k] : 1u) : 0u;
            pb = nb;
            pe = ne;
            pv = vn;
        }
        u64 z1 = 0, z2 = 0;
        uint32_t zo = 0;
        block_reduce(red[2], z1, tw, z2, zo);
        if (full) {
            if (threadIdx.x == 0) a.ovf_rows[atomicAdd(a.ovf_count, 1u)] = v;
            __syncthreads();
            continue;
        }
        const uint32_t best = copra_finish_block(a, v, tie, key, tal, S, tw * kOne, red, klab, kcoef, &kn);
        if (threadIdx.x == 0) chg += a.in[(u64)v * a.stride + 1] != best;
        __syncthreads();  // tables and reductions are reused by the next row
    }
    block_count(chg, a.changed);
}

// Rows left to device-memory tables, in pieces: each block takes a piece
// (row index i of the list, arcs [b0, b1), at most 2048 / V arcs, so at
// most 2048 entries), sums them in a 4096-slot LDS table, then adds each of
// its distinct labels once to row i's table at slab + off[i] (of off[i+1] -
// off[i] slots, empty beforehand) and its weights to total[i].  A hot
// label costs one device atomic per piece, and a long row is spread over
// many blocks.
__global__ __launch_bounds__(256) void copra_gpiece_k(CopraArgs a, const CopraPiece *__restrict__ pieces,
                                                      uint32_t count, const u64 *__restrict__ off, uint32_t *slab_key,
                                                      u64 *slab_tal, u64 *total) {
    __shared__ uint32_t key[kCopraBlockSlots];
    __shared__ u64 tal[kCopraBlockSlots];
    for (uint32_t it = blockIdx.x; it < count; it += gridDim.x) {
        const CopraPiece pc = pieces[it];
        for (uint32_t s = threadIdx.x; s < kCopraBlockSlots; s += 256) {
            key[s] = kEmptyKey;
            tal[s] = 0;
        }
        __syncthreads();
        const u64 o = off[pc.i];
        const uint32_t S = (uint32_t)(off[pc.i + 1] - o);
        u64 tw = 0;
        for (uint64_t k = pc.b0 + threadIdx.x; k < pc.b1; k += 256) {
            const uint32_t we = a.g.w ? a.g.w[k] : 1u;
            tw += we;
            const uint32_t u = a.g.col[k];
            const uint32_t c = a.in[(u64)u * a.stride];
            for (uint32_t i = 0; i < c; ++i) {
                const uint32_t l = a.in[(u64)u * a.stride + 2 + 2 * i];
                const u64 x = (u64)we * a.in[(u64)u * a.stride + 3 + 2 * i];
                // a piece has at most 2048 entries: the LDS table never fills
                if (copra_insert_bounded(key, tal, kCopraBlockSlots - 1, l, x) < 0 &&
                    copra_insert_bounded(slab_key + o, slab_tal + o, S - 1, l, x) < 0)
                    atomicOr(a.err, ERR_TABLE);
            }
        }
        if (tw) atomicAdd(&total[pc.i], tw);
        __syncthreads();
        for (uint32_t s = threadIdx.x; s < kCopraBlockSlots; s += 256) {
            const uint32_t l = key[s];
            if (l != kEmptyKey && copra_insert_bounded(slab_key + o, slab_tal + o, S - 1, l, tal[s]) < 0)
                atomicOr(a.err, ERR_TABLE);  // cannot happen: S >= 2 * distinct labels
        }
        __syncthreads();  // the LDS table is cleared for the next piece
    }
}

// The decision of the listed rows from their filled device-memory tables,
// spread over slices of at most kSliceSlots slots (item = row index i of
// the list, slots [s0, s1) of its table) so that no table is read by one
// block alone.  Per listed row, R holds: m1 (largest tally + 1), bc (largest
// tie code among the heaviest labels), ksum / kcnt (kept tallies), kn and
// up to V kept (label, tally) pairs.  Pass 0 finds m1, pass 1 bc and the
// kept sums, pass 2 lists the kept labels; copra_gdone_k writes the state.
struct CopraRows {
    u64 *m1, *bc, *ksum, *kcnt;
    uint32_t *kn;
    uint32_t *klab;  // V per row
    u64 *ktal;       // V per row
};

template <int PASS>
__global__ __launch_bounds__(256) void copra_gscan_k(CopraArgs a, const uint32_t *__restrict__ rows,
                                                     const CopraPiece *__restrict__ slices, uint32_t count,
                                                     const uint32_t *slab_key, const u64 *slab_tal,
                                                     const u64 *__restrict__ total, CopraRows R) {
    __shared__ BlockRed red;
    const uint32_t V = a.V;
    for (uint32_t it = blockIdx.x; it < count; it += gridDim.x) {
        const CopraPiece sl = slices[it];
        const uint32_t i = sl.i;
        const u64 tot = total[i] * kOne;
        const Tie tie = copra_tie(a, rows[i]);
        const u64 m1 = PASS ? R.m1[i] : 0;
        u64 x = 0, ks = 0, kc = 0;
        uint32_t zo = 0;
        for (uint64_t s = sl.b0 + threadIdx.x; s < sl.b1; s += 256) {
            const uint32_t l = slab_key[s];
            if (l == kEmptyKey) continue;
            const u64 t = slab_tal[s];
            if (PASS == 0) {
                x = umax64(x, t + 1);
            } else if (t > 0 && t * V >= tot) {
                if (PASS == 1) {
                    ks += t;
                    ++kc;
                } else {
                    const uint32_t j = atomicAdd(&R.kn[i], 1u);  // at most V kept labels per row
                    R.klab[(u64)i * V + j] = l;
                    R.ktal[(u64)i * V + j] = t;
                }
            }
            if (PASS == 1 && t + 1 == m1) x = umax64(x, tie_code(tie, l));
        }
        if (PASS < 2) {
            block_reduce(red, x, ks, kc, zo);
            if (threadIdx.x == 0) {
                if (x) atomicMax(PASS == 0 ? &R.m1[i] : &R.bc[i], x);
                if (ks) atomicAdd(&R.ksum[i], ks);
                if (kc) atomicAdd(&R.kcnt[i], kc);
            }
            __syncthreads();  // the reduction slots are reused by the next slice
        }
    }
}

// One wavefront per listed row: the state from the decided quantities.
__global__ __launch_bounds__(256) void copra_gdone_k(CopraArgs a, const uint32_t *__restrict__ rows, uint32_t count,
                                                     CopraRows R) {
    __shared__ uint32_t sklab[4][64], skcoef[4][64];
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t V = a.V;
    u64 chg = 0;
    for (uint32_t i = blockIdx.x * 4 + wave; i < count; i += gridDim.x * 4) {
        const uint32_t v = rows[i];
        const Tie tie = copra_tie(a, v);
        const uint32_t best = tie_label(tie, (uint32_t)R.bc[i]);
        const uint32_t kn = (uint32_t)R.kcnt[i];
        if (kn == 0) {
            if (lane == 0) copra_alone(a, v, best);
        } else {
            const u64 ksum = R.ksum[i];
            if (lane < kn) {
                sklab[wave][lane] = R.klab[(u64)i * V + lane];
                skcoef[wave][lane] = (uint32_t)(R.ktal[(u64)i * V + lane] * kOne / ksum);
            }
            wave_sync();
            copra_store(a, v, lane, sklab[wave], skcoef[wave], kn, best);
        }
        if (lane == 0) chg += a.in[(u64)v * a.stride + 1] != best;
        wave_sync();
    }
    block_count(chg, a.changed);
}

// Slices of the listed rows' tables: row i gets ceil(size / per) slices
// starting at first[i], covering its slots [off[i], off[i+1]).
__global__ void copra_slices_k(const u64 *off, uint32_t count, const u64 *first, uint32_t per,
                               CopraPiece *slices) {
    for (uint32_t i = blockIdx.x; i < count; i += gridDim.x) {
        const u64 b = off[i], e = off[i + 1];
        const u64 p0 = first[i];
        const u64 np = (e - b + per - 1) / per;
        for (u64 j = threadIdx.x; j < np; j += blockDim.x) {
            const uint64_t b0 = b + j * per;
            slices[p0 + j] = CopraPiece{i, 0u, b0, b0 + per < e ? b0 + per : e};
        }
    }
}

// Pieces of the listed rows: row i gets ceil(deg / per) pieces starting at
// first[i] (an exclusive prefix sum), each of at most `per` arcs.
__global__ void copra_pieces_k(Graph g, const uint32_t *rows, uint32_t count, const u64 *first, uint32_t per,
                               CopraPiece *pieces) {
    for (uint32_t i = blockIdx.x; i < count; i += gridDim.x) {
        const uint32_t v = rows[i];
        const uint64_t b = g.rp[v], e = g.rp[v + 1];
        const u64 p0 = first[i];
        const u64 np = (e - b + per - 1) / per;
        for (u64 j = threadIdx.x; j < np; j += blockDim.x) {
            const uint64_t b0 = b + j * per;
            pieces[p0 + j] = CopraPiece{i, 0u, b0, b0 + per < e ? b0 + per : e};
        }
    }
}

// Every vertex its own community with belonging 1.
__global__ void copra_init_k(uint32_t n, uint32_t stride, uint32_t *rec) {
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        uint32_t *r = rec + (u64)v * stride;
        r[0] = 1;
        r[1] = v;
        r[2] = v;
        r[3] = kOne;
    }
}

// Records to the caller's arrays (one thread per vertex).
__global__ void copra_output_k(const uint32_t *rec, uint32_t n, uint32_t V, uint32_t stride, uint32_t *best,
                               uint32_t *labs, uint32_t *coefs, uint32_t *cnt) {
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const uint32_t *r = rec + (u64)v * stride;
        best[v] = r[1];
        if (cnt) cnt[v] = r[0];
        for (uint32_t i = 0; i < r[0]; ++i) {
            if (labs) labs[(u64)v * V + i] = r[2 + 2 * i];
            if (coefs) coefs[(u64)v * V + i] = r[3 + 2 * i];
        }
    }
}

// Rows by class, appended in any order (the result does not depend on it):
// class 0 deg * V <= 32, class 1 <= 512, class 2 larger; rows without arcs
// are in no list (their state never changes: both buffers hold it).  Each
// block takes a contiguous run of vertices, counts its rows per class, takes
// its three list ranges with one device atomic per class, then writes: a
// few hundred atomics in all, not one per wavefront on three hot words.
constexpr uint32_t kListBlocks = 1024;
__device__ __forceinline__ int copra_class(const Graph &g, uint32_t V, uint32_t v) {
    const uint64_t d = (g.rp[v + 1] - g.rp[v]) * V;
    return d == 0 ? -1 : d <= 32 ? 0 : d <= 128 ? 1 : d <= 512 ? 2 : 3;
}
struct CopraLists {
    uint32_t *rows[kCopraClasses];
};
__global__ __launch_bounds__(256) void copra_list_k(Graph g, uint32_t V, CopraLists L, uint32_t *count) {
    constexpr int NC = kCopraClasses;
    __shared__ uint32_t cnt[NC], base[NC];
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t per = (g.n + gridDim.x - 1) / gridDim.x;
    const uint32_t lo = blockIdx.x * per, hi = min(lo + per, g.n);
    if (threadIdx.x < NC) cnt[threadIdx.x] = 0;
    __syncthreads();
    uint32_t mine[NC] = {0, 0, 0, 0};
    for (uint32_t v = lo + threadIdx.x; v < hi; v += 256) {
        const int c = copra_class(g, V, v);
#pragma unroll
        for (int k = 0; k < NC; ++k) mine[k] += c == k ? 1u : 0u;
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const uint32_t t = wave_sum(mine[c]);
        if (lane == 0 && t) atomicAdd(&cnt[c], t);
    }
    __syncthreads();
    if (threadIdx.x < NC) {
        base[threadIdx.x] = cnt[threadIdx.x] ? atomicAdd(&count[threadIdx.x], cnt[threadIdx.x]) : 0u;
        cnt[threadIdx.x] = 0;  // reused as this block's write cursor
    }
    __syncthreads();
    for (uint32_t v0 = lo + (threadIdx.x & ~63u); v0 < hi; v0 += 256) {  // wavefront-uniform steps
        const uint32_t v = v0 + lane;
        const int cls = v < hi ? copra_class(g, V, v) : -1;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const u64 m = __ballot(cls == c);
            if (!m) continue;
            const int lead = __ffsll((long long)m) - 1;
            uint32_t at = 0;
            if ((int)lane == lead) at = atomicAdd(&cnt[c], (uint32_t)__popcll(m));
            at = (uint32_t)__shfl((int)at, lead, 64);
            if (cls == c)
                L.rows[c][base[c] + at +
                       __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u))] = v;
        }
    }
}

// Table sizes of the listed rows, next_pow2(2 * min(deg * V, n)), and their
// numbers of pieces of at most `per` arcs.
__global__ void copra_sizes_k(Graph g, uint32_t V, const uint32_t *rows, uint32_t count, uint32_t per, u64 *size,
                              u64 *npieces) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
        const uint32_t v = rows[i];
        const u64 deg = g.rp[v + 1] - g.rp[v];
        npieces[i] = (deg + per - 1) / per;
        u64 d = deg * V;
        d = d < g.n ? d : g.n;
        u64 s = 1;
        while (s < 2 * d && s < (1ull << 31)) s <<= 1;  // 2^31 slots: more than any row's labels here
        size[i] = s;
    }
}

// The caller's CSR, checked before any round reads it: row_ptr starts at 0,
// never decreases and ends at m; every col < n; every weighted degree below
// 2^32.  With `distinct`, also whether each row's neighbours are strictly
// increasing (each listed once).  One wavefront per 64 rows: rows of at most 8 arcs one lane each,
// longer rows by the whole wavefront.
__global__ __launch_bounds__(256) void csr_check_k(Graph g, uint32_t *err, uint8_t *distinct, u64 *wsum) {
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (blockIdx.x == 0 && threadIdx.x == 0 && (g.rp[0] != 0 || g.rp[g.n] != g.m)) atomicOr(err, ERR_ROWPTR);
    uint32_t bits = 0;
    for (uint32_t base = (blockIdx.x * 4 + wave) * 64; base < g.n; base += gridDim.x * 4 * 64) {
        const uint32_t i = base + lane;
        const bool act = i < g.n;
        const uint32_t v = act ? i : 0u;
        const uint64_t b = g.rp[v], e = g.rp[v + 1];
        const bool bad = act && (b > e || e > g.m);
        bits |= bad ? ERR_ROWPTR : 0u;
        const bool ok = act && !bad;
        const bool one = ok && e - b <= 8;
        if (one) {
            u64 tw = 0;
            bool inc = true;  // neighbours strictly increasing: each listed once
            uint32_t prev = 0;
            for (uint64_t k = b; k < e; ++k) {
                const uint32_t u = g.col[k];
                bits |= u >= g.n ? ERR_COL : 0u;
                inc &= k == b || u > prev;
                prev = u;
                tw += g.w ? g.w[k] : 1u;
            }
            bits |= tw > 0xFFFFFFFFull ? ERR_WOVF : 0u;
            if (distinct) distinct[v] = inc;
        } else if (act && distinct) {
            distinct[v] = 0;
        }
        u64 longm = __ballot(ok && !one);
        while (longm) {
            const int j = __ffsll((long long)longm) - 1;
            longm &= longm - 1;
            const uint64_t bj = __shfl(b, j, 64), ej = __shfl(e, j, 64);
            // the first kHeadArcs arcs here, the rest in csr_check_tail_k
            const uint64_t eh = ej - bj > kHeadArcs ? bj + kHeadArcs : ej;
            u64 tw = 0;
            bool inc = true;
            for (uint64_t k = bj + lane; k < eh; k += 64) {
                const uint32_t u = g.col[k];
                bits |= u >= g.n ? ERR_COL : 0u;
                inc &= k + 1 >= ej || u < g.col[k + 1];
                tw += g.w ? g.w[k] : 1u;
            }
            tw = wave_sum(tw);
            bits |= tw > 0xFFFFFFFFull ? ERR_WOVF : 0u;
            const bool all_inc = __ballot(!inc) == 0;
            if (lane == 0) {
                if (distinct) distinct[base + j] = all_inc;
                if (eh < ej) wsum[base + j] = tw;  // the tail adds the rest
            }
        }
    }
    if (bits) atomicOr(err, bits);
}

// The tails of rows longer than kHeadArcs (see mod_tail_k): col < n, each
// neighbour once, and the weighted degree, completed by device atomics on
// wsum (the adder that completes the row sees its total).
__global__ __launch_bounds__(256) void csr_check_tail_k(Graph g, uint32_t *err, uint8_t *distinct, u64 *wsum) {
    __shared__ BlockRed R;
    __shared__ uint32_t srow;
    const u64 m = g.m;
    const u64 nchunks = (m + kHeadArcs - 1) / kHeadArcs;
    uint32_t bits = 0;
    for (u64 c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const u64 c0 = c * kHeadArcs, c1 = c0 + kHeadArcs < m ? c0 + kHeadArcs : m;
        __syncthreads();  // every wave has read the previous chunk's srow
        if (threadIdx.x == 0) srow = row_of_arc(g, c0);
        __syncthreads();
        const uint32_t r = srow;
        const uint64_t b = g.rp[r], e = g.rp[r + 1];
        if (b > e || e > m) continue;  // malformed row: flagged by csr_check_k
        const uint64_t t0 = c0 > b + kHeadArcs ? c0 : b + kHeadArcs, t1 = c1 < e ? c1 : e;
        if (t0 >= t1) continue;  // uniform: the chunk meets no tail
        u64 tw = 0, z = 0, z2 = 0;
        uint32_t viol = 0;
        for (uint64_t k = t0 + threadIdx.x; k < t1; k += 256) {
            const uint32_t u = g.col[k];
            bits |= u >= g.n ? ERR_COL : 0u;
            viol |= (k + 1 < e && u >= g.col[k + 1]) ? 1u : 0u;
            tw += g.w ? g.w[k] : 1u;
        }
        block_reduce(R, z, tw, z2, viol);
        if (threadIdx.x == 0) {
            if (viol && distinct) distinct[r] = 0;
            const u64 before = atomicAdd(&wsum[r], tw);
            if (before + tw > 0xFFFFFFFFull) bits |= ERR_WOVF;
        }
    }
    if (bits) atomicOr(err, bits);
}

hipError_t launch_csr_check(const Graph &g, uint32_t *err, uint8_t *distinct, u64 *wsum, hipStream_t s) {
    if (g.n == 0) return hipSuccess;
    csr_check_k<<<grid_for(g.n, 256, 4096), 256, 0, s>>>(g, err, distinct, wsum);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && g.m > kHeadArcs) {
        csr_check_tail_k<<<grid_for(g.m, kHeadArcs, 4096), 256, 0, s>>>(g, err, distinct, wsum);
        e = hipGetLastError();
    }
    return e;
}
hipError_t launch_copra_init(uint32_t n, uint32_t stride, uint32_t *rec, hipStream_t s) {
    if (n == 0) return hipSuccess;
    copra_init_k<<<grid_for(n, 256, 8192), 256, 0, s>>>(n, stride, rec);
    return hipGetLastError();
}
hipError_t launch_copra_output(const uint32_t *rec, uint32_t n, uint32_t V, uint32_t stride, uint32_t *best,
                               uint32_t *labs, uint32_t *coefs, uint32_t *cnt, hipStream_t s) {
    if (n == 0) return hipSuccess;
    copra_output_k<<<grid_for(n, 256, 8192), 256, 0, s>>>(rec, n, V, stride, best, labs, coefs, cnt);
    return hipGetLastError();
}
hipError_t launch_copra_list(const Graph &g, uint32_t V, uint32_t *const *rows, uint32_t *count, hipStream_t s) {
    if (g.n == 0) return hipSuccess;
    CopraLists L;
    for (int c = 0; c < kCopraClasses; ++c) L.rows[c] = rows[c];
    copra_list_k<<<grid_for(g.n, 256, kListBlocks), 256, 0, s>>>(g, V, L, count);
    return hipGetLastError();
}
hipError_t launch_copra_sizes(const Graph &g, uint32_t V, const uint32_t *rows, uint32_t count, uint32_t per,
                              u64 *size, u64 *npieces, hipStream_t s) {
    if (count == 0) return hipSuccess;
    copra_sizes_k<<<grid_for(count, 256, 4096), 256, 0, s>>>(g, V, rows, count, per, size, npieces);
    return hipGetLastError();
}
hipError_t launch_copra_round(const CopraArgs &a, const uint32_t *const *rows, const uint32_t *count,
                              hipStream_t s) {
    hipError_t e = hipSuccess;
    if (count[0]) {
        copra_group_k<<<grid_for(count[0], 16, 8192), 256, 0, s>>>(a, rows[0], count[0]);
        e = hipGetLastError();
    }
    if (e == hipSuccess && count[1]) {
        copra_wave_k<kCopraWaveSlotsSmall><<<grid_for(count[1], 4, 8192), 256, 0, s>>>(a, rows[1], count[1]);
        e = hipGetLastError();
    }
    if (e == hipSuccess && count[2]) {
        copra_wave_k<kCopraWaveSlots><<<grid_for(count[2], 4, 8192), 256, 0, s>>>(a, rows[2], count[2]);
        e = hipGetLastError();
    }
    if (e == hipSuccess && count[3]) {
        copra_block_k<<<grid_for(count[3], 1, 4096), 256, 0, s>>>(a, rows[3], count[3]);
        e = hipGetLastError();
    }
    return e;
}
hipError_t launch_copra_global(const CopraArgs &a, const uint32_t *rows, uint32_t count, const u64 *first,
                               uint32_t per, CopraPiece *pieces, uint64_t npieces, const u64 *off, uint32_t *slab_key,
                               u64 *slab_tal, u64 *total, const u64 *sfirst, CopraPiece *slices, uint64_t nslices,
                               u64 *rowstate, hipStream_t s) {
    if (count == 0) return hipSuccess;
    CopraRows R;
    R.m1 = rowstate;
    R.bc = rowstate + count;
    R.ksum = rowstate + 2 * (u64)count;
    R.kcnt = rowstate + 3 * (u64)count;
    R.kn = reinterpret_cast<uint32_t *>(rowstate + 4 * (u64)count);
    R.ktal = rowstate + 5 * (u64)count;
    R.klab = reinterpret_cast<uint32_t *>(rowstate + 5 * (u64)count + (u64)count * a.V);
    copra_pieces_k<<<grid_for(count, 1, 4096), 256, 0, s>>>(a.g, rows, count, first, per, pieces);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) {
        copra_slices_k<<<grid_for(count, 1, 4096), 256, 0, s>>>(off, count, sfirst, kSliceSlots, slices);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        copra_gpiece_k<<<grid_for(npieces, 1, 8192), 256, 0, s>>>(a, pieces, (uint32_t)npieces, off, slab_key,
                                                                  slab_tal, total);
        e = hipGetLastError();
    }
    const unsigned gs = grid_for(nslices, 1, 8192);
    if (e == hipSuccess) {
        copra_gscan_k<0><<<gs, 256, 0, s>>>(a, rows, slices, (uint32_t)nslices, slab_key, slab_tal, total, R);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        copra_gscan_k<1><<<gs, 256, 0, s>>>(a, rows, slices, (uint32_t)nslices, slab_key, slab_tal, total, R);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        copra_gscan_k<2><<<gs, 256, 0, s>>>(a, rows, slices, (uint32_t)nslices, slab_key, slab_tal, total, R);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        copra_gdone_k<<<grid_for(count, 4, 4096), 256, 0, s>>>(a, rows, count, R);
        e = hipGetLastError();
    }
    return e;
}

}  // namespace lpa
