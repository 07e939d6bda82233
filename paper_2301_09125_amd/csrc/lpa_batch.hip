// lpa_batch.hip -- RAK (arXiv 2301.09125, Section 3.2) on many independent
// graphs at once, all rounds in one persistent launch.
//
// The graphs are packed into one CSR whose arcs stay inside their graph and
// relabelled like a single graph (lpa_internal.h).  Inside a degree bin the
// internal ids keep the original order, so the rows of graph g in bin b form
// one contiguous segment seg_lo[b][g] .. + seg_cnt[b][g].  Each graph keeps
// its own tolerance test (changed_g <= floor(tol * n_g)) and round count; a
// graph that passes it (or reaches max_iter) stops voting, and its labels stay
// in the buffer its last round wrote, so every graph ends exactly as a run of
// that graph alone.
//
// Work units: one row (long, wide and wavefront bins) or 64 rows of one lane
// each (thread and group bins), never spanning two graphs.
// One launch of co-resident blocks; per round:
//   phase A  for each bin, the units of the graphs still voting are split
//            into equal contiguous ranges, one per block, whose wavefronts
//            take chunks of it from an LDS counter; a wavefront adds its
//            changed count to a graph's counter once per run of units of
//            that graph.
//   barrier
//   phase B  every block applies the tolerance test of the graphs of its
//            slice (G / nblocks graphs, rounded up to a power of two), then
//            prefix-sums the units of the slice's graphs that go on (per
//            bin) and publishes the slice's totals.
//   barrier  every block leaves once no graph is voting; otherwise each
//            block prefix-sums the slices' totals in LDS (a graph's prefix
//            is its slice's base plus its prefix inside the slice).
// Barriers count arrivals with an atomic and release on a generation
// number; a wait longer than the time limit raises ERR_TIMEOUT and every
// block leaves the kernel, so the launch always ends.

#include "lpa_sortnet.h"
#include "lpa_vote_dev.h"

namespace lpa {

constexpr int kBatchThreads = 1024;
constexpr int kBatchWaves = kBatchThreads / 64;

// rows per work unit of each bin
__device__ __forceinline__ uint32_t unit_rows(int b) { return b == BIN_THREAD || b == BIN_GROUP ? 64u : 1u; }

// Grid-wide barrier over `nblocks` co-resident blocks, in two levels: the
// blocks are split into up to kBarGroups groups (block k in group
// k % groups), each counting its arrivals in a word of its own, and the last
// arrival of each group counts the group in the top word; the last group's
// last block advances the generation.  So no more than kBarGroups arrivals
// meet on one word (every device-scope atomic on a word is serialised where
// the dies meet).  The counters only grow (cleared before the launch): the
// k-th arrival of a group of size s closes it when k % s == 0.  The waiting
// blocks poll the generation word with relaxed loads and acquire once,
// after it moved: an acquiring load at device scope also invalidates the L2
// of the CU's die, so polling with it would keep evicting the labels of the
// blocks that are still voting.
constexpr uint32_t kBarGroups = 16;
constexpr uint32_t kBarStride = 32;  // words between counters (128 bytes)
static_assert(kBarStride * (1 + kBarGroups) <= (uint32_t)kBatchBarWords, "barrier words");
__device__ __forceinline__ bool grid_barrier(const BatchArgs &b, uint32_t nblocks) {
    __shared__ int failed;
    __syncthreads();
    if (threadIdx.x == 0) {
        failed = 0;
        const uint32_t ng = nblocks < kBarGroups ? nblocks : kBarGroups;
        const uint32_t grp = blockIdx.x % ng;
        const uint32_t gsize = (nblocks - grp + ng - 1) / ng;
        const uint32_t gen = __hip_atomic_load(&b.bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        bool last = false;
        if ((atomicAdd(&b.bar[kBarStride * (1 + grp)], 1u) + 1) % gsize == 0)
            last = (atomicAdd(&b.bar[0], 1u) + 1) % ng == 0;
        if (last) {
            __threadfence();
            __hip_atomic_fetch_add(&b.bar[1], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            const uint64_t t0 = wall_clock64();
            // a block that gave up never arrives again: the others leave as
            // soon as they see its error bit instead of running into their
            // own limits
            while (__hip_atomic_load(&b.bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                __builtin_amdgcn_s_sleep(1);
                if (wall_clock64() - t0 > b.timeout_ticks ||
                    (__hip_atomic_load(b.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & ERR_TIMEOUT)) {
                    atomicOr(b.err, ERR_TIMEOUT);
                    failed = 1;
                    break;
                }
            }
        }
        __threadfence();
        if (__hip_atomic_load(b.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & ERR_TIMEOUT) failed = 1;
    }
    __syncthreads();
    return failed == 0;
}

// In round 1, every arc must stay inside its graph.
template <int A>
__device__ __forceinline__ void check_graph(const BatchArgs &b, const uint32_t (&u)[A], uint32_t valid,
                                            uint32_t g) {
    uint32_t gj[A];
#pragma unroll
    for (int j = 0; j < A; ++j) gj[j] = b.gid[u[j]];  // u = 0 past the row: every lookup in flight at once
    bool bad = false;
#pragma unroll
    for (int j = 0; j < A; ++j) bad |= (valid >> j & 1u) && gj[j] != g;
    if (bad) atomicOr(b.err, ERR_GRAPH);
}

// One row v of graph g: at most SLOTS/2 arcs through the wavefront's LDS
// table, or, when `long_row` (h = its index among the long rows), any number
// of arcs in SLOTS/2-arc chunks merged exactly in the row's global slab.
template <int SLOTS>
__device__ uint32_t unit_wave(const BatchArgs &b, const RoundArgs &a, u64 *T, uint32_t v, uint32_t h, uint32_t g,
                              bool long_row, bool round1) {
    constexpr int CHUNK = SLOTS / 2, A = CHUNK / 64;
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t rb = a.g.rp[v], re = a.g.rp[v + 1];
    const uint32_t own = a.L_old[v];
    u64 own_w = 0, rs = 0, best = 0;
    uint32_t own_hit = 0;
    for (uint64_t k0 = rb; k0 < re; k0 += CHUNK) {
        const uint64_t k1 = re < k0 + CHUNK ? re : k0 + CHUNK;
        uint32_t u[A], lab[A], wt[A], valid = 0;
        load_arcs<A, 64>(a, k0 + lane, k1, u, wt, valid);
        if (round1) check_graph<A>(b, u, valid, g);
        gather_labels<A>(a, u, valid, lab);
        uint32_t rem = 0;
        split_own<A>(lab, wt, valid, own, own_w, own_hit, rem, rs);
        uint32_t S = next_pow2(2u * (uint32_t)(k1 - k0));
        S = S < 64u ? 64u : (S > (uint32_t)SLOTS ? (uint32_t)SLOTS : S);
        if (__ballot(rem != 0)) {
            wave_peel<A, 2>(T, S - 1, lab, wt, rem);
#pragma unroll
            for (int j = 0; j < A; ++j)
                if (rem >> j & 1u) lds_insert(T, S - 1, lab[j], wt[j]);
            wave_sync();
            if (long_row) {
                flush_table(T, S, b.slab + b.slab_off[h], b.slab_mask[h], b.touched + b.touched_off[h],
                            &b.tcount[h]);
            } else {
                for (uint32_t s = lane; s < S; s += 64) {
                    const u64 x = T[s];
                    if (x != EMPTY_SLOT) {
                        best = umax64(best, slot_key(kStrict, x));
                        T[s] = EMPTY_SLOT;
                    }
                }
            }
            wave_sync();
        }
    }
    if (long_row) {
        // the row's slab holds its exact tallies: take the max over the
        // claimed slots and clear them for the next round (only this
        // wavefront touches the row's slab)
        __threadfence();
        const uint32_t tc = __hip_atomic_load(&b.tcount[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        u64 *slab = b.slab + b.slab_off[h];
        const uint32_t *tl = b.touched + b.touched_off[h];
        for (uint32_t p = lane; p < tc; p += 64) {
            const uint32_t s = tl[p];
            if (s != kNone) {
                best = umax64(best,
                              slot_key(kStrict, __hip_atomic_load(&slab[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)));
                __hip_atomic_store(&slab[s], EMPTY_SLOT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        if (lane == 0) __hip_atomic_store(&b.tcount[h], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    best = wave_max64(best);
    own_w = wave_sum(own_w);
    own_hit = __ballot(own_hit != 0) != 0;
    rs = wave_sum(rs);
    bool ch = false;
    if (lane == 0) {
        if (own_hit || a.sw) best = umax64(best, vote_key(kStrict, own, own_w + a.sw));
        const uint32_t nl = best ? key_label(kStrict, best) : own;
        a.L_new[v] = nl;
        ch = nl != own;
        if (round1 && rs + a.sw > 0xFFFFFFFFull) atomicOr(a.err, ERR_WOVF);
    }
    return (uint32_t)__popcll(__ballot(ch));
}

// Position of one work unit: its graph and its rows v0 .. min(v0 + R, end) - 1.
struct UnitPos {
    uint32_t g, v0, end;
};

// Row bounds and own label of row v (v < end), or an empty row: loads are
// issued unconditionally (row 0 stands in) so that the loads of several
// units are in flight together.
__device__ __forceinline__ void row_head(const RoundArgs &a, uint32_t v, bool act, uint64_t &rb, uint64_t &re,
                                         uint32_t &own) {
    const uint32_t x = act ? v : 0u;
    const uint64_t b0 = a.g.rp[x], b1 = a.g.rp[x + 1];
    own = a.L_old[x];
    rb = b0;
    re = act ? b1 : b0;
}

// One row of d <= D arcs per lane.  The lane reads arcs o .. o + D - 1 of
// the unit (from cb, the unit's first arc; o4 = 4 o): those past its row
// belong to later rows or to the pad of kLaneArcPad arcs behind the CSR, and
// are masked (neighbour 0, label 0xFFFFFFFF - j, weight 0).  The labels are
// sorted in registers by Batcher's network (with their weights when W), then
// read run by run in increasing label order, keeping the first run of the
// largest tally: (bt, bl).  The own label's self weight is applied after the
// scan, from its plain tally ow (own_hit: it occurs among the neighbours), so
// the scan needs no per-arc test for it.  R1 (round 1): every column id is
// checked (< n, inside graph g) and the weighted degree summed into rs.
template <int D, bool W, bool R1>
__device__ __forceinline__ uint32_t lane_vote(const BatchArgs &b, const RoundArgs &a, const uint32_t *cb,
                                              const uint32_t *wb, uint32_t o4, uint32_t d, uint32_t own, uint32_t g,
                                              u64 &rs) {
    const uint32_t *cl = (const uint32_t *)((const char *)cb + o4);
    uint32_t u[D], lab[D], wt[D];
    // every read is in bounds (the pad), so none waits behind a branch
#pragma unroll
    for (int j = 0; j < D; ++j) {
        const uint32_t x = cl[j];
        u[j] = (uint32_t)j < d ? x : 0u;
    }
    if constexpr (W) {
        const uint32_t *wl = (const uint32_t *)((const char *)wb + o4);
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const uint32_t x = wl[j];
            wt[j] = (uint32_t)j < d ? x : 0u;
        }
    }
    if constexpr (R1) {
        bool bad = false;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            bad |= u[j] >= a.g.n;
            u[j] = u[j] >= a.g.n ? 0u : u[j];
        }
        if (bad) atomicOr(a.err, ERR_COL);
        check_graph<D>(b, u, d >= 32 ? 0xFFFFFFFFu : (1u << d) - 1u, g);
#pragma unroll
        for (int j = 0; j < D; ++j) rs += W ? wt[j] : ((uint32_t)j < d ? 1u : 0u);
    }
    uint32_t ow = 0;
    bool own_hit = false;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        const uint32_t x = a.L_old[u[j]];
        lab[j] = (uint32_t)j < d ? x : 0xFFFFFFFFu - (uint32_t)j;
        const bool mine = lab[j] == own;
        own_hit |= mine;
        ow += mine ? (W ? wt[j] : 1u) : 0u;
    }
    constexpr SortNet net = SortNetFor<D>::net;
#pragma unroll
    for (int c = 0; c < net.n; ++c) {
        const int i = net.a[c], k = net.b[c];
        if constexpr (W) {
            const bool s = lab[k] < lab[i];
            const uint32_t li = s ? lab[k] : lab[i], lk = s ? lab[i] : lab[k];
            const uint32_t wi = s ? wt[k] : wt[i], wk = s ? wt[i] : wt[k];
            lab[i] = li;
            lab[k] = lk;
            wt[i] = wi;
            wt[k] = wk;
        } else {
            const uint32_t lo = lab[i] < lab[k] ? lab[i] : lab[k], hi = lab[i] < lab[k] ? lab[k] : lab[i];
            lab[i] = lo;
            lab[k] = hi;
        }
    }
    // Tallies fit 32 bits: round 1 rejects rows whose weights and self weight
    // sum past them.  The distinct pad labels tally 1 (0 when W) and come
    // after every real label, so they never win while the row has an arc.
    uint32_t bt = 0, bl = 0, run = 0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        const bool same = j > 0 && lab[j] == lab[j > 0 ? j - 1 : 0];
        run = (same ? run : 0u) + (W ? wt[j] : 1u);
        const bool gt = run > bt;
        bt = gt ? run : bt;
        bl = gt ? lab[j] : bl;
    }
    if (d == 0) return own;                 // no arcs: the label stays
    if (W && bt == 0) bl = lab[0];          // every tally 0: the lowest label
    if (bl == own) return own;
    const uint32_t ot = ow + a.sw;          // the own label with its self weight
    if ((own_hit || a.sw) && (ot > bt || (ot == bt && own < bl))) return own;
    return bl;
}

// Unweighted one-lane units stage their labels in the wavefront's LDS:
// 64 rows of at most 32 arcs, so at most kLaneStage labels.
constexpr int kLaneStage = 64 * kSortNetMax;

// The labels of the unit's arcs B .. B + nA - 1 (nA >= 1), read 64
// consecutive arcs per pass (lanes past the end repeat the last arc) into
// stage[0 .. nA).  R1: every column id is checked (< n, inside graph g).
template <bool R1>
__device__ __forceinline__ void stage_labels(const BatchArgs &b, const RoundArgs &a, const uint32_t *cb, uint32_t nA,
                                             uint32_t g, uint32_t *stage) {
    constexpr int P = 16;  // passes in flight: a unit of up to 1024 arcs in one round trip
    const uint32_t lane = threadIdx.x & 63;
    bool bad_col = false, bad_graph = false;
    for (uint32_t q0 = 0; q0 < nA; q0 += 64 * P) {
        uint32_t q[P], u[P], x[P];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            q[p] = q0 + (uint32_t)p * 64u + lane;
            q[p] = q[p] < nA ? q[p] : nA - 1;
            u[p] = cb[q[p]];
        }
        if constexpr (R1) {
            uint32_t gj[P];
#pragma unroll
            for (int p = 0; p < P; ++p) {
                bad_col |= u[p] >= a.g.n;
                u[p] = u[p] >= a.g.n ? 0u : u[p];
                gj[p] = b.gid[u[p]];
            }
#pragma unroll
            for (int p = 0; p < P; ++p) bad_graph |= gj[p] != g;
        }
#pragma unroll
        for (int p = 0; p < P; ++p) x[p] = a.L_old[u[p]];
#pragma unroll
        for (int p = 0; p < P; ++p) stage[q[p]] = x[p];
    }
    if constexpr (R1) {
        if (bad_col) atomicOr(a.err, ERR_COL);
        if (bad_graph) atomicOr(b.err, ERR_GRAPH);
    }
}

// lane_vote for an unweighted row whose labels sit in the LDS stage from
// sl on (sl[j], j < d; what follows belongs to later rows or is stale, and
// is masked as in lane_vote).
template <int D>
__device__ __forceinline__ uint32_t lane_vote_lds(const RoundArgs &a, const uint32_t *sl, uint32_t d, uint32_t own) {
    uint32_t lab[D];
    uint32_t ow = 0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        const uint32_t x = sl[j];
        lab[j] = (uint32_t)j < d ? x : 0xFFFFFFFFu - (uint32_t)j;
        ow += lab[j] == own ? 1u : 0u;
    }
    constexpr SortNet net = SortNetFor<D>::net;
#pragma unroll
    for (int c = 0; c < net.n; ++c) {
        const int i = net.a[c], k = net.b[c];
        const uint32_t lo = lab[i] < lab[k] ? lab[i] : lab[k], hi = lab[i] < lab[k] ? lab[k] : lab[i];
        lab[i] = lo;
        lab[k] = hi;
    }
    uint32_t bt = 0, bl = 0, run = 0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        const bool same = j > 0 && lab[j] == lab[j > 0 ? j - 1 : 0];
        run = (same ? run : 0u) + 1u;
        const bool gt = run > bt;
        bt = gt ? run : bt;
        bl = gt ? lab[j] : bl;
    }
    if (d == 0) return own;
    if (bl == own) return own;
    const uint32_t ot = ow + a.sw;
    if ((ow || a.sw) && (ot > bt || (ot == bt && own < bl))) return own;
    return bl;
}

// One unit of the thread or group bin: 64 rows, one per lane, each voted by
// lane_vote (lane_vote_lds when unweighted) with the smallest network that
// holds the unit's longest row (the bin bounds it by group_max <= 32; the
// weighted round 1 takes the 32-input one).  T: the wavefront's LDS (at
// least kLaneStage words plus kSortNetMax of slack behind the last one).
template <bool W>
__device__ uint32_t unit_lanes(const BatchArgs &b, const RoundArgs &a, u64 *T, const UnitPos &up, bool round1) {
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t v = up.v0 + lane;
    const bool act = v < up.end;
    uint64_t rb, re;
    uint32_t own;
    row_head(a, v, act, rb, re, own);
    // the unit's rows hold at most 64 * 32 arcs from B on (lane 0's row is
    // always one of them)
    const uint64_t B = ((uint64_t)__builtin_amdgcn_readfirstlane((int)(rb >> 32)) << 32) |
                       (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)rb);
    const uint32_t d = (uint32_t)(re - rb);
    const uint32_t o = act ? (uint32_t)(rb - B) : 0u;
    const uint32_t *cb = a.g.col + B;
    uint32_t nl;
    u64 rs = a.sw;
    if constexpr (!W) {
        const uint32_t last = (up.end - up.v0 < 64u ? up.end - up.v0 : 64u) - 1u;
        const uint32_t nA = (uint32_t)(a.g.rp[up.v0 + last + 1] - B);
        uint32_t *stage = reinterpret_cast<uint32_t *>(T);
        wave_sync();  // the previous unit's reads of the stage are done
        if (nA) {
            if (round1)
                stage_labels<true>(b, a, cb, nA, up.g, stage);
            else
                stage_labels<false>(b, a, cb, nA, up.g, stage);
        }
        wave_sync();
        const uint32_t *sl = stage + o;
        if (__ballot(d > 16)) {
            if (!__ballot(d > 24))
                nl = lane_vote_lds<24>(a, sl, d, own);
            else
                nl = lane_vote_lds<32>(a, sl, d, own);
        } else if (__ballot(d > 8)) {
            nl = lane_vote_lds<16>(a, sl, d, own);
        } else if (__ballot(d > 4)) {
            nl = lane_vote_lds<8>(a, sl, d, own);
        } else {
            nl = lane_vote_lds<4>(a, sl, d, own);
        }
    } else {
        const uint32_t o4 = o * 4u;
        const uint32_t *wb = a.g.w + B;
        if (round1)
            nl = lane_vote<32, W, true>(b, a, cb, wb, o4, d, own, up.g, rs);
        else if (__ballot(d > 16))
            nl = lane_vote<32, W, false>(b, a, cb, wb, o4, d, own, up.g, rs);
        else
            nl = lane_vote<16, W, false>(b, a, cb, wb, o4, d, own, up.g, rs);
    }
    bool c = false;
    if (act) {
        a.L_new[v] = nl;
        c = nl != own;
        if (round1 && rs > 0xFFFFFFFFull) atomicOr(a.err, ERR_WOVF);
    }
    return (uint32_t)__popcll(__ballot(c));
}

// The units of a bin as the blocks see them in a round: the prefix sum of
// graph g is the base of its decision slice (the exclusive prefix of the
// slices' totals, in LDS) plus its prefix inside the slice.
struct PrefView {
    const uint32_t *local;  // b.pref of the bin
    const uint32_t *sbase;  // [slices] in LDS
    uint32_t G, shift, total;
    __device__ __forceinline__ uint32_t operator[](uint32_t g) const {
        return g >= G ? total : sbase[g >> shift] + local[g];
    }
};

// The segment (graph) that holds unit i of a bin: the largest g in
// [lo, lo + span) with pref[g] <= i, for non-decreasing pref, given
// pref[lo] <= i < pref[lo + span].  Searched by a whole wavefront, 64 probes
// per step (two dependent loads for span <= 4096): the answer stays in
// [lo, lo + span) with pref[lo] <= i, and the probes' test is monotone in
// the lane.
__device__ __forceinline__ uint32_t segment_search(const PrefView &pref, uint32_t lo, uint32_t span, uint32_t i) {
    const uint32_t lane = threadIdx.x & 63;
    while (span > 1) {
        const uint32_t step = (span + 63) / 64;
        const uint32_t off = lane * step;
        const bool ok = off < span && pref[lo + off] <= i;
        const u64 m = __ballot(ok);  // lane 0's probe is pref[lo] <= i
        const uint32_t J = 63u - (uint32_t)__clzll((long long)m);
        lo += J * step;
        span = span - J * step < step ? span - J * step : step;
    }
    return lo;
}

// The segment that holds unit i, from segment g on (pref[g] <= i < pref[G]):
// g itself when i < pref[g + 1], else a search of the segments after it
// (never a walk over the empty segments of graphs that stopped voting).
__device__ __forceinline__ uint32_t segment_from(const PrefView &pref, uint32_t G, uint32_t g, uint32_t i) {
    if (i < pref[g + 1]) return g;
    return segment_search(pref, g + 1, G - g - 1, i);
}

// Units i0 .. i1-1 of the thread or group bin (64 rows each, one per lane);
// changed counts go to each unit's graph, one atomic per run of units of
// one graph.  (g, p0, p1, lo, end): the segment of unit i0, as run_bin found
// it.
__device__ void run_units(const BatchArgs &b, const RoundArgs &a, u64 *T, int bin, const PrefView &pref, uint32_t i0,
                          uint32_t i1, uint32_t g, uint32_t p0, uint32_t p1, uint32_t lo, uint32_t end, bool round1) {
    uint32_t gacc = g, wch = 0;
    for (uint32_t i = i0; i < i1; ++i) {
        if (i >= p1) {  // next segment that has units this round
            if (wch && (threadIdx.x & 63) == 0) atomicAdd(&b.changed[gacc], (u64)wch);
            wch = 0;
            g = segment_from(pref, b.G, g, i);
            p0 = pref[g];
            p1 = pref[g + 1];
            lo = b.seg_lo[(size_t)bin * b.G + g];
            end = lo + b.seg_cnt[(size_t)bin * b.G + g];
            gacc = g;
        }
        const UnitPos up{g, lo + (i - p0) * 64u, end};
        wch += a.g.w ? unit_lanes<true>(b, a, T, up, round1) : unit_lanes<false>(b, a, T, up, round1);
    }
    if (wch && (threadIdx.x & 63) == 0) atomicAdd(&b.changed[gacc], (u64)wch);
}

// Units [i0, i1) of bin `bin`; g0 is the segment that holds unit i0.
template <int SLOTS>
__device__ void run_range(const BatchArgs &b, const RoundArgs &a, u64 *T, int bin, const PrefView &pref, uint32_t i0,
                          uint32_t i1, uint32_t g0, bool round1) {
    const uint32_t R = unit_rows(bin);
    uint32_t g = g0;
    uint32_t p0 = pref[g], p1 = pref[g + 1];
    uint32_t lo = b.seg_lo[(size_t)bin * b.G + g], end = lo + b.seg_cnt[(size_t)bin * b.G + g];
    // rows of at most group_max arcs: one lane each
    if (bin == BIN_THREAD || bin == BIN_GROUP) {
        run_units(b, a, T, bin, pref, i0, i1, g, p0, p1, lo, end, round1);
        return;
    }
    uint32_t wch = 0;
    for (uint32_t i = i0; i < i1; ++i) {
        if (i >= p1) {  // next segment that has units this round
            if (wch && (threadIdx.x & 63) == 0) atomicAdd(&b.changed[g], (u64)wch);
            wch = 0;
            g = segment_from(pref, b.G, g, i);
            p0 = pref[g];
            p1 = pref[g + 1];
            lo = b.seg_lo[(size_t)bin * b.G + g];
            end = lo + b.seg_cnt[(size_t)bin * b.G + g];
        }
        const uint32_t v0 = lo + (i - p0) * R;
        wch += unit_wave<SLOTS>(b, a, T, v0, v0 - b.lo[BIN_HUB], g, bin == BIN_HUB, round1);
    }
    if (wch && (threadIdx.x & 63) == 0) atomicAdd(&b.changed[g], (u64)wch);
}

// Units a wavefront takes at a time from its block's share of a bin: about
// the same work per chunk (a thread or group unit is 64 rows).
__device__ __forceinline__ uint32_t chunk_units(int bin) {
    return bin == BIN_WAVE ? 4u : (bin == BIN_WIDE ? 2u : 1u);
}

// The block's units of bin `bin` below `hi`, handed to its wavefronts a
// chunk at a time from the LDS counter *next, so that the wavefronts the
// SIMDs issue less often (the younger ones) do less of the work instead of
// finishing last; g is the segment of the block's first unit.
template <int SLOTS>
__device__ void run_bin(const BatchArgs &b, const RoundArgs &a, u64 *T, int bin, const PrefView &pref, uint32_t hi,
                        uint32_t g, uint32_t *next, bool round1) {
    const uint32_t CH = chunk_units(bin);
    for (;;) {
        uint32_t i0 = 0;
        if ((threadIdx.x & 63) == 0) i0 = atomicAdd(next, CH);
        i0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)__shfl((int)i0, 0, 64));
        if (i0 >= hi) break;
        const uint32_t i1 = i0 + CH < hi ? i0 + CH : hi;
        g = segment_from(pref, b.G, g, i0);  // a wavefront's chunks only move forward
        run_range<SLOTS>(b, a, T, bin, pref, i0, i1, g, round1);
    }
}

// Phase B, run by every block on its slice of the graphs,
// [blockIdx.x << dshift, (blockIdx.x + 1) << dshift) clipped to G: the
// tolerance tests of round t (none for t = 0), then the slice's per-bin
// prefix sums of the units of its graphs that go on voting (pref, from 0 at
// the slice's first graph) and their totals (btot[bin][block]); the block's
// voting graphs are added to n_active[t & 1], and block 0 clears the other
// word for round t + 1.  Each thread takes kDecideJ consecutive graphs per
// pass and issues all their loads (state and segment sizes) at once, so a
// slice of up to kDecideJ * kBatchThreads graphs costs one round trip to
// memory and one block-wide scan.
constexpr int kDecideJ = 4;
__device__ void decide(const BatchArgs &b, uint32_t t) {
    constexpr int J = kDecideJ;
    __shared__ uint32_t wsum[kBatchWaves][kBatchBins + 1];
    __shared__ uint32_t carry[kBatchBins + 1];
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t G = b.G;
    const uint32_t s0 = blockIdx.x << b.dshift;
    const uint32_t s1 = s0 < G ? (G - s0 < (1u << b.dshift) ? G : s0 + (1u << b.dshift)) : s0;
    if (tid == 0 && blockIdx.x == 0) b.n_active[(t + 1) & 1] = 0;
    if (tid <= kBatchBins) carry[tid] = 0;
    __syncthreads();
    for (uint32_t base = s0; base < s1; base += J * kBatchThreads) {
        const uint32_t g0 = base + tid * J;
        uint32_t act[J], cnt[J][kBatchBins];
        u64 ch[J], th[J];
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const uint32_t gc = g0 + j < s1 ? g0 + j : s0;  // s0 < s1 here
            act[j] = b.active[gc];
            ch[j] = b.changed[gc];
            th[j] = b.thr[gc];
#pragma unroll
            for (int k = 0; k < kBatchBins; ++k) cnt[j][k] = b.seg_cnt[(size_t)k * G + gc];
        }
        // x[j][k]: units of graph g0 + j in bin k if it goes on voting;
        // x[j][kBatchBins]: 1 if it does
        uint32_t x[J][kBatchBins + 1];
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const uint32_t g = g0 + j;
            bool live = g < s1 && act[j];
            if (live && t > 0) {
                b.changed[g] = 0;
                b.last[g] = ch[j];
                b.iters[g] = t;
                if (t <= b.hist_len) b.hist[(u64)g * b.hist_len + (t - 1)] = ch[j];
                const bool ok = ch[j] <= th[j];
                if (ok || t == b.max_iter) {
                    b.conv[g] = ok ? 1 : 0;
                    b.active[g] = 0;
                    live = false;
                }
            }
#pragma unroll
            for (int k = 0; k < kBatchBins; ++k) x[j][k] = live ? (cnt[j][k] + unit_rows(k) - 1) / unit_rows(k) : 0u;
            x[j][kBatchBins] = live ? 1u : 0u;
        }
        uint32_t ex[kBatchBins + 1];
#pragma unroll
        for (int k = 0; k <= kBatchBins; ++k) {
            uint32_t tot = 0;
#pragma unroll
            for (int j = 0; j < J; ++j) tot += x[j][k];
            uint32_t sc = tot;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const uint32_t y = __shfl_up(sc, off, 64);
                if ((int)lane >= off) sc += y;
            }
            if (lane == 63) wsum[wave][k] = sc;
            ex[k] = sc - tot;  // exclusive within the wavefront
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kBatchBins; ++k) {
            uint32_t off = carry[k] + ex[k];
            for (uint32_t q = 0; q < wave; ++q) off += wsum[q][k];
#pragma unroll
            for (int j = 0; j < J; ++j) {
                if (g0 + j < s1) b.pref[(size_t)k * (G + 1) + g0 + j] = off;
                off += x[j][k];
            }
        }
        __syncthreads();
        if (tid <= kBatchBins) {
            uint32_t sc = 0;
            for (int q = 0; q < kBatchWaves; ++q) sc += wsum[q][tid];
            carry[tid] += sc;
        }
        __syncthreads();
    }
    if (tid < kBatchBins) b.btot[(size_t)tid * kBatchMaxBlocks + blockIdx.x] = carry[tid];
    if (tid == kBatchBins && carry[kBatchBins]) atomicAdd(&b.n_active[t & 1], carry[kBatchBins]);
}

// Arcs voted by the graphs of this block's decision slice, once every graph
// has stopped: m_g times its rounds.
__device__ void slice_arcs(const BatchArgs &b) {
    const uint32_t G = b.G;
    const uint32_t s0 = blockIdx.x << b.dshift;
    const uint32_t s1 = s0 < G ? (G - s0 < (1u << b.dshift) ? G : s0 + (1u << b.dshift)) : s0;
    u64 arcs = 0;
    for (uint32_t g = s0 + threadIdx.x; g < s1; g += kBatchThreads) {
        const uint64_t v0 = b.gv[g], v1 = b.gv[g + 1];
        arcs += (u64)(b.orp[v1] - b.orp[v0]) * b.iters[g];
    }
    arcs = wave_sum(arcs);
    if ((threadIdx.x & 63) == 0 && arcs) atomicAdd(b.arcs, arcs);
}

template <int SLOTS>
__global__ __launch_bounds__(kBatchThreads) void batch_k(BatchArgs b, uint32_t nblocks) {
    // each wavefront's LDS: the SLOTS-slot table of its one-row units, or
    // the label stage of its one-lane units (the same words: the table is
    // cleared again at the start of every round, before the one-row bins);
    // kSortNetMax words of slack behind the last wavefront's
    constexpr int WL = SLOTS > kLaneStage / 2 ? SLOTS : kLaneStage / 2;
    __shared__ u64 table[kBatchWaves * WL + kSortNetMax / 2];
    __shared__ uint32_t next_unit[kBatchBins], share_hi[kBatchBins], share_seg[kBatchBins];
    // per bin: the exclusive prefix of the decision slices' unit totals
    __shared__ uint32_t sbase[kBatchBins][kBatchMaxBlocks], stot[kBatchBins];
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    u64 *T = table + wave * WL;
    if (blockIdx.x == 0 && threadIdx.x == 0) b.clock[0] = wall_clock64();
    // the work split of round 1: every graph votes
    decide(b, 0);
    if (!grid_barrier(b, nblocks)) return;
    for (uint32_t t = 1; t <= b.max_iter; ++t) {
        RoundArgs a;
        a.g = b.g;
        a.L_old = (t & 1) ? b.L0 : b.L1;
        a.L_new = (t & 1) ? b.L1 : b.L0;
        a.rowflag = nullptr;
        a.sw = b.sw;
        a.check = t == 1;
        a.changed = nullptr;
        a.err = b.err;
        a.list = nullptr;
        a.list_n = nullptr;
        a.top1 = a.top2 = nullptr;
        a.skip_distinct = 0;
        a.insum = nullptr;
        a.half = 0;  // synchronous rounds, strict ties
        a.tie = 0;
        a.t = t;
        a.seed = 0;
        a.orig = nullptr;
        const bool round1 = t == 1;
        // wavefront k works out bin k: the slices' bases (the exclusive
        // prefix of btot[k][0 .. nblocks), up to 64 * 8 entries), then this
        // block's share of the bin's units, [lo, hi), and the segment of its
        // first unit
        if (wave < (uint32_t)kBatchBins) {
            constexpr int C = kBatchMaxBlocks / 64;
            uint32_t v[C], sum = 0;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const uint32_t j = lane * C + c;
                v[c] = j < nblocks ? b.btot[(size_t)wave * kBatchMaxBlocks + j] : 0u;
                sum += v[c];
            }
            uint32_t incl = sum;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const uint32_t y = __shfl_up(incl, off, 64);
                if ((int)lane >= off) incl += y;
            }
            uint32_t run = incl - sum;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                sbase[wave][lane * C + c] = run;
                run += v[c];
            }
            const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
            wave_sync();
            const PrefView pv{b.pref + (size_t)wave * (b.G + 1), sbase[wave], b.G, b.dshift, total};
            const uint32_t lo = (uint32_t)((u64)blockIdx.x * total / nblocks);
            const uint32_t hi = (uint32_t)((u64)(blockIdx.x + 1) * total / nblocks);
            const uint32_t seg = lo < hi ? segment_search(pv, 0, b.G, lo) : 0u;
            if (lane == 0) {
                next_unit[wave] = lo;
                share_hi[wave] = hi;
                share_seg[wave] = seg;
                stot[wave] = total;
            }
        }
        for (uint32_t s = lane; s < SLOTS; s += 64) T[s] = EMPTY_SLOT;
        __syncthreads();
        for (int bin = BIN_HUB; bin <= BIN_THREAD; ++bin) {
            const PrefView pv{b.pref + (size_t)bin * (b.G + 1), sbase[bin], b.G, b.dshift, stot[bin]};
            run_bin<SLOTS>(b, a, T, bin, pv, share_hi[bin], share_seg[bin], &next_unit[bin], round1);
        }
        if (!grid_barrier(b, nblocks)) return;
        decide(b, t);
        if (!grid_barrier(b, nblocks)) return;
        if (__hip_atomic_load(&b.n_active[t & 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) break;
        if (__hip_atomic_load(b.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & (ERR_COL | ERR_GRAPH)) break;
    }
    slice_arcs(b);
    if (blockIdx.x == 0 && threadIdx.x == 0) b.clock[1] = wall_clock64();
}

// Graph of each internal vertex: binary search of old_of[r] in gv.
__global__ void batch_gid_k(const uint32_t *old_of, uint32_t n, const uint64_t *gv, uint32_t G, uint32_t *gid) {
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
        const uint64_t v = old_of[r];
        uint32_t lo = 0, hi = G;  // gv[lo] <= v < gv[hi]
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) / 2;
            if (gv[mid] <= v)
                lo = mid;
            else
                hi = mid;
        }
        gid[r] = lo;
    }
}

// Segment of graph g in bin k: the rows of the bin whose gid is g (gid does
// not decrease inside a bin).
__global__ void batch_seg_k(const uint32_t *gid, Bins bins, uint32_t G, uint32_t *seg_lo, uint32_t *seg_cnt) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (uint32_t)kBatchBins * G) return;
    const uint32_t k = i / G, g = i % G;
    const uint32_t lo = bins.lo[k], cnt = bins.cnt[k];
    uint32_t first = 0, last = 0;
    for (int pass = 0; pass < 2; ++pass) {
        const uint32_t key = g + pass;
        uint32_t l = 0, h = cnt;  // first row with gid >= key
        while (l < h) {
            const uint32_t mid = (l + h) / 2;
            if (gid[lo + mid] < key)
                l = mid + 1;
            else
                h = mid;
        }
        if (pass == 0)
            first = l;
        else
            last = l;
    }
    seg_lo[i] = lo + first;
    seg_cnt[i] = last - first;
}

// labels_out[old_of[r]] = final label of r, as an id local to its graph.
__global__ void batch_out_k(uint32_t *out, const uint32_t *old_of, const uint32_t *gid, const uint32_t *L0,
                            const uint32_t *L1, const uint32_t *iters, const uint64_t *gv, uint32_t n) {
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
        const uint32_t g = gid[r];
        const uint32_t lab = (iters[g] & 1u) ? L1[r] : L0[r];
        out[old_of[r]] = (uint32_t)(lab - gv[g]);
    }
}

hipError_t launch_batch_gid(const uint32_t *old_of, uint32_t n, const uint64_t *gv, uint32_t G, uint32_t *gid,
                            hipStream_t s) {
    if (n == 0) return hipSuccess;
    batch_gid_k<<<grid_for(n, 256, 8192), 256, 0, s>>>(old_of, n, gv, G, gid);
    return hipGetLastError();
}
hipError_t launch_batch_seg(const uint32_t *gid, const Bins &bins, uint32_t G, uint32_t *seg_lo, uint32_t *seg_cnt,
                            hipStream_t s) {
    const uint64_t total = (uint64_t)kBatchBins * G;
    if (total == 0) return hipSuccess;
    batch_seg_k<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(gid, bins, G, seg_lo, seg_cnt);
    return hipGetLastError();
}
hipError_t launch_batch_out(uint32_t *out, const uint32_t *old_of, const uint32_t *gid, const uint32_t *L0,
                            const uint32_t *L1, const uint32_t *iters, const uint64_t *gv, uint32_t n,
                            hipStream_t s) {
    if (n == 0) return hipSuccess;
    batch_out_k<<<grid_for(n, 256, 8192), 256, 0, s>>>(out, old_of, gid, L0, L1, iters, gv, n);
    return hipGetLastError();
}

int batch_slots(const Bins &bins) { return bins.cnt[BIN_WIDE] ? kWaveSlots : kWaveSlotsSmall; }

int batch_blocks_per_cu(int slots) {
    int per_cu = 0;
    const hipError_t e =
        slots == kWaveSlots
            ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_k<kWaveSlots>, kBatchThreads, 0)
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_k<kWaveSlotsSmall>, kBatchThreads, 0);
    if (e != hipSuccess || per_cu < 1) per_cu = 1;
    return per_cu;
}

int batch_waves_per_block() { return kBatchWaves; }

hipError_t launch_batch(const BatchArgs &b, uint32_t nblocks, int slots, hipStream_t s) {
    void *args[] = {(void *)&b, (void *)&nblocks};
    if (slots == kWaveSlots)
        return hipLaunchCooperativeKernel((const void *)batch_k<kWaveSlots>, dim3(nblocks), dim3(kBatchThreads), args,
                                          0, s);
    return hipLaunchCooperativeKernel((const void *)batch_k<kWaveSlotsSmall>, dim3(nblocks), dim3(kBatchThreads),
                                      args, 0, s);
}

}  // namespace lpa
