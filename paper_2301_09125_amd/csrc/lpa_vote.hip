// lpa_vote.hip -- the per-round vote kernels on the internal graph.
//
// Method (arXiv 2301.09125, Section 3.2): in every round each vertex adopts
// the label with the largest total edge weight among its neighbours (plus a
// self weight on its own label, the Section 3.1.2 self-loop), ties going to
// the lowest label; rounds are synchronous (read L_old, write L_new).
//
// A vote is the max over candidate labels of the 64-bit key
//     (tally << 32) | ~label,
// which orders by tally first and, among equal tallies, prefers the lowest
// label.  Tallies are u32 (weighted degrees >= 2^32 are rejected in round
// 1), all accumulation is integer, so the result does not depend on the
// order in which atomics land: the labels are deterministic.
//
// Bins (contiguous ranges of internal ids):
//   vote_thread_k  1 <= d <= 8     one lane, registers, pairwise tally
//   vote_group_k   d <= 32         16-lane group, 64-slot LDS table
//   vote_wave_k    d <= 128        one wavefront, 256-slot LDS table
//                  d <= 512        one wavefront, 1024-slot LDS table
//   vote_hub_k     d > 512         one wavefront per 512-arc segment, rows
//                                  finished by the merge kernels below
// Hashtable slots are u64 (label << 32 | tally); EMPTY has the label field all
// ones, a value no label takes (labels < n <= 2^32 - 2).  A label is claimed
// with one 64-bit CAS carrying its first weight, later hits add to the low
// half, so a slot never holds a label without its weight.
//
// Work that would serialise on one address is avoided: every vertex's own
// label is tallied in registers (most neighbours hold it in late rounds),
// and changed counts go to per-block partials spread over cache lines.
// (Pre-summing a wavefront's most frequent labels before its table, as the
// batched kernel does, measured slower in these tables.)
// Every kernel loop is wavefront-uniform and uses no block barrier, so the
// wavefronts of a block proceed independently.
//
// Round 1 from the unique initial labels needs no table for a row that lists
// each neighbour once: every label then occurs once, its tally is that arc's
// weight, and the vote is a plain max over the row.

#include "lpa_vote_dev.h"

namespace lpa {

// ---------------------------------------------------------- one lane --

// FEAT: also record the winning and the runner-up tally of every row.
template <bool FEAT>
__global__ __launch_bounds__(256) void vote_thread_k(RoundArgs a, uint32_t lo, uint32_t cnt) {
    constexpr int D = kThreadMaxCap;
    if (a.list) cnt = min(cnt, *a.list_n);
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t stride = gridDim.x * 256;
    u64 wchg = 0, ins = 0;
    // row of this lane's next work item, loaded one iteration ahead
    uint32_t vnext = 0;
    {
        const uint32_t i0 = blockIdx.x * 256 + (threadIdx.x & ~63u) + lane;
        if (i0 < cnt) vnext = row_of(a, lo, i0);
    }
    for (uint32_t base = blockIdx.x * 256 + (threadIdx.x & ~63u); base < cnt; base += stride) {
        const uint32_t i = base + lane;
        const uint32_t vcur = vnext;
        if (i + stride < cnt) vnext = row_of(a, lo, i + stride);
        bool ch = false;
        const RowMode rm = row_mode(a, vcur);  // vcur is a row of the launch (or row lo)
        if (i < cnt && !rm.on) {
            a.L_new[vcur] = a.L_old[vcur];  // the other half of a semi-synchronous round
        } else if (i < cnt && !(a.skip_distinct && (a.rowflag[vcur] & ROW_DISTINCT))) {
            const uint32_t v = vcur;
            const Tie tie = rm.tie;
            const uint64_t b = a.g.rp[v];
            const uint64_t e = a.g.rp[v + 1];
            const uint32_t own = a.L_old[v];
            uint32_t u[D], lab[D], wt[D], tl[D];
            uint32_t valid = 0;
            load_arcs<D, 1>(a, b, e, u, wt, valid);
            gather_labels<D>(a, u, valid, lab);
            u64 rs = a.sw;
#pragma unroll
            for (int j = 0; j < D; ++j) {
                rs += wt[j];
                tl[j] = wt[j] + (lab[j] == own ? a.sw : 0u);
                ins += (lab[j] == own) ? wt[j] : 0u;  // wt = 0 past the row
            }
#pragma unroll
            for (int j = 0; j < D; ++j)
#pragma unroll
                for (int k = j + 1; k < D; ++k)
                    if (lab[j] == lab[k]) {
                        tl[j] += wt[k];
                        tl[k] += wt[j];
                    }
            u64 best = a.sw ? vote_key(tie, own, a.sw) : 0ull;
            if (FEAT) {
                // the own label's key with its full tally (equal keys of one
                // label collapse in top2_add)
                u64 own_t = a.sw;
#pragma unroll
                for (int j = 0; j < D; ++j)
                    if ((valid >> j & 1u) && lab[j] == own) own_t += wt[j];
                u64 k2 = 0;
                best = a.sw ? vote_key(tie, own, own_t) : 0ull;
#pragma unroll
                for (int j = 0; j < D; ++j)
                    if (valid >> j & 1u) top2_add(best, k2, vote_key(tie, lab[j], tl[j]));
                a.top1[v] = (uint32_t)(best >> 32);
                a.top2[v] = (uint32_t)(k2 >> 32);
            } else {
#pragma unroll
                for (int j = 0; j < D; ++j)
                    if (valid >> j & 1u) best = umax64(best, vote_key(tie, lab[j], tl[j]));
            }
            const uint32_t nl = best ? key_label(tie, best) : own;
            a.L_new[v] = nl;
            ch = nl != own;
            if (a.check && rs > 0xFFFFFFFFull) atomicOr(a.err, ERR_WOVF);
        }
        wchg += __popcll(__ballot(ch));
    }
    block_counts(lane == 0 ? wchg : 0, ins, a.changed, a.insum);
}

// ---------------------------------------------- group / wavefront per row --

// G lanes per vertex (G divides 64) with a CAP-slot LDS table per group; each
// lane holds up to A = CAP / (2G) arcs.  A group's table is only touched by
// lanes of its own wavefront.
template <int G, int CAP, bool FIRST, bool FEAT>
__global__ __launch_bounds__(256) void vote_group_k(RoundArgs a, uint32_t lo, uint32_t cnt) {
    constexpr int GPB = 256 / G;  // groups per block
    constexpr int GPW = 64 / G;   // groups per wavefront
    constexpr int A = CAP / (2 * G);
    __shared__ u64 table[GPB * CAP];
    if (a.list) cnt = min(cnt, *a.list_n);
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t gl = threadIdx.x & (G - 1);
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    u64 *T = table + (threadIdx.x / G) * CAP;
    for (uint32_t s = gl; s < CAP; s += G) T[s] = EMPTY_SLOT;
    wave_sync();
    u64 wchg = 0, ins = 0;
    const uint32_t stride = gridDim.x * GPB;
    uint32_t vnext = 0;  // row of the group's next work item, loaded one iteration ahead
    {
        const uint32_t i0 = blockIdx.x * GPB + wave * GPW + lane / G;
        if (i0 < cnt) vnext = row_of(a, lo, i0);
    }
    for (uint32_t base = blockIdx.x * GPB + wave * GPW; base < cnt; base += stride) {
        const uint32_t idx = base + lane / G;
        bool act = idx < cnt;
        const uint32_t v = act ? vnext : 0u;
        if (idx + stride < cnt) vnext = row_of(a, lo, idx + stride);
        if (FIRST && act && a.skip_distinct && (a.rowflag[v] & ROW_DISTINCT)) act = false;
        const RowMode rm = row_mode(a, v);
        const Tie tie = rm.tie;  // the same in every lane of the group
        const bool keep = act && !rm.on;  // the other half of a semi-synchronous round
        act = act && rm.on;
        uint64_t b = 0, e = 0;
        uint32_t own = 0;
        if (act) {
            b = a.g.rp[v];
            e = a.g.rp[v + 1];
            own = a.L_old[v];
        }
        uint32_t u[A], lab[A], wt[A];
        uint32_t valid = 0;
        load_arcs<A, G>(a, b + gl, e, u, wt, valid);
        gather_labels<A>(a, u, valid, lab);
        u64 own_w = 0, rs = 0;
        uint32_t own_hit = 0, rem = 0;
        split_own<A>(lab, wt, valid, own, own_w, own_hit, rem, rs);
        const bool direct = FIRST && act && (a.rowflag[v] & ROW_DISTINCT);
        uint32_t S = next_pow2(2u * (uint32_t)(e - b));
        S = S < (uint32_t)G ? (uint32_t)G : (S > (uint32_t)CAP ? (uint32_t)CAP : S);
        const uint32_t mask = S - 1;
        u64 best = 0, k2 = 0;
        if (direct) {
#pragma unroll
            for (int j = 0; j < A; ++j)
                if (rem >> j & 1u) {
                    if (FEAT)
                        top2_add(best, k2, vote_key(tie, lab[j], wt[j]));
                    else
                        best = umax64(best, vote_key(tie, lab[j], wt[j]));
                }
        } else {
#pragma unroll
            for (int j = 0; j < A; ++j)
                if (rem >> j & 1u) lds_insert(T, mask, lab[j], wt[j]);
        }
        wave_sync();
        if (!direct) {
            for (uint32_t s = gl; s < S; s += G) {
                const u64 x = T[s];
                if (x != EMPTY_SLOT) {
                    if (FEAT)
                        top2_add(best, k2, slot_key(tie, x));
                    else
                        best = umax64(best, slot_key(tie, x));
                    T[s] = EMPTY_SLOT;
                }
            }
        }
        if (FEAT) {
#pragma unroll
            for (int off = G / 2; off > 0; off >>= 1) top2_xor(best, k2, off);
        }
        if (G == 16 || G == 32) {  // a group is one or two DPP rows
            if (!FEAT) best = row_max64(best);
            own_w = row_sum64(own_w);
            own_hit = row_sum32(own_hit);
            rs = row_sum64(rs);
            if (G == 32) {
                if (!FEAT) best = umax64(best, __shfl_xor(best, 16, 64));
                own_w += __shfl_xor(own_w, 16, 64);
                own_hit += __shfl_xor(own_hit, 16, 64);
                rs += __shfl_xor(rs, 16, 64);
            }
        } else {
#pragma unroll
            for (int off = G / 2; off > 0; off >>= 1) {
                if (!FEAT) best = umax64(best, __shfl_xor(best, off, 64));
                own_w += __shfl_xor(own_w, off, 64);
                own_hit |= __shfl_xor(own_hit, off, 64);
                rs += __shfl_xor(rs, off, 64);
            }
        }
        bool ch = false;
        if (act && gl == 0) {
            ins += own_w;
            if (own_hit || a.sw) {
                if (FEAT)
                    top2_add(best, k2, vote_key(tie, own, own_w + a.sw));
                else
                    best = umax64(best, vote_key(tie, own, own_w + a.sw));
            }
            if (FEAT) {
                a.top1[v] = (uint32_t)(best >> 32);
                a.top2[v] = (uint32_t)(k2 >> 32);
            }
            const uint32_t nl = best ? key_label(tie, best) : own;
            a.L_new[v] = nl;
            ch = nl != own;
            if (a.check && rs + a.sw > 0xFFFFFFFFull) atomicOr(a.err, ERR_WOVF);
        }
        if (keep && gl == 0) a.L_new[v] = a.L_old[v];
        wchg += __popcll(__ballot(ch));
        wave_sync();
    }
    block_counts(lane == 0 ? wchg : 0, ins, a.changed, a.insum);
}

// One wavefront per row of at most A*64 arcs, A arcs per lane, SLOTS LDS
// slots; the own label is summed in registers, every other arc goes to the
// table.  The next row's arcs are loaded while the current one is voted.
template <bool FIRST, bool FEAT, int A, int SLOTS>
__global__ __launch_bounds__(256) void vote_wave_k(RoundArgs a, uint32_t lo, uint32_t cnt) {
    __shared__ u64 table[4 * SLOTS];
    if (a.list) cnt = min(cnt, *a.list_n);
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    u64 *T = table + wave * SLOTS;
    for (uint32_t s = lane; s < (uint32_t)SLOTS; s += 64) T[s] = EMPTY_SLOT;
    wave_sync();
    u64 wchg = 0, ins = 0;
    const uint32_t stride = gridDim.x * 4;
    uint32_t i = blockIdx.x * 4 + wave;
    uint64_t b = 0, e = 0;
    uint32_t u[A], wt[A], valid = 0;
    uint32_t v = 0;
    // rows this launch does not vote are skipped (no loads): in round 1 the
    // rows the relabel pass already voted, in a half of a semi-synchronous
    // round the rows of the other half (`keep`: they copy their label)
    auto skipped = [&](uint32_t row) { return FIRST && a.skip_distinct && (a.rowflag[row] & ROW_DISTINCT); };
    auto other_half = [&](uint32_t row) { return a.half != 0 && !row_mode(a, row).on; };
    bool skip = false, keep = false;
    if (i < cnt) {
        v = row_of(a, lo, i);
        keep = other_half(v);
        skip = keep || skipped(v);
        if (!skip) {
            b = a.g.rp[v];
            e = a.g.rp[v + 1];
            issue_arcs<A, 64>(a, b + lane, e, u, wt, valid);
        }
    }
    while (i < cnt) {
        const uint32_t inext = i + stride;
        uint64_t nb = 0, ne = 0;
        uint32_t nu[A], nwt[A], nvalid = 0, nv = 0;
        bool nskip = false, nkeep = false;
        if (inext < cnt) {
            nv = row_of(a, lo, inext);
            nkeep = other_half(nv);
            nskip = nkeep || skipped(nv);
            if (!nskip) {
                nb = a.g.rp[nv];
                ne = a.g.rp[nv + 1];
                issue_arcs<A, 64>(a, nb + lane, ne, nu, nwt, nvalid);
            }
        }
        if (nskip || inext >= cnt) {
#pragma unroll
            for (int j = 0; j < A; ++j) nu[j] = nwt[j] = 0;
        }
        if (keep && lane == 0) a.L_new[v] = a.L_old[v];
        if (!skip) {
        check_arcs<A>(a, u);
        const Tie tie = row_mode(a, v).tie;
        const uint32_t own = a.L_old[v];
        uint32_t lab[A];
        gather_labels<A>(a, u, valid, lab);
        u64 own_w = 0, rs = 0;
        uint32_t own_hit = 0, rem = 0;
        split_own<A>(lab, wt, valid, own, own_w, own_hit, rem, rs);
        const bool direct = FIRST && (a.rowflag[v] & ROW_DISTINCT);
        uint32_t S = next_pow2(2u * (uint32_t)(e - b));
        S = S < 64u ? 64u : (S > (uint32_t)SLOTS ? (uint32_t)SLOTS : S);
        const uint32_t mask = S - 1;
        u64 best = 0, k2 = 0;
        if (direct) {
#pragma unroll
            for (int j = 0; j < A; ++j)
                if (rem >> j & 1u) {
                    if (FEAT)
                        top2_add(best, k2, vote_key(tie, lab[j], wt[j]));
                    else
                        best = umax64(best, vote_key(tie, lab[j], wt[j]));
                }
        } else if (__ballot(rem != 0)) {  // some label other than the own one
#pragma unroll
            for (int j = 0; j < A; ++j)
                if (rem >> j & 1u) lds_insert(T, mask, lab[j], wt[j]);
            wave_sync();
            for (uint32_t s = lane; s < S; s += 64) {
                const u64 x = T[s];
                if (x != EMPTY_SLOT) {
                    if (FEAT)
                        top2_add(best, k2, slot_key(tie, x));
                    else
                        best = umax64(best, slot_key(tie, x));
                    T[s] = EMPTY_SLOT;
                }
            }
        }
        if (FEAT) {
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) top2_xor(best, k2, off);
        } else {
            best = wave_max64(best);
        }
        own_w = wave_sum(own_w);
        own_hit = __ballot(own_hit != 0) != 0;
        if (a.check) rs = wave_sum(rs);
        if (lane == 0) {
            ins += own_w;
            if (own_hit || a.sw) {
                if (FEAT)
                    top2_add(best, k2, vote_key(tie, own, own_w + a.sw));
                else
                    best = umax64(best, vote_key(tie, own, own_w + a.sw));
            }
            if (FEAT) {
                a.top1[v] = (uint32_t)(best >> 32);
                a.top2[v] = (uint32_t)(k2 >> 32);
            }
            const uint32_t nl = best ? key_label(tie, best) : own;
            a.L_new[v] = nl;
            wchg += nl != own;
            if (a.check && rs + a.sw > 0xFFFFFFFFull) atomicOr(a.err, ERR_WOVF);
        }
        wave_sync();
        }
        i = inext;
        v = nv;
        skip = nskip;
        keep = nkeep;
        b = nb;
        e = ne;
        valid = nvalid;
#pragma unroll
        for (int j = 0; j < A; ++j) {
            u[j] = nu[j];
            wt[j] = nwt[j];
        }
    }
    // the partials go through this wavefront's own table (no longer in use):
    // a separate LDS array would push a 1024-slot block past the 32 KB that
    // lets five blocks share a CU
    block_counts_at(T, SLOTS, lane == 0 ? wchg : 0, ins, a.changed, a.insum);
}

// Blocks of 256 threads of kernel K that one CU holds at once, as its
// registers and LDS allow (queried once per kernel).
template <auto K>
static unsigned resident_per_cu() {
    static const unsigned nb = [] {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, K, 256, 0) != hipSuccess || n < 1) n = 1;
        return (unsigned)n;
    }();
    return nb;
}

// Grid of a grid-stride launch of K over `units` work units, `per_block` per
// block: at most kStrideRounds whole rounds of the blocks that fit at once.
// Every block gets the same share, so a grid just above one round (5 blocks
// per CU where 4 fit) would leave most of the chip idle while its last
// blocks run.
constexpr unsigned kStrideRounds = 4;
template <auto K>
static unsigned stride_grid(uint64_t units, unsigned per_block, int num_cu) {
    return grid_for(units, per_block, resident_per_cu<K>() * (unsigned)(num_cu > 0 ? num_cu : 1) * kStrideRounds);
}

template <bool FEAT>
static void launch_thread_t(const RoundArgs &a, uint32_t lo, uint32_t cnt, int num_cu, hipStream_t s) {
    constexpr auto K = vote_thread_k<FEAT>;
    K<<<stride_grid<K>(cnt, 256, num_cu), 256, 0, s>>>(a, lo, cnt);
}
hipError_t launch_vote_thread(const RoundArgs &a, uint32_t lo, uint32_t cnt, int, int feat, int num_cu,
                              hipStream_t s) {
    if (cnt == 0) return hipSuccess;
    feat ? launch_thread_t<true>(a, lo, cnt, num_cu, s) : launch_thread_t<false>(a, lo, cnt, num_cu, s);
    return hipGetLastError();
}
template <bool FIRST, bool FEAT>
static void launch_group_t(const RoundArgs &a, uint32_t lo, uint32_t cnt, int num_cu, hipStream_t s) {
    constexpr int GL = kGroupLanes, GS = kGroupSlots;
    constexpr auto K = vote_group_k<GL, GS, FIRST, FEAT>;
    K<<<stride_grid<K>(cnt, 256 / GL, num_cu), 256, 0, s>>>(a, lo, cnt);
}
hipError_t launch_vote_group(const RoundArgs &a, uint32_t lo, uint32_t cnt, int first, int feat, int num_cu,
                             hipStream_t s) {
    if (cnt == 0) return hipSuccess;
    if (first)
        feat ? launch_group_t<true, true>(a, lo, cnt, num_cu, s) : launch_group_t<true, false>(a, lo, cnt, num_cu, s);
    else
        feat ? launch_group_t<false, true>(a, lo, cnt, num_cu, s)
             : launch_group_t<false, false>(a, lo, cnt, num_cu, s);
    return hipGetLastError();
}

// Rows of at most 128 arcs: after round 1 two rows per wavefront (32-lane
// groups, 4 arcs per lane, a 256-slot table each) -- 20 % faster than a
// wavefront per row, whose fixed per-row work is spread over too few arcs;
// round 1 keeps the wavefront kernel, which skips the rows the relabel pass
// already voted without loading them.
template <bool FIRST, bool FEAT>
static void launch_wave_t(const RoundArgs &a, uint32_t lo, uint32_t cnt, int wide, int num_cu, hipStream_t s) {
    constexpr int AS = kWaveArcsSmall / 64, AW = kWaveArcs / 64;
    static_assert(kWaveSlotsSmall / (2 * 32) * 32 == kWaveArcsSmall, "32-lane groups hold a whole row");
    constexpr auto KW = vote_wave_k<FIRST, FEAT, AW, kWaveSlots>;
    constexpr auto KS = vote_wave_k<FIRST, FEAT, AS, kWaveSlotsSmall>;
    constexpr auto KG = vote_group_k<32, kWaveSlotsSmall, FIRST, FEAT>;
    if (wide)
        KW<<<stride_grid<KW>(cnt, 4, num_cu), 256, 0, s>>>(a, lo, cnt);
    else if (FIRST)
        KS<<<stride_grid<KS>(cnt, 4, num_cu), 256, 0, s>>>(a, lo, cnt);
    else
        KG<<<stride_grid<KG>(cnt, 8, num_cu), 256, 0, s>>>(a, lo, cnt);
}

hipError_t launch_vote_wave(const RoundArgs &a, uint32_t lo, uint32_t cnt, int wide, int first, int feat,
                            int num_cu, hipStream_t s) {
    if (cnt == 0) return hipSuccess;
    if (first)
        feat ? launch_wave_t<true, true>(a, lo, cnt, wide, num_cu, s)
             : launch_wave_t<true, false>(a, lo, cnt, wide, num_cu, s);
    else
        feat ? launch_wave_t<false, true>(a, lo, cnt, wide, num_cu, s)
             : launch_wave_t<false, false>(a, lo, cnt, wide, num_cu, s);
    return hipGetLastError();
}

// ------------------------------------------------------------- long rows --
//
// A row longer than 512 arcs is split into 512-arc segments, one wavefront
// each.  Per round:
//   vote_hub_k     every segment tallies its labels in an LDS table and
//                  reports its kTopK heaviest (label, tally) pairs plus thr,
//                  the tally of its (kTopK+1)-th label: no label it did not
//                  report reaches more than thr in this segment.  Round 1
//                  rows that list each neighbour once report just their max
//                  key (every tally is one arc's weight).  HUB_BIG rows go
//                  straight to the slab merge below.
//   hub_merge_*    per row, lower bound LB(x) = reported tallies of x, upper
//                  bound UB(x) = LB(x) + sum of thr over the segments that
//                  did not report x, and any label nobody reported is below
//                  T = sum of all thr.  The leader x* (max key over LB and the
//                  row's exact own-label tally) is the exact winner when
//                  every other label's best possible key is below x*'s
//                  guaranteed key and T is below x*'s tally.  Otherwise the
//                  row is marked HUB_FALLBACK.
//   hub_fallback_k the segments of HUB_FALLBACK rows merge their exact
//                  tables in the row's global slab (open addressing, 2 x
//                  degree slots); hub_reduce_k takes the max over the slots
//                  they claimed; hub_final_k picks the winner of every row
//                  decided through best[] and resets the per-round state.

// Report the kTopK heaviest entries of a segment's listed table (clearing
// it) to cand[it * kTopK ...] and the (kTopK+1)-th tally to thr[it].  Keys are
// unique (one slot per label), so round k takes the largest key below the
// previous round's.  J = key columns per lane in use.
template <int J>
__device__ __forceinline__ void select_topk(const u64 (&keys)[kWaveArcs / 64], u64 &mine, uint32_t &thr) {
    const uint32_t lane = threadIdx.x & 63;
    u64 prev = ~0ull;
#pragma unroll 1
    for (int k = 0; k <= kTopK; ++k) {
        u64 lm = 0;
#pragma unroll
        for (int j = 0; j < J; ++j)
            if (keys[j] < prev) lm = umax64(lm, keys[j]);
        const u64 wm = wave_max64(lm);
        if (k == kTopK) {
            thr = (uint32_t)(wm >> 32);
            break;
        }
        if ((int)lane == k) mine = wm;
        if (wm == 0) break;
        prev = wm;
    }
}

__device__ __forceinline__ void report_topk(ListedTable &t, Tie tie, const HubState &hs, uint32_t it) {
    const uint32_t lane = threadIdx.x & 63;
    u64 keys[kWaveArcs / 64];
    const uint32_t J = listed_take(t, tie, keys);
    u64 mine = 0;
    uint32_t thr = 0;
    if (J == 1)
        select_topk<1>(keys, mine, thr);
    else if (J == 2)
        select_topk<2>(keys, mine, thr);
    else if (J != 0 && J <= 4)
        select_topk<4>(keys, mine, thr);
    else if (J != 0)
        select_topk<kWaveArcs / 64>(keys, mine, thr);
    if (lane == 0) hs.thr[it] = thr;
    if (lane < (uint32_t)kTopK)
        hs.cand[(u64)it * kTopK + lane] = mine ? (((u64)key_label(tie, mine) << 32) | (mine >> 32)) : EMPTY_SLOT;
}

// Round 1 rows that list each neighbour once: every tally is one arc's
// weight, so a segment only needs its max key (no table, no LDS).  Rows
// with HUB_REPEATS are left to vote_hub_k.
__global__ __launch_bounds__(256) void vote_hub_direct_k(RoundArgs a, const HubItem *__restrict__ items,
                                                         uint32_t count, HubState hs) {
    constexpr int A = kWaveArcs / 64;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (uint32_t it = blockIdx.x * 4 + wave; it < count; it += gridDim.x * 4) {
        const HubItem item = items[it];
        const uint32_t h = item.r;
        if (hs.flags[h] & HUB_REPEATS) continue;  // uniform over the wavefront
        const RowMode rm = row_mode(a, h);
        if (!rm.on) continue;  // the other half: hub_final_k copies its label
        uint32_t u[A], wt[A], valid = 0, lab[A];
        load_arcs<A, 64>(a, item.b0 + lane, item.b1, u, wt, valid);
        gather_labels<A>(a, u, valid, lab);
        const uint32_t own = a.L_old[h];
        u64 own_w = 0, rs = 0;
        uint32_t own_hit = 0, rem = 0;
        split_own<A>(lab, wt, valid, own, own_w, own_hit, rem, rs);
        u64 best = 0;
#pragma unroll
        for (int j = 0; j < A; ++j)
            if (rem >> j & 1u) best = umax64(best, vote_key(rm.tie, lab[j], wt[j]));
        best = wave_max64(best);
        own_w = wave_sum(own_w);
        own_hit = __ballot(own_hit != 0) != 0;
        rs = wave_sum(rs);
        if (lane == 0) {
            if (best) atomicMax(&hs.best[h], best);
            if (own_w) atomicAdd(&hs.own_sum[h], own_w);
            if (own_hit) atomicOr(&hs.flags[h], HUB_OWN_SEEN);
            if (a.check) atomicAdd(&hs.rowsum[h], rs);
        }
    }
}

// Every other round (and round-1 rows with HUB_REPEATS): one LDS table per
// wavefront and segment, reported as top-K, or merged into the slab for
// HUB_BIG rows.  A segment whose table would pass kHubSpill distinct labels
// marks its row HUB_FALLBACK (the merge then skips the row and the slab pass
// counts it exactly); HUB_BIG rows flush a full table and go on.  Three
// segments are in flight per wavefront: the arcs of the one after next load
// and the labels of the next one are gathered while the current one is
// tallied.
// Arc loads of one lane of a long-row segment: columns, and weights only
// for weighted graphs (W); unit weights are the `valid` bits.
template <int A, bool W>
__device__ __forceinline__ void issue_hub_arcs(const RoundArgs &a, uint64_t k0, uint64_t e, uint32_t (&u)[A],
                                               uint32_t (&wt)[W ? A : 1], uint32_t &valid) {
    valid = 0;
#pragma unroll
    for (int j = 0; j < A; ++j) {
        const uint64_t k = k0 + (uint64_t)j * 64;
        const bool in = k < e;
        valid |= (uint32_t)in << j;
        const uint32_t x = a.g.col[in ? k : 0];  // branch-free, as issue_arcs
        u[j] = in ? x : 0u;
    }
    if (W) {
#pragma unroll
        for (int j = 0; j < (W ? A : 1); ++j) {
            const uint64_t k = k0 + (uint64_t)j * 64;
            const uint32_t x = a.g.w[(valid >> j & 1u) ? k : 0];
            wt[j] = (valid >> j & 1u) ? x : 0u;
        }
    } else {
        wt[0] = 0;
    }
}

template <bool FIRST, bool W>
__global__ __launch_bounds__(256) void vote_hub_k(RoundArgs a, const HubItem *__restrict__ items, uint32_t count,
                                                  HubState hs) {
    constexpr int A = kWaveArcs / 64;
    // round 1 after the relabel pass: only rows flagged HUB_REPEATS need a
    // table, and usually there are none
    if (FIRST && a.skip_distinct && __hip_atomic_load(hs.repeats, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
        return;
    __shared__ u64 table[4 * kHubSlots];
    __shared__ uint16_t lists[4 * kHubSlots];
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    ListedTable t{table + wave * kHubSlots, lists + wave * kHubSlots, 0, 0};
    for (uint32_t s = lane; s < (uint32_t)kHubSlots; s += 64) t.T[s] = EMPTY_SLOT;
    wave_sync();
    const uint32_t stride = gridDim.x * 4;
    // stage 0: the current segment (labels in flight); stage 1: the next
    // segment (arcs in flight)
    // Every stage issues its loads unconditionally (an item past the end or
    // skipped in round 1 is an empty segment of row 0), so the compiler can
    // wait for exactly the stage it needs.
    // The row's flags travel in the item's spare word, read when the item is
    // fetched, so no load of the current stage is issued behind the others.
    auto fetch = [&](uint32_t k, bool &act_k) {
        HubItem x{0, 0, 0, 0};
        act_k = false;
        if (k < count) {
            x = items[k];
            x.pad = hs.flags[x.r];
            act_k = !FIRST || (x.pad & HUB_REPEATS);
            // the other half of a semi-synchronous round: hub_final_k copies
            if (act_k && a.half && !row_mode(a, x.r).on) act_k = false;
            if (!act_k) x = HubItem{0, 0, 0, 0};
        }
        return x;
    };
    uint32_t it = blockIdx.x * 4 + wave;
    bool act, nact;
    HubItem item = fetch(it, act), nitem = fetch(it + stride, nact);
    uint32_t lab[A], wt[W ? A : 1], valid = 0, own = 0;
    uint32_t nu[A], nwt[W ? A : 1], nvalid = 0;
    issue_hub_arcs<A, W>(a, item.b0 + lane, item.b1, lab, wt, valid);
    check_arcs<A>(a, lab);
    gather_labels<A>(a, lab, valid, lab);
    own = a.L_old[item.r];
    issue_hub_arcs<A, W>(a, nitem.b0 + lane, nitem.b1, nu, nwt, nvalid);
    while (it < count) {
        // stage 2: arcs of the segment after next
        bool act2;
        const HubItem item2 = fetch(it + 2 * stride, act2);
        uint32_t u2[A], wt2[W ? A : 1], valid2 = 0;
        issue_hub_arcs<A, W>(a, item2.b0 + lane, item2.b1, u2, wt2, valid2);
        // stage 1 -> labels of the next segment
        check_arcs<A>(a, nu);
        gather_labels<A>(a, nu, nvalid, nu);
        const uint32_t nown = a.L_old[nitem.r];
        if (act) {
            const uint32_t h = item.r;
            const uint32_t flags = item.pad;
            uint32_t w[A];
#pragma unroll
            for (int j = 0; j < A; ++j) w[j] = W ? wt[j < (W ? A : 1) ? j : 0] : (valid >> j & 1u);
            u64 own_w = 0, rs = 0;
            uint32_t own_hit = 0, rem = 0;
            split_own<A>(lab, w, valid, own, own_w, own_hit, rem, rs);
            uint32_t S = next_pow2(2u * (uint32_t)(item.b1 - item.b0));
            S = S < 64u ? 64u : (S > (uint32_t)kHubSlots ? (uint32_t)kHubSlots : S);
            t.mask = S - 1;
            if (flags & HUB_BIG) {
                bool flushed = false;
                rem = listed_tally<A>(t, lab, w, rem, kHubSpill);
                for (;;) {
                    wave_sync();
                    if (t.n) {
                        flush_listed_to_slab(t, hs, h);
                        flushed = true;
                        wave_sync();
                    }
                    if (!__ballot(rem != 0)) break;
                    rem = listed_tally<A>(t, lab, w, rem, kHubSpill);
                }
                if (lane == 0 && flushed) atomicOr(hs.pending, 1u);
            } else {
                const bool any = __ballot(rem != 0) != 0;
                bool spilled = false;
                if (any) {
                    rem = listed_tally<A>(t, lab, w, rem, kHubSpill);
                    spilled = __ballot(rem != 0) != 0;
                    wave_sync();
                }
                if (spilled) {
                    listed_clear(t);
                    if (lane == 0) {
                        atomicOr(&hs.flags[h], HUB_FALLBACK);
                        atomicOr(hs.pending, 1u);
                    }
                } else {
                    report_topk(t, row_mode(a, h).tie, hs, it);
                }
            }
            own_w = wave_sum(own_w);
            own_hit = __ballot(own_hit != 0) != 0;
            if (a.check) rs = wave_sum(rs);
            if (lane == 0) {
                if (own_w) atomicAdd(&hs.own_sum[h], own_w);
                if (own_hit) atomicOr(&hs.flags[h], HUB_OWN_SEEN);
                if (a.check) atomicAdd(&hs.rowsum[h], rs);
            }
            wave_sync();
        }
        it += stride;
        item = nitem;
        act = nact;
        own = nown;
        valid = nvalid;
        nitem = item2;
        nact = act2;
        nvalid = valid2;
#pragma unroll
        for (int j = 0; j < A; ++j) {
            lab[j] = nu[j];
            nu[j] = u2[j];
        }
#pragma unroll
        for (int j = 0; j < (W ? A : 1); ++j) {
            wt[j] = nwt[j];
            nwt[j] = wt2[j];
        }
    }
}

// Second pass over the segments of rows the merge could not decide: exact
// tables merged through the slab (own-label tallies are already counted).
__global__ __launch_bounds__(256) void hub_fallback_k(RoundArgs a, const HubItem *__restrict__ items,
                                                      uint32_t count, HubState hs) {
    if (!*hs.pending) return;  // no row fell back this round
    constexpr int A = kWaveArcs / 64;
    __shared__ u64 table[4 * kWaveSlots];
    __shared__ uint16_t lists[4 * kWaveArcs];
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    ListedTable t{table + wave * kWaveSlots, lists + wave * kWaveArcs, 0, 0};
    for (uint32_t s = lane; s < kWaveSlots; s += 64) t.T[s] = EMPTY_SLOT;
    wave_sync();
    // The wavefront's items are wid, wid + stride, ...; their rows' flags are
    // read 64 items at a time (one per lane), so the few segments of rows that
    // fell back are found without a dependent load chain per item.
    const uint64_t wid = blockIdx.x * 4 + wave, stride = gridDim.x * 4;
    for (uint64_t j0 = 0; wid + j0 * stride < count; j0 += 64) {
        const uint64_t i = wid + (j0 + lane) * stride;
        bool fb = false;
        if (i < count) fb = (hs.flags[items[i].r] & HUB_FALLBACK) != 0;
        for (u64 m = __ballot(fb); m; m &= m - 1) {
            const HubItem item = items[wid + (j0 + (uint64_t)__builtin_ctzll(m)) * stride];
            const uint32_t h = item.r;
            const uint32_t own = a.L_old[h];
            uint32_t u[A], lab[A], wt[A];
            uint32_t valid = 0;
            load_arcs<A, 64>(a, item.b0 + lane, item.b1, u, wt, valid);
            gather_labels<A>(a, u, valid, lab);
            u64 own_w = 0, rs = 0;
            uint32_t own_hit = 0, rem = 0;
            split_own<A>(lab, wt, valid, own, own_w, own_hit, rem, rs);
            uint32_t S = next_pow2(2u * (uint32_t)(item.b1 - item.b0));
            S = S < 64u ? 64u : (S > (uint32_t)kWaveSlots ? (uint32_t)kWaveSlots : S);
            t.mask = S - 1;
            listed_tally<A>(t, lab, wt, rem);
            wave_sync();
            flush_listed_to_slab(t, hs, h);
            wave_sync();
        }
    }
}

// Add one report (label, tally, its segment's thr) to a merge table of
// mask+1 slots: keys, lower bounds LB and sums of reporting segments' thr.
__device__ __forceinline__ void merge_insert(uint32_t *mk, uint32_t *mlb, uint32_t *mtr, uint32_t mask, uint32_t lab,
                                             uint32_t c, uint32_t t) {
    uint32_t h = hmix(lab) & mask;
    for (;;) {
        const uint32_t prev = atomicCAS(&mk[h], kNone, lab);
        if (prev == kNone || prev == lab) {
            atomicAdd(&mlb[h], c);
            atomicAdd(&mtr[h], t);
            return;
        }
        h = (h + 1) & mask;
    }
}

// One wavefront per row of at most kMergeWaveSegs segments.
__global__ __launch_bounds__(256) void hub_merge_wave_k(RoundArgs a, HubState hs, const uint32_t *__restrict__ rows,
                                                        uint32_t count, int first) {
    constexpr uint32_t MS = 2 * kMergeWaveSegs * kTopK;  // at most half full
    __shared__ uint32_t mkey[4][MS], mlb[4][MS], mtr[4][MS];
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    uint32_t *mk = mkey[wave], *lb = mlb[wave], *tr = mtr[wave];
    for (uint32_t s = lane; s < MS; s += 64) {
        mk[s] = kNone;
        lb[s] = 0;
        tr[s] = 0;
    }
    wave_sync();
    u64 wchg = 0;
    // The wavefront's rows are rows[wid], rows[wid + stride], ...; 64 of them
    // are looked up at once (one per lane: row, flags, segment range, own
    // label and tally), then merged one after the other.
    const uint64_t wid = blockIdx.x * 4 + wave, stride = gridDim.x * 4;
    for (uint64_t j0 = 0; wid + j0 * stride < count; j0 += 64) {
        const uint64_t ii = wid + (j0 + lane) * stride;
        uint32_t hl = 0, fl = 0, lol = 0, nsl = 0, ownl = 0;
        u64 osl = 0;
        bool go = false;
        if (ii < count) {
            hl = rows[ii];
            fl = hs.flags[hl];
            // rows decided through best[] in round 1, rows whose segment
            // spilled (slab pass), and the other half of a semi-synchronous
            // round (hub_final_k copies its label) are not merged here
            go = !(first && !(fl & HUB_REPEATS)) && !(fl & HUB_FALLBACK) && row_mode(a, hl).on;
            if (go) {
                lol = hs.item_lo[hl];
                nsl = hs.item_lo[hl + 1] - lol;
                ownl = a.L_old[hl];
                osl = hs.own_sum[hl];
            }
        }
        // the reports of a row: its segments' thr (one per lane) and up to
        // 2 * 64 candidates with their segments' thr; the next row's are
        // requested before the current one is merged
        constexpr int CQ = kMergeWaveSegs * kTopK / 64;
        static_assert(CQ * 64 == kMergeWaveSegs * kTopK, "candidates per lane");
        auto fetch_row = [&](int l, uint32_t &th, u64 (&cx)[CQ], uint32_t (&ct)[CQ]) {
            const uint32_t lo = __builtin_amdgcn_readlane(lol, l), ns = __builtin_amdgcn_readlane(nsl, l);
            th = lane < ns ? hs.thr[lo + lane] : 0u;
#pragma unroll
            for (int q = 0; q < CQ; ++q) {
                const uint32_t e = lane + 64u * q;
                const bool in = e < ns * kTopK;
                cx[q] = in ? hs.cand[(u64)lo * kTopK + e] : EMPTY_SLOT;
                ct[q] = in ? hs.thr[lo + e / kTopK] : 0u;
            }
        };
        u64 m = __ballot(go);
        uint32_t th = 0, ct[CQ];
        u64 cx[CQ];
        if (m) fetch_row((int)__builtin_ctzll(m), th, cx, ct);
        for (; m; m &= m - 1) {
            const int l = (int)__builtin_ctzll(m);
            const uint32_t h = __builtin_amdgcn_readlane(hl, l);
            const uint32_t flags = __builtin_amdgcn_readlane(fl, l);
            const uint32_t own = __builtin_amdgcn_readlane(ownl, l);
            const u64 own_sum = ((u64)__builtin_amdgcn_readlane((uint32_t)(osl >> 32), l) << 32) |
                                __builtin_amdgcn_readlane((uint32_t)osl, l);
            const Tie tie = row_mode(a, h).tie;
            const uint32_t cth = th;
            u64 ccx[CQ];
            uint32_t cct[CQ];
#pragma unroll
            for (int q = 0; q < CQ; ++q) {
                ccx[q] = cx[q];
                cct[q] = ct[q];
            }
            const u64 rest = m & (m - 1);
            if (rest) fetch_row((int)__builtin_ctzll(rest), th, cx, ct);
            const u64 T = wave_sum((u64)cth);
#pragma unroll
            for (int q = 0; q < CQ; ++q)
                if (ccx[q] != EMPTY_SLOT) merge_insert(mk, lb, tr, MS - 1, (uint32_t)(ccx[q] >> 32), (uint32_t)ccx[q], cct[q]);
            wave_sync();
            u64 xkey = ((flags & HUB_OWN_SEEN) || a.sw) ? vote_key(tie, own, own_sum + a.sw) : 0ull;
            for (uint32_t s = lane; s < MS; s += 64)
                if (mk[s] != kNone) xkey = umax64(xkey, vote_key(tie, mk[s], lb[s]));
            xkey = wave_max64(xkey);
            const uint32_t xs = key_label(tie, xkey);
            const u64 V = xkey >> 32;
            bool bad = false;
            for (uint32_t s = lane; s < MS; s += 64) {
                const uint32_t lab = mk[s];
                if (lab != kNone) {
                    if (lab != xs && vote_key(tie, lab, (u64)lb[s] + T - tr[s]) >= xkey) bad = true;
                    mk[s] = kNone;
                    lb[s] = 0;
                    tr[s] = 0;
                }
            }
            bad |= (T > 0 && T >= V);
            const bool decided = __ballot(bad) == 0;
            if (lane == 0) {
                if (decided) {
                    const uint32_t nl = xkey ? xs : own;
                    a.L_new[h] = nl;
                    wchg += nl != own;
                } else {
                    atomicOr(&hs.flags[h], HUB_FALLBACK);
                    atomicOr(hs.pending, 1u);
                }
            }
            wave_sync();
        }
    }
    block_count(lane == 0 ? wchg : 0, a.changed);
}

// One 256-thread block per row of kMergeWaveSegs+1 .. kMergeBlockSegs segments.
__global__ __launch_bounds__(256) void hub_merge_block_k(RoundArgs a, HubState hs, const uint32_t *__restrict__ rows,
                                                         uint32_t count, int first) {
    constexpr uint32_t MS = kMergeBlockSlots;
    __shared__ uint32_t mk[MS], lb[MS], tr[MS];
    __shared__ BlockRed R;
    for (uint32_t s = threadIdx.x; s < MS; s += 256) {
        mk[s] = kNone;
        lb[s] = 0;
        tr[s] = 0;
    }
    __syncthreads();
    u64 bchg = 0;
    for (uint32_t i = blockIdx.x; i < count; i += gridDim.x) {
        const uint32_t h = rows[i];
        const uint32_t flags = hs.flags[h];
        if (first && !(flags & HUB_REPEATS)) continue;  // uniform over the block
        if (flags & HUB_FALLBACK) continue;              // a segment spilled: slab pass
        const RowMode rm = row_mode(a, h);
        if (!rm.on) continue;  // the other half: hub_final_k copies its label
        const Tie tie = rm.tie;
        const uint32_t lo = hs.item_lo[h], ns = hs.item_lo[h + 1] - lo;
        u64 T = 0, z1 = 0, z2 = 0;
        uint32_t zo = 0;
        for (uint32_t sgi = threadIdx.x; sgi < ns; sgi += 256) T += hs.thr[lo + sgi];
        for (uint32_t e = threadIdx.x; e < ns * kTopK; e += 256) {
            const u64 x = hs.cand[(u64)lo * kTopK + e];
            if (x != EMPTY_SLOT) merge_insert(mk, lb, tr, MS - 1, (uint32_t)(x >> 32), (uint32_t)x, hs.thr[lo + e / kTopK]);
        }
        block_reduce(R, z1, T, z2, zo);  // T summed, includes a barrier
        const uint32_t own = a.L_old[h];
        u64 xkey = ((flags & HUB_OWN_SEEN) || a.sw) ? vote_key(tie, own, hs.own_sum[h] + a.sw) : 0ull;
        for (uint32_t s = threadIdx.x; s < MS; s += 256)
            if (mk[s] != kNone) xkey = umax64(xkey, vote_key(tie, mk[s], lb[s]));
        __syncthreads();
        u64 z3 = 0, z4 = 0;
        block_reduce(R, xkey, z3, z4, zo);
        const uint32_t xs = key_label(tie, xkey);
        const u64 V = xkey >> 32;
        uint32_t bad = 0;
        for (uint32_t s = threadIdx.x; s < MS; s += 256) {
            const uint32_t lab = mk[s];
            if (lab != kNone) {
                if (lab != xs && vote_key(tie, lab, (u64)lb[s] + T - tr[s]) >= xkey) bad = 1;
                mk[s] = kNone;
                lb[s] = 0;
                tr[s] = 0;
            }
        }
        bad |= (T > 0 && T >= V) ? 1u : 0u;
        bad = __syncthreads_or((int)bad);
        if (threadIdx.x == 0) {
            if (!bad) {
                const uint32_t nl = xkey ? xs : own;
                a.L_new[h] = nl;
                bchg += nl != own;
            } else {
                atomicOr(&hs.flags[h], HUB_FALLBACK);
                atomicOr(hs.pending, 1u);
            }
        }
        __syncthreads();
    }
    block_count(threadIdx.x == 0 ? bchg : 0, a.changed);
}

// Phase 2: max key over the slab slots claimed by a row, clearing them for
// the next round.  One block per item of <= 2048 touched-list positions.
__global__ __launch_bounds__(256) void hub_reduce_k(RoundArgs a, HubState hs, const ReduceItem *__restrict__ items,
                                                    uint32_t count) {
    __shared__ BlockRed R;
    __shared__ uint32_t act[256];
    __shared__ uint32_t nact;
    if (!*hs.pending) return;  // no slab was used this round
    // The block's items are blockIdx.x, + gridDim.x, ...; 256 of them are
    // checked at once (one per thread) and only those whose row claimed slots
    // in their range are reduced, so skipped items cost no dependent loads.
    for (uint64_t k0 = 0; blockIdx.x + k0 * gridDim.x < count; k0 += 256) {
        __syncthreads();  // every thread has read the previous batch's count
        if (threadIdx.x == 0) nact = 0;
        __syncthreads();
        const uint64_t i = blockIdx.x + (k0 + threadIdx.x) * gridDim.x;
        if (i < count) {
            const ReduceItem r = items[i];
            if (r.t0 < min(r.t1, hs.tcount[r.hub])) act[atomicAdd(&nact, 1u)] = (uint32_t)i;
        }
        __syncthreads();
        const uint32_t na = nact;
        for (uint32_t q = 0; q < na; ++q) {
            const ReduceItem r = items[act[q]];
            const uint32_t t1 = min(r.t1, hs.tcount[r.hub]);
            u64 *slab = hs.slab + hs.slab_off[r.hub];
            const uint32_t *tlist = hs.touched + hs.touched_off[r.hub];
            const Tie tie = row_mode(a, r.hub).tie;  // rows of the other half claimed no slot
            u64 best = 0, z0 = 0, z1 = 0;
            uint32_t z2 = 0;
            for (uint32_t p = r.t0 + threadIdx.x; p < t1; p += 256) {
                const uint32_t s = tlist[p];
                if (s != kNone) {
                    best = umax64(best, slot_key(tie, slab[s]));
                    slab[s] = EMPTY_SLOT;
                }
            }
            block_reduce(R, best, z0, z1, z2);
            if (threadIdx.x == 0 && best) atomicMax(&hs.best[r.hub], best);
            __syncthreads();
        }
    }
}

// Phase 3: one lane per long row.  Rows decided through best[] (round-1
// direct rows, HUB_BIG rows, HUB_FALLBACK rows) pick their winner here; every
// row's per-round state is reset.
__global__ __launch_bounds__(256) void hub_final_k(RoundArgs a, HubState hs, uint32_t count, int first) {
    const uint32_t lane = threadIdx.x & 63;
    u64 wchg = 0, ins = 0;
    for (uint32_t base = blockIdx.x * 256 + (threadIdx.x & ~63u); base < count; base += gridDim.x * 256) {
        const uint32_t i = base + lane;
        bool ch = false;
        if (i < count) {
            const uint32_t f = hs.flags[i];
            ins += hs.own_sum[i];
            const RowMode rm = row_mode(a, i);
            const bool via_best = (first && !(f & HUB_REPEATS)) || (f & (HUB_BIG | HUB_FALLBACK));
            if (!rm.on) {
                a.L_new[i] = a.L_old[i];  // the other half of a semi-synchronous round
            } else if (via_best) {
                const uint32_t own = a.L_old[i];
                u64 best = hs.best[i];
                if ((f & HUB_OWN_SEEN) || a.sw) best = umax64(best, vote_key(rm.tie, own, hs.own_sum[i] + a.sw));
                const uint32_t nl = best ? key_label(rm.tie, best) : own;
                a.L_new[i] = nl;
                ch = nl != own;
            }
            if (a.check && hs.rowsum[i] + a.sw > 0xFFFFFFFFull) atomicOr(a.err, ERR_WOVF);
            hs.best[i] = 0;
            hs.own_sum[i] = 0;
            hs.flags[i] = f & (HUB_REPEATS | HUB_BIG);
            hs.tcount[i] = 0;
            hs.rowsum[i] = 0;
        }
        wchg += __popcll(__ballot(ch));
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *hs.pending = 0;
    block_counts(lane == 0 ? wchg : 0, ins, a.changed, a.insum);
}

template <bool FIRST, bool W>
static void launch_hub_t(const RoundArgs &a, const HubItem *items, uint32_t count, const HubState &hs, int num_cu,
                         hipStream_t s) {
    constexpr auto K = vote_hub_k<FIRST, W>;
    K<<<stride_grid<K>(count, 4, num_cu), 256, 0, s>>>(a, items, count, hs);
}
hipError_t launch_vote_hub(const RoundArgs &a, const HubItem *items, uint32_t count, const HubState &hs,
                           int first, int fused, int num_cu, hipStream_t s) {
    if (count == 0) return hipSuccess;
    const bool w = a.g.w != nullptr;
    if (first) {
        // fused: the relabel pass already gathered the direct rows' partials
        if (!fused)
            vote_hub_direct_k<<<stride_grid<vote_hub_direct_k>(count, 4, num_cu), 256, 0, s>>>(a, items, count, hs);
        w ? launch_hub_t<true, true>(a, items, count, hs, num_cu, s)
          : launch_hub_t<true, false>(a, items, count, hs, num_cu, s);
    } else {
        w ? launch_hub_t<false, true>(a, items, count, hs, num_cu, s)
          : launch_hub_t<false, false>(a, items, count, hs, num_cu, s);
    }
    return hipGetLastError();
}
hipError_t launch_hub_merge(const RoundArgs &a, const HubState &hs, const uint32_t *rows, uint32_t count,
                            int per_block, int first, hipStream_t s) {
    if (count == 0) return hipSuccess;
    if (per_block)
        hub_merge_block_k<<<grid_for(count, 1, 512), 256, 0, s>>>(a, hs, rows, count, first);
    else
        hub_merge_wave_k<<<grid_for(count, 4, 2048), 256, 0, s>>>(a, hs, rows, count, first);
    return hipGetLastError();
}
hipError_t launch_hub_fallback(const RoundArgs &a, const HubItem *items, uint32_t count, const HubState &hs,
                               int num_cu, hipStream_t s) {
    if (count == 0) return hipSuccess;
    hub_fallback_k<<<stride_grid<hub_fallback_k>(count, 4, num_cu), 256, 0, s>>>(a, items, count, hs);
    return hipGetLastError();
}
hipError_t launch_hub_reduce(const RoundArgs &a, const HubState &hs, const ReduceItem *items, uint32_t count,
                             hipStream_t s) {
    if (count == 0) return hipSuccess;
    hub_reduce_k<<<grid_for(count, 1, 4096), 256, 0, s>>>(a, hs, items, count);
    return hipGetLastError();
}
hipError_t launch_hub_final(const RoundArgs &a, const HubState &hs, uint32_t count, int first, hipStream_t s) {
    if (count == 0) return hipSuccess;
    hub_final_k<<<grid_for(count, 256, 1024), 256, 0, s>>>(a, hs, count, first);
    return hipGetLastError();
}

}  // namespace lpa
