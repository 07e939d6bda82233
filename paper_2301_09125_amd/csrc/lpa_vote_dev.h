// lpa_vote_dev.h -- device building blocks of a vote shared by the per-round
// kernels (lpa_vote.hip) and the persistent batch kernel (lpa_batch.hip):
// arc loading, label gathering, own-label tally, wavefront pre-aggregation
// (the batch kernel's), LDS tables and the global slab used to merge the
// tallies of long rows.
#pragma once

#include "lpa_device.h"

namespace lpa {

// Row of work item i of a launch over [lo, lo + cnt) or over a list.
__device__ __forceinline__ uint32_t row_of(const RoundArgs &a, uint32_t lo, uint32_t i) {
    return a.list ? a.list[i] : lo + i;
}

// Whether internal row v votes in this launch, and its tie rule.  The draws
// of a vertex in round t are SplitMix64 outputs number 2c + 1 (the top bit
// gives its half of a semi-synchronous round) and 2c + 2 (its tie key) for
// c = t * 2^32 + (original id of v).
struct RowMode {
    bool on;
    Tie tie;
};
__device__ __forceinline__ RowMode row_mode(const RoundArgs &a, uint32_t v) {
    RowMode m{true, Tie{a.tie, 0u}};
    if (a.half | a.tie) {
        const u64 c = (((u64)a.t << 32) | a.orig[v]) << 1;
        if (a.half) m.on = (uint32_t)(splitmix64_at(a.seed, c) >> 63) == a.half - 1;
        if (a.tie) m.tie.k = (uint32_t)splitmix64_at(a.seed, c | 1u);
    }
    return m;
}

// Two largest distinct vote keys seen so far (0 = none).  Selects only: a
// branchy form gets the pair spilled to scratch memory and indexed.
__device__ __forceinline__ void top2_add(u64 &k1, u64 &k2, u64 k) {
    const bool above = k > k1;
    const bool between = k < k1 && k > k2;
    const u64 n2 = above ? k1 : (between ? k : k2);
    k1 = above ? k : k1;
    k2 = n2;
}

// Merge the top-two pairs of lanes that are `off` apart (xor pattern).
__device__ __forceinline__ void top2_xor(u64 &k1, u64 &k2, int off) {
    const u64 o1 = __shfl_xor(k1, off, 64), o2 = __shfl_xor(k2, off, 64);
    top2_add(k1, k2, o1);
    top2_add(k1, k2, o2);
}

// Issue the loads of arcs k0 + j*STRIDE (j < A, below e) of one lane:
// internal ids into u, weights into wt, bit j of `valid` set for loaded
// arcs.  Nothing here waits for the data, so the loads of the next work item
// can be in flight while the current one is processed.  Every lane issues
// every load (arcs past the row read arc 0, which exists whenever a vote
// kernel runs, and are masked through `valid`): loads behind per-lane
// branches leave the compiler unable to count the loads in flight, and it
// then waits for all of them, prefetches included.
template <int A, int STRIDE>
__device__ __forceinline__ void issue_arcs(const RoundArgs &a, uint64_t k0, uint64_t e, uint32_t (&u)[A],
                                           uint32_t (&wt)[A], uint32_t &valid) {
    const uint32_t *__restrict__ col = a.g.col;
    const uint32_t *__restrict__ w = a.g.w;
    valid = 0;
#pragma unroll
    for (int j = 0; j < A; ++j) {
        const uint64_t k = k0 + (uint64_t)j * STRIDE;
        const bool in = k < e;
        valid |= (uint32_t)in << j;
        const uint32_t x = col[in ? k : 0];
        u[j] = in ? x : 0u;
    }
    if (w) {
#pragma unroll
        for (int j = 0; j < A; ++j) {
            const uint64_t k = k0 + (uint64_t)j * STRIDE;
            const uint32_t x = w[(valid >> j & 1u) ? k : 0];
            wt[j] = (valid >> j & 1u) ? x : 0u;
        }
    } else {
#pragma unroll
        for (int j = 0; j < A; ++j) wt[j] = (valid >> j) & 1u;
    }
}

// Out-of-range ids raise ERR_COL once and are read as vertex 0, so no later
// access leaves the arrays.
template <int A>
__device__ __forceinline__ void check_arcs(const RoundArgs &a, uint32_t (&u)[A]) {
    bool bad = false;
#pragma unroll
    for (int j = 0; j < A; ++j) {
        bad |= u[j] >= a.g.n;
        u[j] = u[j] >= a.g.n ? 0u : u[j];
    }
    if (bad) atomicOr(a.err, ERR_COL);
}

template <int A, int STRIDE>
__device__ __forceinline__ void load_arcs(const RoundArgs &a, uint64_t k0, uint64_t e, uint32_t (&u)[A],
                                          uint32_t (&wt)[A], uint32_t &valid) {
    issue_arcs<A, STRIDE>(a, k0, e, u, wt, valid);
    check_arcs<A>(a, u);
}

template <int A>
__device__ __forceinline__ void gather_labels(const RoundArgs &a, const uint32_t (&u)[A], uint32_t valid,
                                              uint32_t (&lab)[A]) {
    const uint32_t *__restrict__ L = a.L_old;
#pragma unroll
    for (int j = 0; j < A; ++j) {
        const uint32_t x = L[u[j]];  // u = 0 past the row: no branch (see issue_arcs)
        lab[j] = (valid >> j & 1u) ? x : 0xFFFFFFFFu;
    }
}

// Split loaded arcs into the own-label tally and the bit set `rem` of arcs
// whose label must go through a table.
template <int A>
__device__ __forceinline__ void split_own(const uint32_t (&lab)[A], const uint32_t (&wt)[A], uint32_t valid,
                                          uint32_t own, u64 &own_w, uint32_t &own_hit, uint32_t &rem, u64 &rs) {
#pragma unroll
    for (int j = 0; j < A; ++j)
        if (valid >> j & 1u) {
            rs += wt[j];
            if (lab[j] == own) {
                own_w += wt[j];
                own_hit = 1;
            } else {
                rem |= 1u << j;
            }
        }
}

// Wavefront pre-aggregation: up to NPEEL times, take the first remaining
// label of the lowest lane that has one, sum the weights of every remaining
// arc of the wavefront with that label and insert the sum once.  All 64
// lanes call this together.
template <int A, int NPEEL>
__device__ __forceinline__ void wave_peel(u64 *T, uint32_t mask, const uint32_t (&lab)[A],
                                          const uint32_t (&wt)[A], uint32_t &rem) {
    const uint32_t lane = threadIdx.x & 63;
#pragma unroll
    for (int p = 0; p < NPEEL; ++p) {
        const u64 m = __ballot(rem != 0);
        if (!m) return;
        const int lead = __ffsll((long long)m) - 1;
        uint32_t mine = 0;
#pragma unroll
        for (int j = A - 1; j >= 0; --j)
            if (rem >> j & 1u) mine = lab[j];
        const uint32_t L = (uint32_t)__builtin_amdgcn_readlane((int)mine, lead);
        uint32_t s = 0;
#pragma unroll
        for (int j = 0; j < A; ++j)
            if ((rem >> j & 1u) && lab[j] == L) {
                s += wt[j];
                rem &= ~(1u << j);
            }
        s = wave_sum(s);
        if ((int)lane == lead) lds_insert(T, mask, L, s);
    }
}

// Number of lanes below this one whose bit is set in m.
__device__ __forceinline__ uint32_t lanes_below(u64 m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// A wavefront's LDS hashtable together with the list of the slots it has
// claimed, in claim order, so that reading and clearing the table costs the
// number of distinct labels in it instead of its number of slots.  `n` holds
// the same value in every lane.
struct ListedTable {
    u64 *T;
    uint16_t *lst;
    uint32_t mask;
    uint32_t n;
};

// Insert (lab, wv) for every lane whose `go` is set.  All 64 lanes call this
// together: the probe loop runs until no lane has a pair left, so the claim
// count advances in step in every lane.  The caller guarantees more slots
// than distinct labels.
__device__ __forceinline__ void listed_insert(ListedTable &t, bool go, uint32_t lab, uint32_t wv) {
    uint32_t h = hmix(lab) & t.mask;
    const u64 desired = ((u64)lab << 32) | wv;
    while (__ballot(go)) {
        bool claimed = false;
        if (go) {
            const u64 prev = atomicCAS(&t.T[h], EMPTY_SLOT, desired);
            if (prev == EMPTY_SLOT) {
                claimed = true;
                go = false;
            } else if ((uint32_t)(prev >> 32) == lab) {
                atomicAdd(&t.T[h], (u64)wv);
                go = false;
            } else {
                h = (h + 1) & t.mask;
            }
        }
        const u64 m = __ballot(claimed);
        if (claimed) t.lst[t.n + lanes_below(m)] = (uint16_t)h;
        t.n += (uint32_t)__popcll(m);
    }
}

// Insert the arcs of `rem`, one column j at a time, stopping once the table
// holds more than `cap` labels.  Returns the bits of `rem` not inserted (0
// when everything went in).  Each step claims at most 64 slots, so a table of
// at least cap + 65 slots never fills up.  (Summing the most frequent label
// across the wavefront first, as wave_peel does, costs these tables more
// than the LDS atomics it saves.)
template <int A>
__device__ __forceinline__ uint32_t listed_tally(ListedTable &t, const uint32_t (&lab)[A], const uint32_t (&wt)[A],
                                                 uint32_t rem, uint32_t cap = 0xFFFFFFFFu) {
#pragma unroll
    for (int j = 0; j < A; ++j) {
        if (t.n > cap) return rem;
        listed_insert(t, rem >> j & 1u, lab[j], wt[j]);
        rem &= ~(1u << j);
    }
    return rem;
}

// Clear the listed slots without reading them.
__device__ __forceinline__ void listed_clear(ListedTable &t) {
    for (uint32_t e = threadIdx.x & 63; e < t.n; e += 64) t.T[t.lst[e]] = EMPTY_SLOT;
    t.n = 0;
}

// Read and clear the listed entries: entry lane + 64 j becomes keys[j] as a
// vote key (0 where there is none).  Returns how many key columns are used.
template <int J>
__device__ __forceinline__ uint32_t listed_take(ListedTable &t, Tie tie, u64 (&keys)[J]) {
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t D = t.n;
#pragma unroll
    for (int j = 0; j < J; ++j) {
        keys[j] = 0;
        const uint32_t e = lane + 64u * j;
        if (e < D) {
            const uint32_t s = t.lst[e];
            keys[j] = slot_key(tie, t.T[s]);
            t.T[s] = EMPTY_SLOT;
        }
    }
    t.n = 0;
    return (D + 63) >> 6;
}

// Merge (lab, cnt) into a row's global slab.  Returns the slot index if this
// call claimed a new slot, else kNone.
__device__ __forceinline__ uint32_t slab_insert(u64 *S, uint32_t mask, uint32_t lab, uint32_t cnt) {
    uint32_t h = hmix(lab) & mask;
    const u64 desired = ((u64)lab << 32) | cnt;
    for (;;) {
        const u64 prev = atomicCAS(&S[h], EMPTY_SLOT, desired);
        if (prev == EMPTY_SLOT) return h;
        if ((uint32_t)(prev >> 32) == lab) {
            atomicAdd(&S[h], (u64)cnt);
            return kNone;
        }
        h = (h + 1) & mask;
    }
}

// Move the S-slot LDS table of one wavefront into a row's slab (`slab`,
// `smask` + 1 slots), recording per non-empty slot the slab slot it claimed
// (or kNone) in the row's touched list; the entries are reserved with one
// atomic per wavefront on *tcount.
__device__ __forceinline__ void flush_table(u64 *T, uint32_t S, u64 *slab, uint32_t smask, uint32_t *touched,
                                            uint32_t *tcount) {
    const uint32_t lane = threadIdx.x & 63;
    uint32_t ne = 0;
    for (uint32_t s = lane; s < S; s += 64) ne += T[s] != EMPTY_SLOT;
    uint32_t pre = ne;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(pre, off, 64);
        if ((int)lane >= off) pre += y;
    }
    const uint32_t total = __shfl(pre, 63, 64);
    pre -= ne;
    uint32_t tbase = 0;
    if (lane == 0 && total) tbase = atomicAdd(tcount, total);
    tbase = __shfl(tbase, 0, 64);
    uint32_t *tl = touched + tbase + pre;
    for (uint32_t s = lane; s < S; s += 64) {
        const u64 x = T[s];
        if (x != EMPTY_SLOT) {
            *tl++ = slab_insert(slab, smask, (uint32_t)(x >> 32), (uint32_t)x);
            T[s] = EMPTY_SLOT;
        }
    }
}

__device__ __forceinline__ void flush_to_slab(u64 *T, uint32_t S, const HubState &hs, uint32_t h) {
    flush_table(T, S, hs.slab + hs.slab_off[h], hs.slab_mask[h], hs.touched + hs.touched_off[h], &hs.tcount[h]);
}

// flush_table for a listed table: only the claimed slots are visited.
__device__ __forceinline__ void flush_listed(ListedTable &t, u64 *slab, uint32_t smask, uint32_t *touched,
                                             uint32_t *tcount) {
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t D = t.n;
    uint32_t tbase = 0;
    if (lane == 0 && D) tbase = atomicAdd(tcount, D);
    tbase = __shfl(tbase, 0, 64);
    for (uint32_t e = lane; e < D; e += 64) {
        const uint32_t s = t.lst[e];
        const u64 x = t.T[s];
        touched[tbase + e] = slab_insert(slab, smask, (uint32_t)(x >> 32), (uint32_t)x);
        t.T[s] = EMPTY_SLOT;
    }
    t.n = 0;
}

__device__ __forceinline__ void flush_listed_to_slab(ListedTable &t, const HubState &hs, uint32_t h) {
    flush_listed(t, hs.slab + hs.slab_off[h], hs.slab_mask[h], hs.touched + hs.touched_off[h], &hs.tcount[h]);
}

}  // namespace lpa
