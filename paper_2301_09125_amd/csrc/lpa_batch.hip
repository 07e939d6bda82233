// lpa_batch.hip -- RAK (arXiv 2301.09125, Section 3.2) on many independent
// graphs at once, all rounds in one persistent launch.
//
// The graphs are packed into one CSR whose arcs stay inside their graph and
// relabelled like a single graph (lpa_internal.h), so every degree bin is a
// contiguous range of internal ids across all graphs.  gid[r] names the
// graph of internal vertex r.  Each graph keeps its own tolerance test
// (changed_g <= floor(tol * n_g)) and its own round count: a graph that
// converges (or reaches max_iter) stops being voted, and its labels stay in
// the buffer its last round wrote.  The result of every graph therefore
// equals a run of that graph alone.
//
// One launch, `nblocks` co-resident blocks; per round:
//   phase A  every wavefront takes work units from a fixed interleaved list:
//            one long row (> wide_max arcs; its 512-arc segments are merged
//            exactly through the row's global slab by the same wavefront),
//            one wavefront row, four 16-lane rows or 64 one-lane rows.
//            Rows of converged graphs are skipped.  Changed counts are added
//            per graph (one atomic per graph present in a wavefront).
//   barrier
//   phase B  one lane per active graph records the round and applies its
//            tolerance test; the number of running graphs drops as they stop.
//   barrier  then every block leaves once no graph is running.
// Barriers count arrivals with an atomic and release on a generation
// number; a wait that exceeds a wall-clock limit raises ERR_TIMEOUT and
// every block leaves the kernel, so the launch always ends.

#include "lpa_vote_dev.h"

namespace lpa {

// Grid-wide barrier over `nblocks` blocks that are all resident.
__device__ __forceinline__ bool grid_barrier(const BatchArgs &b, uint32_t nblocks) {
    __shared__ int failed;
    __syncthreads();
    if (threadIdx.x == 0) {
        failed = 0;
        const uint32_t gen = __hip_atomic_load(&b.bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        const uint32_t arrived = atomicAdd(&b.bar[0], 1u) + 1;
        if (arrived == nblocks) {
            __hip_atomic_store(&b.bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __threadfence();
            __hip_atomic_fetch_add(&b.bar[1], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            const uint64_t t0 = wall_clock64();
            while (__hip_atomic_load(&b.bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                __builtin_amdgcn_s_sleep(2);
                if (wall_clock64() - t0 > b.timeout_ticks) {
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

// Add the changed flags of the wavefront's lanes to their graphs' counters:
// one atomic per distinct graph among the changed lanes.
__device__ __forceinline__ void count_per_graph(const BatchArgs &b, bool ch, uint32_t g) {
    const uint32_t lane = threadIdx.x & 63;
    u64 m = __ballot(ch);
    while (m) {
        const int lead = __ffsll((long long)m) - 1;
        const uint32_t gl = __shfl(g, lead, 64);
        const u64 same = __ballot(ch && g == gl);
        if (lane == 0) atomicAdd(&b.changed[gl], (u64)__popcll(same));
        m &= ~same;
    }
}

// In round 1, arcs must stay inside their graph.
template <int A>
__device__ __forceinline__ void check_graph(const BatchArgs &b, const uint32_t (&u)[A], uint32_t valid,
                                            uint32_t g) {
    bool bad = false;
#pragma unroll
    for (int j = 0; j < A; ++j)
        if (valid >> j & 1u) bad |= b.gid[u[j]] != g;
    if (bad) atomicOr(b.err, ERR_GRAPH);
}

// 64 one-lane rows (degree <= 8).
__device__ void unit_thread(const BatchArgs &b, const RoundArgs &a, uint32_t v0, uint32_t v1, bool round1) {
    constexpr int D = kThreadMaxCap;
    const uint32_t v = v0 + (threadIdx.x & 63);
    bool ch = false;
    uint32_t g = 0;
    if (v < v1) {
        g = b.gid[v];
        if (b.active[g]) {
            const uint64_t rb = a.g.rp[v], re = a.g.rp[v + 1];
            const uint32_t own = a.L_old[v];
            uint32_t u[D], lab[D], wt[D], tl[D], valid = 0;
            load_arcs<D, 1>(a, rb, re, u, wt, valid);
            if (round1) check_graph<D>(b, u, valid, g);
            gather_labels<D>(a, u, valid, lab);
            u64 rs = a.sw;
#pragma unroll
            for (int j = 0; j < D; ++j) {
                rs += wt[j];
                tl[j] = wt[j] + (lab[j] == own ? a.sw : 0u);
            }
#pragma unroll
            for (int j = 0; j < D; ++j)
#pragma unroll
                for (int k = j + 1; k < D; ++k)
                    if (lab[j] == lab[k]) {
                        tl[j] += wt[k];
                        tl[k] += wt[j];
                    }
            u64 best = a.sw ? vote_key(own, a.sw) : 0ull;
#pragma unroll
            for (int j = 0; j < D; ++j)
                if (valid >> j & 1u) best = umax64(best, vote_key(lab[j], tl[j]));
            const uint32_t nl = best ? ~(uint32_t)best : own;
            a.L_new[v] = nl;
            ch = nl != own;
            if (round1 && rs > 0xFFFFFFFFull) atomicOr(a.err, ERR_WOVF);
        }
    }
    count_per_graph(b, ch, g);
}

// Four 16-lane rows (degree <= 32), one 64-slot table each inside T.
__device__ void unit_group(const BatchArgs &b, const RoundArgs &a, u64 *T, uint32_t v0, uint32_t v1, bool round1) {
    constexpr int G = kGroupLanes, CAP = kGroupSlots, A = CAP / (2 * G);
    const uint32_t lane = threadIdx.x & 63, gl = lane & (G - 1);
    u64 *Tg = T + (lane / G) * CAP;
    const uint32_t v = v0 + lane / G;
    bool act = v < v1;
    uint32_t g = 0;
    if (act) {
        g = b.gid[v];
        act = b.active[g] != 0;
    }
    uint64_t rb = 0, re = 0;
    uint32_t own = 0;
    if (act) {
        rb = a.g.rp[v];
        re = a.g.rp[v + 1];
        own = a.L_old[v];
    }
    uint32_t u[A], lab[A], wt[A], valid = 0;
    load_arcs<A, G>(a, rb + gl, re, u, wt, valid);
    if (round1) check_graph<A>(b, u, valid, g);
    gather_labels<A>(a, u, valid, lab);
    u64 own_w = 0, rs = 0;
    uint32_t own_hit = 0, rem = 0;
    split_own<A>(lab, wt, valid, own, own_w, own_hit, rem, rs);
    uint32_t S = next_pow2(2u * (uint32_t)(re - rb));
    S = S < (uint32_t)G ? (uint32_t)G : (S > (uint32_t)CAP ? (uint32_t)CAP : S);
#pragma unroll
    for (int j = 0; j < A; ++j)
        if (rem >> j & 1u) lds_insert(Tg, S - 1, lab[j], wt[j]);
    wave_sync();
    u64 best = 0;
    for (uint32_t s = gl; s < S; s += G) {
        const u64 x = Tg[s];
        if (x != EMPTY_SLOT) {
            best = umax64(best, slot_key(x));
            Tg[s] = EMPTY_SLOT;
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
        if (own_hit || a.sw) best = umax64(best, vote_key(own, own_w + a.sw));
        const uint32_t nl = best ? ~(uint32_t)best : own;
        a.L_new[v] = nl;
        ch = nl != own;
        if (round1 && rs + a.sw > 0xFFFFFFFFull) atomicOr(a.err, ERR_WOVF);
    }
    wave_sync();
    count_per_graph(b, ch, g);
}

// One row of at most 512 arcs, or of any length through its global slab
// when `long_row` (h = its index among the long rows).
__device__ void unit_wave(const BatchArgs &b, const RoundArgs &a, u64 *T, uint32_t v, uint32_t h, bool long_row,
                          bool round1) {
    constexpr int A = kWaveArcs / 64;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t g = b.gid[v];
    if (!b.active[g]) return;  // uniform over the wavefront
    const uint64_t rb = a.g.rp[v], re = a.g.rp[v + 1];
    const uint32_t own = a.L_old[v];
    u64 own_w = 0, rs = 0, best = 0;
    uint32_t own_hit = 0;
    for (uint64_t k0 = rb; k0 < re; k0 += kWaveArcs) {
        const uint64_t k1 = re < k0 + kWaveArcs ? re : k0 + kWaveArcs;
        uint32_t u[A], lab[A], wt[A], valid = 0;
        load_arcs<A, 64>(a, k0 + lane, k1, u, wt, valid);
        if (round1) check_graph<A>(b, u, valid, g);
        gather_labels<A>(a, u, valid, lab);
        uint32_t rem = 0;
        split_own<A>(lab, wt, valid, own, own_w, own_hit, rem, rs);
        uint32_t S = next_pow2(2u * (uint32_t)(k1 - k0));
        S = S < 64u ? 64u : (S > (uint32_t)kWaveSlots ? (uint32_t)kWaveSlots : S);
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
                        best = umax64(best, slot_key(x));
                        T[s] = EMPTY_SLOT;
                    }
                }
            }
            wave_sync();
        }
    }
    if (long_row) {
        // the row's slab holds its exact tallies: take the max over the
        // claimed slots and clear them for the next round
        __threadfence();
        const uint32_t tc = __hip_atomic_load(&b.tcount[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        u64 *slab = b.slab + b.slab_off[h];
        const uint32_t *tl = b.touched + b.touched_off[h];
        for (uint32_t p = lane; p < tc; p += 64) {
            const uint32_t s = tl[p];
            if (s != kNone) {
                best = umax64(best, slot_key(__hip_atomic_load(&slab[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)));
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
        if (own_hit || a.sw) best = umax64(best, vote_key(own, own_w + a.sw));
        const uint32_t nl = best ? ~(uint32_t)best : own;
        a.L_new[v] = nl;
        ch = nl != own;
        if (round1 && rs + a.sw > 0xFFFFFFFFull) atomicOr(a.err, ERR_WOVF);
    }
    count_per_graph(b, ch, g);
}

__global__ __launch_bounds__(256) void batch_k(BatchArgs b, uint32_t nblocks) {
    __shared__ u64 table[4 * kWaveSlots];
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    u64 *T = table + wave * kWaveSlots;
    for (uint32_t s = lane; s < kWaveSlots; s += 64) T[s] = EMPTY_SLOT;
    wave_sync();
    const uint32_t n_long = b.cnt[BIN_HUB];
    const uint32_t n_wave = b.cnt[BIN_WIDE] + b.cnt[BIN_WAVE];
    const uint32_t n_group = (b.cnt[BIN_GROUP] + 3) / 4;
    const uint32_t n_thread = (b.cnt[BIN_THREAD] + 63) / 64;
    const uint32_t units = n_long + n_wave + n_group + n_thread;
    const uint32_t wid = blockIdx.x * 4 + wave, nw = nblocks * 4;
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
        const bool round1 = t == 1;
        // phase A
        for (uint32_t u = wid; u < units; u += nw) {
            if (u < n_long) {
                unit_wave(b, a, T, b.lo[BIN_HUB] + u, u, true, round1);
            } else if (u < n_long + n_wave) {
                unit_wave(b, a, T, b.lo[BIN_WIDE] + (u - n_long), 0, false, round1);
            } else if (u < n_long + n_wave + n_group) {
                const uint32_t v0 = b.lo[BIN_GROUP] + 4 * (u - n_long - n_wave);
                unit_group(b, a, T, v0, b.lo[BIN_GROUP] + b.cnt[BIN_GROUP], round1);
            } else {
                const uint32_t v0 = b.lo[BIN_THREAD] + 64 * (u - n_long - n_wave - n_group);
                unit_thread(b, a, v0, b.lo[BIN_THREAD] + b.cnt[BIN_THREAD], round1);
            }
        }
        if (!grid_barrier(b, nblocks)) return;
        // phase B: tolerance test per graph
        for (uint32_t g = blockIdx.x * 256 + threadIdx.x; g < b.G; g += nblocks * 256) {
            if (b.active[g]) {
                const u64 ch = b.changed[g];
                b.changed[g] = 0;
                b.last[g] = ch;
                b.iters[g] = t;
                if (t <= b.hist_len) b.hist[(u64)g * b.hist_len + (t - 1)] = ch;
                const bool ok = ch <= b.thr[g];
                if (ok || t == b.max_iter) {
                    b.conv[g] = ok ? 1 : 0;
                    b.active[g] = 0;
                    atomicSub(b.n_active, 1u);
                    atomicAdd(b.arcs, (u64)(b.orp[b.gv[g + 1]] - b.orp[b.gv[g]]) * t);
                }
            }
        }
        if (!grid_barrier(b, nblocks)) return;
        if (__hip_atomic_load(b.n_active, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) break;
        if (__hip_atomic_load(b.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & (ERR_COL | ERR_GRAPH)) break;
    }
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
hipError_t launch_batch_out(uint32_t *out, const uint32_t *old_of, const uint32_t *gid, const uint32_t *L0,
                            const uint32_t *L1, const uint32_t *iters, const uint64_t *gv, uint32_t n,
                            hipStream_t s) {
    if (n == 0) return hipSuccess;
    batch_out_k<<<grid_for(n, 256, 8192), 256, 0, s>>>(out, old_of, gid, L0, L1, iters, gv, n);
    return hipGetLastError();
}

int batch_blocks_per_cu() {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_k, 256, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    return per_cu;
}

hipError_t launch_batch(const BatchArgs &b, uint32_t nblocks, hipStream_t s) {
    void *args[] = {(void *)&b, (void *)&nblocks};
    return hipLaunchCooperativeKernel((const void *)batch_k, dim3(nblocks), dim3(256), args, 0, s);
}

}  // namespace lpa
