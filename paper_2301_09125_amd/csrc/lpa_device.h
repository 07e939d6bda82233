// lpa_device.h -- device helpers shared by the kernel sources of the
// label-propagation library (wavefront reductions, LDS hashtables).
#pragma once

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

// Inverse of hmix (published with lowbias32).
__device__ __forceinline__ uint32_t hmix_inv(uint32_t x) {
    x ^= x >> 16;
    x *= 0x43021123u;
    x ^= (x >> 15) ^ (x >> 30);
    x *= 0x1d69e2a5u;
    x ^= x >> 16;
    return x;
}

// SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): output number c + 1 of the
// generator started from state `seed`.
__device__ __forceinline__ unsigned long long splitmix64_at(unsigned long long seed, unsigned long long c) {
    unsigned long long z = seed + 0x9E3779B97F4A7C15ull * (c + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Vote keys.  A candidate label is scored (tally << 32) | code(label), so one
// unsigned max picks the heaviest label and, among equal tallies, the one
// with the largest code.  Strict ties (Section 3.2, "the first" tied label,
// read as the lowest): code = ~label.  Hashed ties (the non-strict mode made
// reproducible): code = lowbias32(label ^ k) with a key k per vertex and
// round; lowbias32 is a bijection, so codes never collide and decode back.
// `hashed` comes from a kernel argument (uniform), `k` is per row.
struct Tie {
    uint32_t hashed;
    uint32_t k;
};
__device__ __forceinline__ uint32_t tie_code(Tie t, uint32_t lab) { return t.hashed ? hmix(lab ^ t.k) : ~lab; }
__device__ __forceinline__ uint32_t tie_label(Tie t, uint32_t code) {
    return t.hashed ? hmix_inv(code) ^ t.k : ~code;
}

// Make this wavefront's LDS writes visible to its other lanes.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ u64 umax64(u64 a, u64 b) { return a > b ? a : b; }

// slot (label << 32 | tally)  ->  vote key (tally << 32 | code(label))
__device__ __forceinline__ u64 slot_key(Tie t, u64 x) { return (x << 32) | tie_code(t, (uint32_t)(x >> 32)); }

__device__ __forceinline__ u64 vote_key(Tie t, uint32_t lab, u64 tally) { return (tally << 32) | tie_code(t, lab); }

// The label a vote key stands for.
__device__ __forceinline__ uint32_t key_label(Tie t, u64 key) { return tie_label(t, (uint32_t)key); }

constexpr Tie kStrict{0u, 0u};

__device__ __forceinline__ uint32_t next_pow2(uint32_t x) {
    return x <= 1 ? 1u : 1u << (32 - __clz(x - 1));
}

// Wavefront reductions on DPP lane moves (no LDS crossbar): swaps inside
// quads, then half-row and row mirrors leave every lane of a 16-lane row
// with the row's result; the row broadcasts 15 and 31 carry rows 0-2 into
// row 3, and lane 63 holds the wavefront's result.  Lanes a move does not
// write receive 0, the identity of both max and sum.
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ uint32_t dpp32(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROWS, 0xF, false);
}
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ u64 dpp64(u64 x) {
    return (u64)dpp32<CTRL, ROWS>((uint32_t)x) | ((u64)dpp32<CTRL, ROWS>((uint32_t)(x >> 32)) << 32);
}
constexpr int kDppXor1 = 0xB1;        // quad_perm [1, 0, 3, 2]
constexpr int kDppXor2 = 0x4E;        // quad_perm [2, 3, 0, 1]
constexpr int kDppHalfMirror = 0x141;  // row_half_mirror
constexpr int kDppMirror = 0x140;      // row_mirror
constexpr int kDppBcast15 = 0x142;     // row_bcast:15 (rows 1 and 3)
constexpr int kDppBcast31 = 0x143;     // row_bcast:31 (rows 2 and 3)

// Sum / max over each 16-lane row, returned to every lane of the row.
__device__ __forceinline__ uint32_t row_sum32(uint32_t x) {
    x += dpp32<kDppXor1>(x);
    x += dpp32<kDppXor2>(x);
    x += dpp32<kDppHalfMirror>(x);
    x += dpp32<kDppMirror>(x);
    return x;
}
__device__ __forceinline__ u64 row_sum64(u64 x) {
    x += dpp64<kDppXor1>(x);
    x += dpp64<kDppXor2>(x);
    x += dpp64<kDppHalfMirror>(x);
    x += dpp64<kDppMirror>(x);
    return x;
}
__device__ __forceinline__ u64 row_max64(u64 x) {
    x = umax64(x, dpp64<kDppXor1>(x));
    x = umax64(x, dpp64<kDppXor2>(x));
    x = umax64(x, dpp64<kDppHalfMirror>(x));
    x = umax64(x, dpp64<kDppMirror>(x));
    return x;
}

__device__ __forceinline__ uint32_t lane63_32(uint32_t x) { return (uint32_t)__builtin_amdgcn_readlane((int)x, 63); }
__device__ __forceinline__ u64 lane63_64(u64 x) {
    return (u64)lane63_32((uint32_t)x) | ((u64)lane63_32((uint32_t)(x >> 32)) << 32);
}

__device__ __forceinline__ uint32_t wave_sum32(uint32_t x) {
    x = row_sum32(x);
    x += dpp32<kDppBcast15, 0xA>(x);
    x += dpp32<kDppBcast31, 0xC>(x);
    return lane63_32(x);
}
__device__ __forceinline__ u64 wave_sum64(u64 x) {
    x = row_sum64(x);
    x += dpp64<kDppBcast15, 0xA>(x);
    x += dpp64<kDppBcast31, 0xC>(x);
    return lane63_64(x);
}
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ float dppf(float x) {
    return __uint_as_float(dpp32<CTRL, ROWS>(__float_as_uint(x)));
}
__device__ __forceinline__ float wave_sum(float x) {
    x += dppf<kDppXor1>(x);
    x += dppf<kDppXor2>(x);
    x += dppf<kDppHalfMirror>(x);
    x += dppf<kDppMirror>(x);
    x += dppf<kDppBcast15, 0xA>(x);  // lanes not written get +0.0f
    x += dppf<kDppBcast31, 0xC>(x);
    return __uint_as_float(lane63_32(__float_as_uint(x)));
}
template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
    static_assert(sizeof(T) == 4 || sizeof(T) == 8, "wave_sum: 32- or 64-bit integers");
    if constexpr (sizeof(T) == 4)
        return (T)wave_sum32((uint32_t)x);
    else
        return (T)wave_sum64((u64)x);
}
__device__ __forceinline__ u64 wave_max64(u64 x) {
    x = row_max64(x);
    x = umax64(x, dpp64<kDppBcast15, 0xA>(x));
    x = umax64(x, dpp64<kDppBcast31, 0xC>(x));
    return lane63_64(x);
}

// Inclusive prefix sum over the wavefront's lanes: shifts right by 1, 2, 4
// and 8 lanes inside each 16-lane row (lanes shifted in from outside the row
// receive 0), then the row broadcasts carry the totals of the rows below.
constexpr int kDppShr1 = 0x111, kDppShr2 = 0x112, kDppShr4 = 0x114, kDppShr8 = 0x118;  // row_shr:n
__device__ __forceinline__ u64 wave_scan_incl64(u64 x) {
    x += dpp64<kDppShr1>(x);
    x += dpp64<kDppShr2>(x);
    x += dpp64<kDppShr4>(x);
    x += dpp64<kDppShr8>(x);
    x += dpp64<kDppBcast15, 0xA>(x);
    x += dpp64<kDppBcast31, 0xC>(x);
    return x;
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

// Add this thread's count c into a round's counter words: one atomic per
// block, blocks spread over kCountSlots cache lines.  Every thread of a
// 256-thread block calls this once.
__device__ __forceinline__ void block_count(u64 c, u64 *slots) {
    __shared__ u64 part[4];
    c = wave_sum(c);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        const u64 s = part[0] + part[1] + part[2] + part[3];
        if (s) atomicAdd(&slots[(blockIdx.x % kCountSlots) * kCountStride], s);
    }
}

// block_count for two counts into two sets of counter words (one barrier).
__device__ __forceinline__ void block_count2(u64 c1, u64 *slots1, u64 c2, u64 *slots2) {
    __shared__ u64 part[2][4];
    c1 = wave_sum(c1);
    c2 = wave_sum(c2);
    if ((threadIdx.x & 63) == 0) {
        part[0][threadIdx.x >> 6] = c1;
        part[1][threadIdx.x >> 6] = c2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const u64 s1 = part[0][0] + part[0][1] + part[0][2] + part[0][3];
        const u64 s2 = part[1][0] + part[1][1] + part[1][2] + part[1][3];
        const uint32_t w = (blockIdx.x % kCountSlots) * kCountStride;
        if (s1) atomicAdd(&slots1[w], s1);
        if (s2) atomicAdd(&slots2[w], s2);
    }
}

// The changed count of a vote kernel and, when the round asks for it, its
// own-label weight sum.  Every thread of a 256-thread block calls this once.
__device__ __forceinline__ void block_counts(u64 chg, u64 ins, u64 *changed, u64 *insum) {
    if (insum)
        block_count2(chg, changed, ins, insum);
    else
        block_count(chg, changed);
}

// block_counts with the per-wavefront partials in LDS the caller provides:
// `mine` is this wavefront's own slice of a table it no longer uses (the
// slices of wavefronts 0..3 lie `stride` words apart, wavefront 0's first),
// so no barrier is needed before the write.
__device__ __forceinline__ void block_counts_at(u64 *mine, uint32_t stride, u64 chg, u64 ins, u64 *changed,
                                                u64 *insum) {
    chg = wave_sum(chg);
    if (insum) ins = wave_sum(ins);
    if ((threadIdx.x & 63) == 0) {
        mine[0] = chg;
        mine[1] = ins;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const u64 *p = mine;  // thread 0 is in wavefront 0
        const u64 s1 = p[0] + p[stride] + p[2 * stride] + p[3 * stride];
        const u64 s2 = p[1] + p[stride + 1] + p[2 * stride + 1] + p[3 * stride + 1];
        const uint32_t k = (blockIdx.x % kCountSlots) * kCountStride;
        if (s1) atomicAdd(&changed[k], s1);
        if (insum && s2) atomicAdd(&insum[k], s2);
    }
}

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

static inline unsigned grid_for(uint64_t count, unsigned per_block, unsigned cap) {
    uint64_t g = (count + per_block - 1) / per_block;
    if (g < 1) g = 1;
    return (unsigned)(g < cap ? g : cap);
}

}  // namespace lpa
