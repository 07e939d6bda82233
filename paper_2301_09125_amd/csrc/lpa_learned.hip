// lpa_learned.hip -- frontier-restricted RAK rounds and the learned vertex
// predictor (inference on MFMA, training on the vector units).
//
// Frontier.  A vertex whose closed neighbourhood did not change in round t-1
// and that was voted in round t-1 sees the same tally in round t, so it keeps
// its label: only the dirty vertices -- those with a changed neighbour or
// themselves changed (front[v] == t), plus those skipped earlier (stale[v])
// -- can change (frontier-based label propagation is named in Section 2 of
// arXiv 2301.09125).  push_*_k stamp front[] after every round.
//
// Predictor.  For every dirty vertex a 6-32-32-1 network scores whether it
// will change; only vertices scoring at least the cut are voted, the others
// copy their label and stay stale.  A vertex skipped in one round is always
// voted in the next (its features would be a round old).  Features (computed here, in FP32, then
// rounded to bfloat16):
//   f1 log2(1+deg)   f2 (top1-top2)/(k+sw)   f3 changed in round t-1
//   f4 top1/(k+sw)   f5 dirty through a neighbour   f6 t/max_iter
// (top1/top2: winning and runner-up tally of the vertex's last vote, k its
// weighted degree).  Network: h1 = relu(x W1 + b1), h2 = relu(bf16(h1) W2 +
// b2), z = h2 . w3 + b3 with bfloat16 x, W1, W2, w3 and FP32 accumulation.
// Both dense layers run on v_mfma_f32_32x32x8_bf16 in the transposed form
// (hidden units as rows, 32 candidates as columns): the accumulator of
// layer 1 is, register for register, the B operand of layer 2, so no data
// moves between the layers.
//
// Training: one thread per sample, forward and backward in FP32 with the same
// roundings (straight-through), per-block gradient sums written to their own
// slots and summed in a fixed order (deterministic), Adam on FP32 weights.

#include <algorithm>

#include "lpa_vote_dev.h"

namespace lpa {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ uint32_t f2bf(float f) {  // round to nearest even
    const uint32_t u = __builtin_bit_cast(uint32_t, f);
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ float bf2f(uint32_t b) { return __builtin_bit_cast(float, b << 16); }
__device__ __forceinline__ float bfround(float f) { return bf2f(f2bf(f)); }

// hidden unit held in accumulator register r of lane l (32x32 MFMA output)
__device__ __forceinline__ int acc_row(int r, int l) { return 8 * (r >> 2) + 4 * (l >> 5) + (r & 3); }

// Load a model from global memory into LDS (whole block).
__device__ __forceinline__ void load_model(MlpDev &dst, const MlpDev *src) {
    const uint32_t *s = reinterpret_cast<const uint32_t *>(src);
    uint32_t *d = reinterpret_cast<uint32_t *>(&dst);
    for (uint32_t i = threadIdx.x; i < sizeof(MlpDev) / 4; i += blockDim.x) d[i] = s[i];
    __syncthreads();
}

// Logit of the candidate held by each lane.  fa packs features 0..3, fb
// features 4..5 (then two zeros), as bfloat16.  All 64 lanes take part.
__device__ float mlp_wave(const MlpDev &M, uint64_t fa, uint64_t fb) {
    const int l = threadIdx.x & 63;
    float z_out = 0.f;
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        // column j of this pass = the candidate of lane 32p + j; lane half h
        // supplies features 4h .. 4h+3
        const int src = 32 * p + (l & 31);
        const uint64_t xa = __shfl(fa, src, 64), xb = __shfl(fb, src, 64);
        const uint64_t bx = (l < 32) ? xa : xb;
        f32x16 acc;
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[r] = M.b1[acc_row(r, l)];
        acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(__builtin_bit_cast(bf16x4, M.a1[l]),
                                                       __builtin_bit_cast(bf16x4, bx), acc, 0, 0, 0);
        uint64_t h[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            uint64_t w = 0;
#pragma unroll
            for (int c = 0; c < 4; ++c) w |= (uint64_t)f2bf(fmaxf(acc[4 * s + c], 0.f)) << (16 * c);
            h[s] = w;
        }
        f32x16 acc2;
#pragma unroll
        for (int r = 0; r < 16; ++r) acc2[r] = M.b2[acc_row(r, l)];
#pragma unroll
        for (int s = 0; s < 4; ++s)
            acc2 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(__builtin_bit_cast(bf16x4, M.a2[s][l]),
                                                            __builtin_bit_cast(bf16x4, h[s]), acc2, 0, 0, 0);
        float part = 0.f;
#pragma unroll
        for (int r = 0; r < 16; ++r) part += M.w3[acc_row(r, l)] * fmaxf(acc2[r], 0.f);
        part += __shfl_xor(part, 32, 64);
        if ((l >> 5) == p) z_out = part + M.b3;
    }
    return z_out;
}

__device__ __forceinline__ void pack_features(const float (&f)[6], uint64_t &fa, uint64_t &fb) {
    fa = (uint64_t)f2bf(f[0]) | (uint64_t)f2bf(f[1]) << 16 | (uint64_t)f2bf(f[2]) << 32 | (uint64_t)f2bf(f[3]) << 48;
    fb = (uint64_t)f2bf(f[4]) | (uint64_t)f2bf(f[5]) << 16;
}

// Features of internal vertex v before round t (see the header comment).
__device__ __forceinline__ void vertex_features(const FrontArgs &p, uint32_t v, bool dirty_nb, float (&f)[6]) {
    const uint64_t deg = p.g.rp[v + 1] - p.g.rp[v];
    const float k = (float)(p.kw ? (uint64_t)p.kw[v] : deg) + (float)p.sw;
    const float den = k > 0.f ? k : 1.f;
    const float t1 = (float)p.top1[v], t2 = (float)p.top2[v];
    f[0] = log2f(1.f + (float)deg);
    f[1] = (t1 - t2) / den;
    f[2] = p.lastchg[v] == p.t - 1 ? 1.f : 0.f;
    f[3] = t1 / den;
    f[4] = dirty_nb ? 1.f : 0.f;
    f[5] = (float)p.t / (float)p.max_iter;
}

// ---------------------------------------------------------------- predict --

// Rows lo .. lo+cnt-1 of one bin (none isolated, none long).  Block b owns
// the index range [b*K*256, (b+1)*K*256); each thread keeps one bit per
// chunk, then the block reserves its part of the output list with one
// atomic.  Decides for every dirty row: keep (vote) or skip (copy the label,
// stay stale); writes the round's vote mask by original id when asked.
__global__ __launch_bounds__(256) void predict_k(FrontArgs p, const MlpDev *model, uint32_t lo, uint32_t cnt,
                                                 uint32_t K, uint32_t *list, uint32_t *list_count) {
    __shared__ MlpDev M;
    __shared__ uint32_t wsum[4][2];
    __shared__ unsigned long long warcs[4], wskip[4];
    __shared__ uint32_t base_s;
    __shared__ u64 mk[32][4];      // kept lanes of each chunk and wavefront
    __shared__ uint32_t offs[32][4];
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid < 128) (&mk[0][0])[tid] = 0;
    if (!p.keep_all)
        load_model(M, model);
    else
        __syncthreads();
    const uint64_t begin = (uint64_t)blockIdx.x * K * 256;
    uint32_t bits = 0, ncand = 0;
    uint64_t karcs = 0, eskip = 0;
    for (uint32_t k = 0; k < K; ++k) {
        const uint64_t i = begin + (uint64_t)k * 256 + tid;
        const bool in = i < cnt;
        const uint32_t v = lo + (uint32_t)(in ? i : 0);
        bool dirty_nb = false, cand = false, was_skipped = false;
        if (in) {
            dirty_nb = p.all_dirty || p.front[v] == p.t;
            was_skipped = p.stale[v] != 0;
            cand = dirty_nb || was_skipped;
        }
        if (!__ballot(cand)) {
            if (in && p.mask) p.mask[p.old_of[v]] = 0;
            continue;  // wavefront-uniform
        }
        bool keep = cand;
        if (!p.keep_all) {
            float f[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            if (cand) vertex_features(p, v, dirty_nb, f);
            uint64_t fa, fb;
            pack_features(f, fa, fb);
            const float z = mlp_wave(M, fa, fb);
            // a row skipped last round is voted now: its features are a
            // round old, and no row stays unvoted two rounds in a row
            keep = cand && (was_skipped || z >= M.zcut);
            if (cand && !keep) eskip += (uint32_t)(1024.f / (1.f + expf(-z)) + 0.5f);
        }
        if (cand) {
            ++ncand;
            if (keep) {
                bits |= 1u << k;
                karcs += p.g.rp[v + 1] - p.g.rp[v];
                if (p.stale[v]) p.stale[v] = 0;
            } else {
                p.L_new[v] = p.L_old[v];
                p.stale[v] = 1;
            }
        }
        if (in && p.mask) p.mask[p.old_of[v]] = keep ? 1 : 0;
        const u64 kb = __ballot(cand && keep);
        if (lane == 0) mk[k][wave] = kb;
    }
    // list positions in vertex order: chunk-major, then wavefront, then lane
    const uint32_t nc = wave_sum(ncand);
    const unsigned long long ka = wave_sum((unsigned long long)karcs);
    const unsigned long long es = wave_sum((unsigned long long)eskip);
    if (lane == 0) {
        wsum[wave][1] = nc;
        warcs[wave] = ka;
        wskip[wave] = es;
    }
    __syncthreads();
    if (tid == 0) {
        uint32_t run = 0, tc = 0;
        unsigned long long ta = 0, ts = 0;
        for (uint32_t k = 0; k < K; ++k)
            for (uint32_t q = 0; q < 4; ++q) {
                offs[k][q] = run;
                run += __popcll(mk[k][q]);
            }
        for (uint32_t q = 0; q < 4; ++q) {
            tc += wsum[q][1];
            ta += warcs[q];
            ts += wskip[q];
        }
        base_s = run ? atomicAdd(list_count, run) : 0u;
        if (tc) atomicAdd(p.cand_count, (unsigned long long)tc);
        if (ta) atomicAdd(p.kept_arcs, ta);
        if (ts) atomicAdd(p.exp_skip, ts);
    }
    __syncthreads();
    const u64 below = (1ull << lane) - 1;
    while (bits) {
        const uint32_t k = __ffs(bits) - 1;
        bits &= bits - 1;
        const uint32_t pos = base_s + offs[k][wave] + __popcll(mk[k][wave] & below);
        list[pos] = lo + (uint32_t)(begin + (uint64_t)k * 256 + tid);
    }
}

// ------------------------------------------------------------------- push --

// After round t (L_old = round t-1, L_new = round t): every changed vertex
// records t in lastchg and, when `mark`, stamps t+1 into front[] for itself
// and its neighbours.  One lane per row.
__global__ void push_small_k(FrontArgs p, uint32_t lo, uint32_t cnt, int mark) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += gridDim.x * blockDim.x) {
        const uint32_t v = lo + i;
        if (p.L_new[v] == p.L_old[v]) continue;
        p.lastchg[v] = p.t;
        if (!mark) continue;
        const uint32_t s = p.t + 1;
        p.front[v] = s;
        for (uint64_t e = p.g.rp[v]; e < p.g.rp[v + 1]; ++e) p.front[p.g.col[e]] = s;
    }
}

// Same for long rows: one wavefront per row.
__global__ void push_rows_k(FrontArgs p, uint32_t lo, uint32_t cnt, int mark) {
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t nw = gridDim.x * (blockDim.x >> 6);
    for (uint32_t i = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); i < cnt; i += nw) {
        const uint32_t v = lo + i;
        if (p.L_new[v] == p.L_old[v]) continue;  // uniform across the wavefront
        if (lane == 0) p.lastchg[v] = p.t;
        if (!mark) continue;
        const uint32_t s = p.t + 1;
        if (lane == 0) p.front[v] = s;
        for (uint64_t e = p.g.rp[v] + lane; e < p.g.rp[v + 1]; e += 64) p.front[p.g.col[e]] = s;
    }
}

// ------------------------------------------------------------------ traces --

// Features of rows lo .. lo+cnt-1 before round t into X[i] (6 FP32 each).
__global__ void trace_x_k(FrontArgs p, uint32_t lo, uint32_t cnt, float *X) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += gridDim.x * blockDim.x) {
        const uint32_t v = lo + i;
        float f[6];
        vertex_features(p, v, p.all_dirty || p.front[v] == p.t, f);
#pragma unroll
        for (int c = 0; c < 6; ++c) X[(uint64_t)i * 6 + c] = f[c];
    }
}

// Labels of the samples: did the row change in this round.
__global__ void trace_y_k(const uint32_t *L_old, const uint32_t *L_new, uint32_t lo, uint32_t cnt, uint8_t *y) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += gridDim.x * blockDim.x)
        y[i] = L_old[lo + i] != L_new[lo + i] ? 1 : 0;
}

// ---------------------------------------------------------------- forward --

// Logits of N feature rows (FP32, 6 per row) with the inference arithmetic.
__global__ __launch_bounds__(256) void mlp_forward_k(const MlpDev *model, const float *X, uint64_t N, float *z) {
    __shared__ MlpDev M;
    load_model(M, model);
    const uint64_t nw = (uint64_t)gridDim.x * 4;
    for (uint64_t w = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6); w * 64 < N; w += nw) {
        const uint64_t i = w * 64 + (threadIdx.x & 63);
        float f[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if (i < N)
#pragma unroll
            for (int c = 0; c < 6; ++c) f[c] = X[i * 6 + c];
        uint64_t fa, fb;
        pack_features(f, fa, fb);
        const float zz = mlp_wave(M, fa, fb);
        if (i < N) z[i] = zz;
    }
}

// --------------------------------------------------------------- training --

constexpr int kH = 32, kF = 6;
constexpr int kParams = kF * kH + kH + kH * kH + kH + kH + 1;  // 1313
// offsets in the flat parameter vector (the lpa_mlp field order)
constexpr int oW1 = 0, oB1 = kF * kH, oW2 = oB1 + kH, oB2 = oW2 + kH * kH, oW3 = oB2 + kH, oB3 = oW3 + kH;

// One thread per sample of the batch: sample s = (mul * (start + i) + add) mod N.
// Writes this block's gradient sums (kParams) and loss sum to part[block].
__global__ __launch_bounds__(256) void train_grad_k(const float *X, const uint8_t *y, uint64_t N, uint64_t mul,
                                                    uint64_t add, uint64_t start, uint32_t bn, const float *wm,
                                                    float pos_weight, float *part) {
    __shared__ float W[kParams];  // weights, W1/W2/w3 rounded to bfloat16
    __shared__ float bufA[4][64][kH + 1];
    __shared__ float bufB[4][64][kH + 1];
    __shared__ float G[4][kParams + 1];
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int i = tid; i < kParams; i += 256) {
        const bool q = (i < oB1) || (i >= oW2 && i < oB2) || (i >= oW3 && i < oB3);
        W[i] = q ? bfround(wm[i]) : wm[i];
    }
    for (int i = tid; i < 4 * (kParams + 1); i += 256) (&G[0][0])[i] = 0.f;
    __syncthreads();
    const uint64_t ib = (uint64_t)blockIdx.x * 256 + tid;
    const bool valid = ib < bn;
    float x[kF], a1[kH], h1[kH], a2[kH];
    float yy = 0.f;
#pragma unroll
    for (int c = 0; c < kF; ++c) x[c] = 0.f;
    if (valid) {
        const uint64_t s = (mul * ((start + ib) % N) + add) % N;
#pragma unroll
        for (int c = 0; c < kF; ++c) x[c] = bfround(X[s * kF + c]);
        yy = y[s] ? 1.f : 0.f;
    }
#pragma unroll
    for (int j = 0; j < kH; ++j) {
        float acc = W[oB1 + j];
#pragma unroll
        for (int c = 0; c < kF; ++c) acc += x[c] * W[oW1 + c * kH + j];
        a1[j] = acc;
        h1[j] = bfround(fmaxf(acc, 0.f));
    }
#pragma unroll
    for (int k = 0; k < kH; ++k) {
        float acc = W[oB2 + k];
#pragma unroll
        for (int j = 0; j < kH; ++j) acc += h1[j] * W[oW2 + j * kH + k];
        a2[k] = acc;
    }
    float z = W[oB3];
#pragma unroll
    for (int k = 0; k < kH; ++k) z += fmaxf(a2[k], 0.f) * W[oW3 + k];
    // weighted BCE on the logit; softplus(x) = max(x,0) + log1p(exp(-|x|))
    const float sp_pos = fmaxf(z, 0.f) + log1pf(expf(-fabsf(z)));  // softplus(z)
    const float sp_neg = sp_pos - z;                                // softplus(-z)
    const float sig = 1.f / (1.f + expf(-z));
    float lossv = 0.f, dz = 0.f;
    if (valid) {
        lossv = pos_weight * yy * sp_neg + (1.f - yy) * sp_pos;
        dz = (sig * (pos_weight * yy + 1.f - yy) - pos_weight * yy) / (float)bn;
    }
    // layer 3 and layer 2 gradients: bufA = h1 (bf16), bufB = da2
#pragma unroll
    for (int k = 0; k < kH; ++k) {
        const float h2 = fmaxf(a2[k], 0.f);
        bufA[wave][lane][k] = h1[k];
        bufB[wave][lane][k] = a2[k] > 0.f ? dz * W[oW3 + k] : 0.f;
        a2[k] = dz * h2;  // reuse: per-sample dw3 contribution
    }
    // dh1 = da2 W2^T
    float dh1[kH];
#pragma unroll
    for (int j = 0; j < kH; ++j) {
        float acc = 0.f;
#pragma unroll
        for (int k = 0; k < kH; ++k) acc += bufB[wave][lane][k] * W[oW2 + j * kH + k];
        dh1[j] = a1[j] > 0.f ? acc : 0.f;  // da1
    }
    // per-wave sums: gw3, gb3, loss via shuffles
#pragma unroll
    for (int k = 0; k < kH; ++k) {
        const float s = wave_sum(a2[k]);
        if (lane == 0) G[wave][oW3 + k] = s;
    }
    {
        const float s = wave_sum(dz), ls = wave_sum(lossv);
        if (lane == 0) {
            G[wave][oB3] = s;
            G[wave][kParams] = ls;
        }
    }
    wave_sync();
    // gw2[j][k] = sum_s h1[s][j] da2[s][k]: lane owns j = lane/2, k in 16*(lane%2) ..+16
    {
        const int j = lane >> 1, k0 = 16 * (lane & 1);
        float acc[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) acc[q] = 0.f;
        float bsum[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) bsum[q] = 0.f;
        for (int s = 0; s < 64; ++s) {
            const float hj = bufA[wave][s][j];
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const float d = bufB[wave][s][k0 + q];
                acc[q] += hj * d;
                bsum[q] += d;
            }
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) G[wave][oW2 + j * kH + k0 + q] = acc[q];
        if (j == 0)
#pragma unroll
            for (int q = 0; q < 16; ++q) G[wave][oB2 + k0 + q] = bsum[q];
    }
    wave_sync();
    // layer 1: bufA[.][0..5] = x, bufB = da1
#pragma unroll
    for (int j = 0; j < kH; ++j) bufB[wave][lane][j] = dh1[j];
#pragma unroll
    for (int c = 0; c < kF; ++c) bufA[wave][lane][c] = x[c];
    wave_sync();
    // gw1[c][j] (192) and gb1[j] (32): lane owns column j = lane % 32 and, for
    // lanes 0..31, rows c = 0..2, for lanes 32..63 rows 3..5 (+ gb1 on 0..31)
    {
        const int j = lane & 31, c0 = 3 * (lane >> 5);
        float acc[3] = {0.f, 0.f, 0.f}, bs = 0.f;
        for (int s = 0; s < 64; ++s) {
            const float d = bufB[wave][s][j];
#pragma unroll
            for (int q = 0; q < 3; ++q) acc[q] += bufA[wave][s][c0 + q] * d;
            bs += d;
        }
#pragma unroll
        for (int q = 0; q < 3; ++q) G[wave][oW1 + (c0 + q) * kH + j] = acc[q];
        if (lane < 32) G[wave][oB1 + j] = bs;
    }
    __syncthreads();
    for (int i = tid; i <= kParams; i += 256)
        part[(uint64_t)blockIdx.x * (kParams + 1) + i] = G[0][i] + G[1][i] + G[2][i] + G[3][i];
}

// Sum the per-block partials in block order (deterministic).
__global__ void train_reduce_k(const float *part, uint32_t nblk, float *grad) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > (uint32_t)kParams) return;
    float s = 0.f;
    for (uint32_t b = 0; b < nblk; ++b) s += part[(uint64_t)b * (kParams + 1) + i];
    grad[i] = s;
}

// Adam step on the FP32 weights; grad[kParams] (the loss) is added to
// loss_acc.
__global__ void adam_k(float *wm, float *m, float *v, const float *grad, float lr, float b1, float b2, float eps,
                       float c1, float c2, float *loss_acc) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == (uint32_t)kParams) loss_acc[0] += grad[kParams];
    if (i >= (uint32_t)kParams) return;
    const float g = grad[i];
    const float mi = b1 * m[i] + (1.f - b1) * g;
    const float vi = b2 * v[i] + (1.f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    wm[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Weighted degree of every row.
__global__ void row_sums_k(Graph g, uint32_t *kw) {
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < g.n; v += gridDim.x * blockDim.x) {
        uint64_t s = 0;
        for (uint64_t e = g.rp[v]; e < g.rp[v + 1]; ++e) s += g.w[e];
        kw[v] = (uint32_t)(s > 0xFFFFFFFFull ? 0xFFFFFFFFull : s);
    }
}

// mask[old_of[r]] = val for rows lo .. lo+cnt-1.
__global__ void mask_rows_k(uint8_t *mask, const uint32_t *old_of, uint32_t lo, uint32_t cnt, uint8_t val) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += gridDim.x * blockDim.x)
        mask[old_of[lo + i]] = val;
}

// ------------------------------------------------------------- launchers --

hipError_t launch_row_sums(const Graph &g, uint32_t *kw, hipStream_t s) {
    if (g.n == 0) return hipSuccess;
    row_sums_k<<<grid_for(g.n, 256, 8192), 256, 0, s>>>(g, kw);
    return hipGetLastError();
}

hipError_t launch_mask_rows(uint8_t *mask, const uint32_t *old_of, uint32_t lo, uint32_t cnt, uint8_t val,
                            hipStream_t s) {
    if (cnt == 0) return hipSuccess;
    mask_rows_k<<<grid_for(cnt, 256, 8192), 256, 0, s>>>(mask, old_of, lo, cnt, val);
    return hipGetLastError();
}

hipError_t launch_predict(const FrontArgs &p, const MlpDev *model, uint32_t lo, uint32_t cnt, uint32_t *list,
                          uint32_t *list_count, int num_cu, hipStream_t s) {
    if (cnt == 0) return hipSuccess;
    // few blocks (each reserves its list range with one atomic on a shared
    // counter), at most 32 chunks of 256 rows per thread
    const uint64_t chunks = (cnt + 255) / 256;
    const uint64_t want = std::max<uint64_t>((uint64_t)num_cu * 2, (chunks + 31) / 32);
    const uint64_t grid = std::min<uint64_t>(chunks, want);
    const uint32_t K = (uint32_t)((chunks + grid - 1) / grid);
    const uint32_t g = (uint32_t)((chunks + K - 1) / K);
    predict_k<<<g, 256, 0, s>>>(p, model, lo, cnt, K, list, list_count);
    return hipGetLastError();
}

hipError_t launch_push(const FrontArgs &p, const Bins &B, int mark, hipStream_t s) {
    const uint32_t rows = B.cnt[BIN_HUB] + B.cnt[BIN_WIDE] + B.cnt[BIN_WAVE];
    if (rows) push_rows_k<<<grid_for(rows, 4, 8192), 256, 0, s>>>(p, B.lo[BIN_HUB], rows, mark);
    const uint32_t small = B.cnt[BIN_GROUP] + B.cnt[BIN_THREAD];
    if (small) push_small_k<<<grid_for(small, 256, 8192), 256, 0, s>>>(p, B.lo[BIN_GROUP], small, mark);
    return hipGetLastError();
}

hipError_t launch_trace_x(const FrontArgs &p, uint32_t lo, uint32_t cnt, float *X, hipStream_t s) {
    if (cnt == 0) return hipSuccess;
    trace_x_k<<<grid_for(cnt, 256, 8192), 256, 0, s>>>(p, lo, cnt, X);
    return hipGetLastError();
}

hipError_t launch_trace_y(const uint32_t *L_old, const uint32_t *L_new, uint32_t lo, uint32_t cnt, uint8_t *y,
                          hipStream_t s) {
    if (cnt == 0) return hipSuccess;
    trace_y_k<<<grid_for(cnt, 256, 8192), 256, 0, s>>>(L_old, L_new, lo, cnt, y);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const MlpDev *model, const float *X, uint64_t N, float *z, hipStream_t s) {
    if (N == 0) return hipSuccess;
    const uint64_t waves = (N + 63) / 64;
    const uint32_t g = (uint32_t)std::min<uint64_t>((waves + 3) / 4, 8192);
    mlp_forward_k<<<g, 256, 0, s>>>(model, X, N, z);
    return hipGetLastError();
}

int mlp_params() { return kParams; }

hipError_t launch_train_step(const float *X, const uint8_t *y, uint64_t N, uint64_t mul, uint64_t add,
                             uint64_t start, uint32_t bn, float *wm, float *m, float *v, float *part, float *grad,
                             float pos_weight, float lr, float c1, float c2, float *loss_acc, int update,
                             hipStream_t s) {
    const uint32_t nblk = (bn + 255) / 256;
    train_grad_k<<<nblk, 256, 0, s>>>(X, y, N, mul, add, start, bn, wm, pos_weight, part);
    train_reduce_k<<<(kParams + 1 + 255) / 256, 256, 0, s>>>(part, nblk, grad);
    if (update) adam_k<<<(kParams + 1 + 255) / 256, 256, 0, s>>>(wm, m, v, grad, lr, 0.9f, 0.999f, 1e-8f, c1, c2,
                                                                 loss_acc);
    return hipGetLastError();
}

}  // namespace lpa
