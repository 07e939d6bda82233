// lpa_prep.hip -- per-run preparation kernels: degree binning, the
// relabelled internal CSR, label initialisation and the final scatter.
//
// Binning is a stable partition of the vertices by degree bin (1024
// vertices per 256-thread block: count, one-block scan, scatter).  The
// scatter also assigns each non-isolated vertex its internal id and the
// start of its internal row (an exclusive prefix of degrees in internal
// order), so the internal row_ptr comes out of the same pass.

#include "lpa_device.h"

namespace lpa {

// ---------------------------------------------------------------- fills --

__global__ void iota_k(uint32_t *a, uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) a[i] = i;
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
__global__ void check_labels_k(const uint32_t *labels, uint32_t n, uint32_t *err) {
    bool bad = false;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        bad |= labels[i] >= n;
    if (bad) atomicOr(err, ERR_LABEL);
}

hipError_t launch_fill_u32_iota(uint32_t *a, uint32_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    iota_k<<<grid_for(n, 256, 8192), 256, 0, s>>>(a, n);
    return hipGetLastError();
}
// Histogram of row lengths in buckets 0, 1, 2..3, 4..7, ... (bucket b > 0
// holds lengths in [2^(b-1), 2^b)); kDegBuckets u64 counters, arcs per
// bucket in the next kDegBuckets.
__global__ void degree_hist_k(const uint64_t *rp, uint32_t n, u64 *hist) {
    __shared__ u64 h[2 * kDegBuckets];
    for (uint32_t i = threadIdx.x; i < 2 * kDegBuckets; i += blockDim.x) h[i] = 0;
    __syncthreads();
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const uint64_t d = rp[v + 1] - rp[v];
        const int b = d == 0 ? 0 : min(kDegBuckets - 1, 64 - __clzll((long long)d));
        atomicAdd(&h[b], 1ull);
        atomicAdd(&h[kDegBuckets + b], (u64)d);
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < 2 * kDegBuckets; i += blockDim.x)
        if (h[i]) atomicAdd(&hist[i], h[i]);
}

hipError_t launch_degree_hist(const uint64_t *rp, uint32_t n, u64 *hist, hipStream_t s) {
    if (n == 0) return hipSuccess;
    degree_hist_k<<<grid_for(n, 256, 1024), 256, 0, s>>>(rp, n, hist);
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
hipError_t launch_check_labels(const uint32_t *labels, uint32_t n, uint32_t *err, hipStream_t s) {
    if (n == 0) return hipSuccess;
    check_labels_k<<<grid_for(n, 256, 4096), 256, 0, s>>>(labels, n, err);
    return hipGetLastError();
}

// -------------------------------------------------------------- binning --

constexpr uint32_t kBinVerts = 1024;

uint32_t bin_blocks(uint32_t n) { return (n + kBinVerts - 1) / kBinVerts; }

__device__ __forceinline__ int bin_of(uint64_t d, const BinCfg &c) {
    return d == 0 ? BIN_ZERO
           : d <= c.tmax ? BIN_THREAD
           : d <= c.gmax ? BIN_GROUP
           : d <= c.wmax ? BIN_WAVE
           : d <= c.xmax ? BIN_WIDE
                         : BIN_HUB;
}

// Bins of the four vertices blockIdx.x * kBinVerts + i * 256 + threadIdx.x
// (-1 past the last vertex or when the vertex's row_ptr entries are
// malformed) and their degrees.  The eight row_ptr loads are issued before
// any is used: rows past the last vertex read the last row's bounds.
__device__ __forceinline__ void vertex_bins4(const Graph &g, const BinCfg &c, int (&bins)[4], uint64_t (&degs)[4],
                                             bool &bad_any) {
    uint64_t ra[4], rb[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t v = blockIdx.x * kBinVerts + i * 256 + threadIdx.x;
        const uint32_t vc = v < g.n ? v : g.n - 1;
        ra[i] = g.rp[vc];
        rb[i] = g.rp[vc + 1];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t v = blockIdx.x * kBinVerts + i * 256 + threadIdx.x;
        const uint64_t a = ra[i], b = rb[i];
        const bool bad = (b < a) || (b > g.m) || (v == 0 && a != 0) || (v + 1 == g.n && b != g.m);
        const bool in = v < g.n;
        bad_any |= in && bad;
        degs[i] = (in && !bad) ? b - a : 0;
        bins[i] = (in && !bad) ? bin_of(degs[i], c) : -1;
    }
}

__global__ __launch_bounds__(256) void bin_count_k(Graph g, BinCfg cfg, uint32_t *blk_counts, u64 *blk_arcs,
                                                   uint32_t nblk, uint32_t *err) {
    __shared__ uint32_t cnt[NBINS];
    __shared__ u64 arcs[NBINS];
    if (threadIdx.x < NBINS) {
        cnt[threadIdx.x] = 0;
        arcs[threadIdx.x] = 0;
    }
    __syncthreads();
    u64 my_arcs[NBINS];
    uint32_t my_cnt[NBINS];
#pragma unroll
    for (int b = 0; b < NBINS; ++b) {
        my_arcs[b] = 0;
        my_cnt[b] = 0;
    }
    bool bad_any = false;
    int bins[4];
    uint64_t degs[4];
    vertex_bins4(g, cfg, bins, degs, bad_any);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int b = 0; b < NBINS; ++b)
            if (bins[i] == b) {
                my_cnt[b] += 1;
                my_arcs[b] += degs[i];
            }
    if (bad_any) atomicOr(err, ERR_ROWPTR);
#pragma unroll
    for (int b = 0; b < NBINS; ++b) {
        const uint32_t c = wave_sum(my_cnt[b]);
        const u64 s = wave_sum(my_arcs[b]);
        if ((threadIdx.x & 63) == 0) {
            if (c) atomicAdd(&cnt[b], c);
            if (s) atomicAdd(&arcs[b], s);
        }
    }
    __syncthreads();
    if (threadIdx.x < NBINS) {
        blk_counts[threadIdx.x * nblk + blockIdx.x] = cnt[threadIdx.x];
        blk_arcs[threadIdx.x * nblk + blockIdx.x] = arcs[threadIdx.x];
    }
}

// Exclusive prefix sums of the per-block counts and arc counts of one bin
// (blockIdx.x), in one block of 1024 threads per bin, and the bin's totals;
// bin_scatter_k adds the totals of the bins before it.  Wavefront w owns a
// contiguous run of whole 64-entry chunks and reads it coalesced, kScanJ
// chunks per step with their loads issued together (the counts were written
// by other CUs, so each load goes to the memory side); pass 1 sums each
// wavefront's run, pass 2 scans it chunk by chunk from the wavefront's offset.
constexpr int kScanJ = 8;
__global__ __launch_bounds__(1024) void bin_scan_k(uint32_t *blk_counts, u64 *blk_arcs, uint32_t nblk,
                                                   uint32_t *totals, u64 *arc_totals) {
    __shared__ uint32_t wtot[16];
    __shared__ u64 watot[16];
    const uint32_t t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const uint32_t b = blockIdx.x;
    const uint32_t chunks = (nblk + 63) / 64;
    const uint32_t cpw = (chunks + 15) / 16;
    const uint32_t lo = min(wave * cpw * 64, nblk), hi = min(lo + cpw * 64, nblk);
    uint32_t *cnt = blk_counts + (size_t)b * nblk;
    u64 *arc = blk_arcs + (size_t)b * nblk;
    uint32_t x = 0;
    u64 y = 0;
    for (uint32_t i0 = lo; i0 < hi; i0 += 64 * kScanJ) {
        uint32_t xs[kScanJ];
        u64 ys[kScanJ];
#pragma unroll
        for (int j = 0; j < kScanJ; ++j) {
            const uint32_t i = i0 + 64u * j + lane;
            const uint32_t ic = i < hi ? i : lo;  // lo < hi here: an entry of this run
            xs[j] = cnt[ic];
            ys[j] = arc[ic];
        }
#pragma unroll
        for (int j = 0; j < kScanJ; ++j)
            if (i0 + 64u * j + lane < hi) {
                x += xs[j];
                y += ys[j];
            }
    }
    x = wave_sum(x);
    y = wave_sum(y);
    if (lane == 0) {
        wtot[wave] = x;
        watot[wave] = y;
    }
    __syncthreads();
    uint32_t run = 0, total = 0;
    u64 arun = 0, atotal = 0;
    for (uint32_t w = 0; w < 16; ++w) {
        if (w < wave) {
            run += wtot[w];
            arun += watot[w];
        }
        total += wtot[w];
        atotal += watot[w];
    }
    for (uint32_t i0 = lo; i0 < hi; i0 += 64 * kScanJ) {
        uint32_t xs[kScanJ];
        u64 ys[kScanJ];
#pragma unroll
        for (int j = 0; j < kScanJ; ++j) {
            const uint32_t i = i0 + 64u * j + lane;
            const uint32_t ic = i < hi ? i : lo;
            const uint32_t xv = cnt[ic];
            const u64 yv = arc[ic];
            xs[j] = i < hi ? xv : 0u;
            ys[j] = i < hi ? yv : 0ull;
        }
#pragma unroll
        for (int j = 0; j < kScanJ; ++j) {
            uint32_t xi = xs[j];
            u64 yi = ys[j];
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const uint32_t xu = __shfl_up(xi, off, 64);
                const u64 yu = __shfl_up(yi, off, 64);
                if ((int)lane >= off) {
                    xi += xu;
                    yi += yu;
                }
            }
            const uint32_t i = i0 + 64u * j + lane;
            if (i < hi) {
                cnt[i] = run + xi - xs[j];
                arc[i] = arun + yi - ys[j];
            }
            run += (uint32_t)__shfl((int)xi, 63, 64);
            arun += __shfl(yi, 63, 64);
        }
    }
    if (t == 0) {
        totals[b] = total;
        arc_totals[b] = atotal;
    }
}

// Internal id, internal row start and the two id maps.
__global__ __launch_bounds__(256) void bin_scatter_k(Graph g, BinCfg cfg, const uint32_t *blk_offsets,
                                                     const u64 *blk_arc_offsets, const uint32_t *totals,
                                                     const u64 *arc_totals, uint32_t nblk, uint32_t *old_of,
                                                     uint32_t *new_of, uint64_t *rp2) {
    __shared__ uint32_t wcnt[4][NBINS];
    __shared__ u64 warc[4][NBINS];
    __shared__ uint32_t run[NBINS];
    __shared__ u64 arun[NBINS];
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // the four vertices' row bounds are loaded before the first barrier
    // (malformed rows were reported by bin_count_k)
    int bins[4];
    uint64_t degs[4];
    bool bad_any = false;
    vertex_bins4(g, cfg, bins, degs, bad_any);
    if (threadIdx.x < NBINS) {
        // offsets inside the bin, plus the totals of the bins before it
        uint32_t tb[NBINS];
        u64 ab[NBINS];
#pragma unroll
        for (int b = 0; b < NBINS; ++b) {
            tb[b] = totals[b];
            ab[b] = arc_totals[b];
        }
        uint32_t base = blk_offsets[(size_t)threadIdx.x * nblk + blockIdx.x];
        u64 abase = blk_arc_offsets[(size_t)threadIdx.x * nblk + blockIdx.x];
#pragma unroll
        for (int b = 0; b < NBINS; ++b)
            if ((uint32_t)b < threadIdx.x) {
                base += tb[b];
                abase += ab[b];
            }
        run[threadIdx.x] = base;
        arun[threadIdx.x] = abase;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t v = blockIdx.x * kBinVerts + i * 256 + threadIdx.x;
        const int bin = bins[i];
        const uint64_t d = degs[i];
        uint32_t rank = 0;
        u64 aex = 0;
#pragma unroll
        for (int b = 0; b < NBINS; ++b) {
            const u64 mask = __ballot(bin == b);
            const u64 x0 = bin == b ? (u64)d : 0ull;
            const u64 x = wave_scan_incl64(x0);
            if (lane == 63) warc[wave][b] = x;
            if (lane == 0) wcnt[wave][b] = (uint32_t)__popcll(mask);
            if (bin == b) {
                rank = (uint32_t)__popcll(mask & ((1ull << lane) - 1));
                aex = x - x0;
            }
        }
        __syncthreads();
        if (bin >= 0) {
            uint32_t off = run[bin];
            u64 aoff = arun[bin];
            for (uint32_t w = 0; w < wave; ++w) {
                off += wcnt[w][bin];
                aoff += warc[w][bin];
            }
            old_of[off + rank] = v;
            new_of[v] = off + rank;
            rp2[off + rank] = aoff + aex;
        }
        __syncthreads();
        if (threadIdx.x < NBINS) {
            const int b = threadIdx.x;
            run[b] += wcnt[0][b] + wcnt[1][b] + wcnt[2][b] + wcnt[3][b];
            arun[b] += warc[0][b] + warc[1][b] + warc[2][b] + warc[3][b];
        }
        __syncthreads();
    }
}

hipError_t launch_bin_count(const Graph &g, const BinCfg &cfg, uint32_t *blk_counts, u64 *blk_arcs, uint32_t nblk,
                            uint32_t *err, hipStream_t s) {
    bin_count_k<<<nblk, 256, 0, s>>>(g, cfg, blk_counts, blk_arcs, nblk, err);
    return hipGetLastError();
}
hipError_t launch_bin_scan(uint32_t *blk_counts, u64 *blk_arcs, uint32_t nblk, uint32_t *totals, u64 *arc_totals,
                           hipStream_t s) {
    bin_scan_k<<<NBINS, 1024, 0, s>>>(blk_counts, blk_arcs, nblk, totals, arc_totals);
    return hipGetLastError();
}
hipError_t launch_bin_scatter(const Graph &g, const BinCfg &cfg, const uint32_t *blk_offsets,
                              const u64 *blk_arc_offsets, const uint32_t *totals, const u64 *arc_totals,
                              uint32_t nblk, uint32_t *old_of, uint32_t *new_of, uint64_t *rp2, hipStream_t s) {
    bin_scatter_k<<<nblk, 256, 0, s>>>(g, cfg, blk_offsets, blk_arc_offsets, totals, arc_totals, nblk, old_of,
                                       new_of, rp2);
    return hipGetLastError();
}

// ----------------------------------------------------------- long rows --
//
// Work layout of the long rows (internal ids 0..H-1), planned on the device:
// per row d arcs, ceil(d/512) wavefront segments (HubItem), a slab of
// pow2(2d) slots, a touched list of d entries, ceil(d/2048) reduce items,
// and a merge class (one wavefront for <= kMergeWaveSegs segments, one block
// up to merge_max, else HUB_BIG: always through the slab).

// Exclusive scan of one value per thread of a 1024-thread block; returns
// the prefix and adds the block total to *carry (all threads see it).
__device__ __forceinline__ u64 block_scan_1024(u64 x, u64 *wtot, u64 &carry) {
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    u64 inc = x;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const u64 y = __shfl_up(inc, off, 64);
        if ((int)lane >= off) inc += y;
    }
    if (lane == 63) wtot[wave] = inc;
    __syncthreads();
    u64 before = 0, total = 0;
    for (uint32_t q = 0; q < 16; ++q) {
        if (q < wave) before += wtot[q];
        total += wtot[q];
    }
    const u64 res = carry + before + inc - x;
    __syncthreads();
    carry += total;
    return res;
}

// Per long row h: arcs d, segments, slab slots, reduce items, merge class.
struct HubRow {
    u64 d, nseg, slots, red, mw, mb;
};
__device__ __forceinline__ HubRow hub_row(const uint64_t *rp2, uint32_t h, uint32_t merge_max) {
    HubRow r;
    r.d = rp2[h + 1] - rp2[h];
    r.nseg = (r.d + kWaveArcs - 1) / kWaveArcs;
    r.slots = 1;
    while (r.slots < 2 * r.d) r.slots <<= 1;
    r.red = (r.d + 2047) / 2048;
    const bool big = r.nseg > merge_max;
    r.mw = !big && r.nseg <= (u64)kMergeWaveSegs;
    r.mb = !big && !r.mw;
    return r;
}

// Block sums of the six per-row quantities (1024 rows per block).
__global__ __launch_bounds__(1024) void hub_count_k(const uint64_t *rp2, uint32_t H, uint32_t merge_max,
                                                    u64 *blk) {
    __shared__ u64 wt[16][6];
    const uint32_t h = blockIdx.x * 1024 + threadIdx.x, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    HubRow r{0, 0, 0, 0, 0, 0};
    if (h < H) r = hub_row(rp2, h, merge_max);
    u64 x[6] = {r.nseg, r.slots, r.d, r.red, r.mw, r.mb};
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        x[k] = wave_sum(x[k]);
        if (lane == 0) wt[wave][k] = x[k];
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        u64 s = 0;
        for (int q = 0; q < 16; ++q) s += wt[q][threadIdx.x];
        blk[(size_t)blockIdx.x * 6 + threadIdx.x] = s;
    }
}

// Exclusive scan of the block sums (in place) and the totals.
__global__ __launch_bounds__(1024) void hub_scan_k(u64 *blk, uint32_t nb, u64 *out) {
    __shared__ u64 wtot[16];
    for (int k = 0; k < 6; ++k) {
        u64 carry = 0;
        for (uint32_t base = 0; base < nb; base += 1024) {
            const uint32_t b = base + threadIdx.x;
            const u64 x = b < nb ? blk[(size_t)b * 6 + k] : 0;
            const u64 p = block_scan_1024(x, wtot, carry);
            if (b < nb) blk[(size_t)b * 6 + k] = p;
        }
        if (threadIdx.x == 0) out[k] = carry;
    }
}

// Offsets, segments, reduce items, flags, slab masks and merge lists of
// every long row.  A block's segment and reduce items are written by all its
// threads together (item k of the block goes to the row whose prefix is the
// last one <= k), since one row can hold thousands of them.
__device__ __forceinline__ uint32_t last_at_most(const uint32_t *pre, uint32_t k) {
    uint32_t j = 0;
#pragma unroll
    for (uint32_t step = 512; step >= 1; step >>= 1)
        if (pre[j + step] <= k) j += step;
    return j;  // the largest j <= 1023 with pre[j] <= k (pre[0] = 0, pre nondecreasing)
}

__global__ __launch_bounds__(1024) void hub_fill_k(const uint64_t *rp2, uint32_t H, uint32_t merge_max,
                                                   const u64 *blk, const u64 *tot, uint32_t *item_lo,
                                                   uint64_t *slab_off, uint64_t *touched_off, HubItem *items,
                                                   ReduceItem *ritems, uint32_t *hflags, uint32_t *slab_mask,
                                                   uint32_t *mrows) {
    __shared__ u64 wtot[16];
    __shared__ uint32_t ipre[1025], rpre[1025];  // the block's item and reduce-item prefixes
    const uint32_t h0 = blockIdx.x * 1024, h = h0 + threadIdx.x;
    HubRow r{0, 0, 0, 0, 0, 0};
    if (h < H) r = hub_row(rp2, h, merge_max);
    u64 c0 = blk[(size_t)blockIdx.x * 6 + 0], c1 = blk[(size_t)blockIdx.x * 6 + 1], c2 = blk[(size_t)blockIdx.x * 6 + 2];
    u64 c3 = blk[(size_t)blockIdx.x * 6 + 3], c4 = blk[(size_t)blockIdx.x * 6 + 4], c5 = blk[(size_t)blockIdx.x * 6 + 5];
    const u64 ibase = c0, rbase = c3;
    const u64 pi = block_scan_1024(r.nseg, wtot, c0);
    const u64 ps = block_scan_1024(r.slots, wtot, c1);
    const u64 pt = block_scan_1024(r.d, wtot, c2);
    const u64 pr = block_scan_1024(r.red, wtot, c3);
    const u64 pw = block_scan_1024(r.mw, wtot, c4);
    const u64 pb = block_scan_1024(r.mb, wtot, c5);
    ipre[threadIdx.x] = (uint32_t)(pi - ibase);
    rpre[threadIdx.x] = (uint32_t)(pr - rbase);
    if (threadIdx.x == 0) {
        ipre[1024] = (uint32_t)(c0 - ibase);
        rpre[1024] = (uint32_t)(c3 - rbase);
    }
    if (h < H) {
        item_lo[h] = (uint32_t)pi;
        if (h == H - 1) item_lo[H] = (uint32_t)tot[0];
        slab_off[h] = ps;
        touched_off[h] = pt;
        hflags[h] = (!r.mw && !r.mb) ? HUB_BIG : 0u;
        slab_mask[h] = (uint32_t)(r.slots - 1);
        if (r.mw)
            mrows[pw] = h;
        else if (r.mb)
            mrows[tot[4] + pb] = h;
    }
    __syncthreads();
    const uint32_t ni = (uint32_t)(c0 - ibase), nr = (uint32_t)(c3 - rbase);
    for (uint32_t k = threadIdx.x; k < ni; k += 1024) {
        const uint32_t j = last_at_most(ipre, k);
        const uint64_t b = rp2[h0 + j], e = rp2[h0 + j + 1];
        const uint64_t x = b + (uint64_t)(k - ipre[j]) * kWaveArcs;
        items[ibase + k] = HubItem{h0 + j, 0, x, min(e, x + (uint64_t)kWaveArcs)};
    }
    for (uint32_t k = threadIdx.x; k < nr; k += 1024) {
        const uint32_t j = last_at_most(rpre, k);
        const uint64_t d = rp2[h0 + j + 1] - rp2[h0 + j];
        const uint64_t t = (uint64_t)(k - rpre[j]) * 2048;
        ritems[rbase + k] = ReduceItem{h0 + j, (uint32_t)t, (uint32_t)min(d, t + 2048), 0};
    }
}

hipError_t launch_hub_plan(const uint64_t *rp2, uint32_t H, uint32_t merge_max, u64 *blk, u64 *out, hipStream_t s) {
    const uint32_t nb = (H + 1023) / 1024;
    hub_count_k<<<nb, 1024, 0, s>>>(rp2, H, merge_max, blk);
    hub_scan_k<<<1, 1024, 0, s>>>(blk, nb, out);
    return hipGetLastError();
}

hipError_t launch_hub_fill(const uint64_t *rp2, uint32_t H, uint32_t merge_max, const u64 *blk, const u64 *out,
                           uint32_t *item_lo, uint64_t *slab_off, uint64_t *touched_off, HubItem *items,
                           ReduceItem *ritems, uint32_t *hflags, uint32_t *slab_mask, uint32_t *mrows, hipStream_t s) {
    if (H == 0) return hipSuccess;
    hub_fill_k<<<(H + 1023) / 1024, 1024, 0, s>>>(rp2, H, merge_max, blk, out, item_lo, slab_off, touched_off, items,
                                                   ritems, hflags, slab_mask, mrows);
    return hipGetLastError();
}

// ------------------------------------------------------------- relabel --

struct RelabelArgs {
    Graph g;  // caller's CSR
    const uint32_t *old_of;
    const uint32_t *new_of;
    const uint64_t *rp2;
    uint32_t *col2;
    uint32_t *w2;
    uint32_t *err;
    // round 1 from the unique labels, done while the rows are copied: a
    // row that lists each neighbour once sees every label (= the
    // neighbour's id) once, so its vote is the max of (weight, -id) over the
    // row and its own id with the self weight; NULL L1 = not done here
    uint32_t *L1;       // round-1 labels (internal index)
    u64 *changed;       // round-1 changed counter words
    uint32_t sw;
    HubState hs;        // long rows: best / own_sum / flags / rowsum
    // rows this pass does not vote go to the round-1 lists (Round1Fuse)
    uint32_t *rest_list, *rest_n;
    uint32_t lo, split;
    int bin_a, bin_b;
};

// Queue internal row r, which the pass could not vote, for round 1.
__device__ __forceinline__ void queue_rest(const RelabelArgs &a, uint32_t r) {
    if (!a.rest_list) return;
    const bool first = r < a.split;
    const uint32_t k = atomicAdd(&a.rest_n[first ? a.bin_a : a.bin_b], 1u);
    a.rest_list[(first ? a.lo : a.split) + k] = r;
}

// Round-1 key of the arcs a lane holds (labels = original ids).
template <int A>
__device__ __forceinline__ void round1_keys(const uint32_t (&u)[A], const uint32_t (&wv)[A], uint32_t nvalid_mask,
                                            uint32_t v, u64 &best, u64 &own_w, uint32_t &own_hit, u64 &rs) {
#pragma unroll
    for (int j = 0; j < A; ++j)
        if (nvalid_mask >> j & 1u) {
            rs += wv[j];
            if (u[j] == v) {
                own_w += wv[j];
                own_hit = 1;
            } else {
                best = umax64(best, vote_key(kStrict, u[j], wv[j]));
            }
        }
}

// Rows of at most 32 arcs, one lane each.
__global__ __launch_bounds__(256) void relabel_thread_k(RelabelArgs a, uint8_t *rowflag, uint32_t lo,
                                                        uint32_t cnt) {
    u64 chg = 0;
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < cnt; i += gridDim.x * 256) {
        const uint32_t r = lo + i;
        const uint32_t v = a.old_of[r];
        const uint64_t src = a.g.rp[v], e = a.g.rp[v + 1];
        const uint64_t dst = a.rp2[r];
        uint32_t prev = 0, distinct = 1;
        bool bad = false;
        u64 best = 0, own_w = 0, rs = 0;
        uint32_t own_hit = 0;
        // 8 arcs at a time, every load issued unconditionally (arcs past the
        // row read the row's first arc and are masked) so the id lookups of
        // a chunk are in flight together
        for (uint64_t k = src; k < e; k += 8) {
            uint32_t u[8], wv[8], mk = 0;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const bool in = k + j < e;
                mk |= (uint32_t)in << j;
                const uint32_t x = a.g.col[in ? k + j : src];
                u[j] = in ? x : 0u;
            }
            if (a.g.w) {
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const uint32_t x = a.g.w[(mk >> j & 1u) ? k + j : src];
                    wv[j] = (mk >> j & 1u) ? x : 0u;
                }
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j) wv[j] = mk >> j & 1u;
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                bad |= u[j] >= a.g.n;
                if ((mk >> j & 1u) && k + j > src && !(prev < u[j])) distinct = 0;
                if (mk >> j & 1u) prev = u[j];
                u[j] = u[j] >= a.g.n ? 0u : u[j];
            }
            uint32_t nid[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) nid[j] = a.new_of[u[j]];
#pragma unroll
            for (int j = 0; j < 8; ++j)
                if (mk >> j & 1u) {
                    a.col2[dst + (k + j - src)] = nid[j];
                    if (a.w2) a.w2[dst + (k + j - src)] = wv[j];
                }
            if (a.L1) round1_keys<8>(u, wv, mk, v, best, own_w, own_hit, rs);
        }
        if (bad) atomicOr(a.err, ERR_COL);
        rowflag[r] = distinct ? ROW_DISTINCT : 0;
        if (a.L1 && distinct) {
            if (own_hit || a.sw) best = umax64(best, vote_key(kStrict, v, own_w + a.sw));
            const uint32_t nl = best ? key_label(kStrict, best) : v;
            a.L1[r] = nl;
            chg += nl != v;
            if (rs + a.sw > 0xFFFFFFFFull) atomicOr(a.err, ERR_WOVF);
        } else if (a.L1) {
            queue_rest(a, r);
        }
    }
    if (a.L1) block_count(chg, a.changed);
}

// Copy arcs [b0, b0 + len) of internal row r (one wavefront, 1 <= len <= 512
// arcs) from the caller's row of old_of[r]; returns 1 if they are strictly
// increasing (also across the segment's first boundary inside the row).
// Every load is issued by every lane (lanes past the segment read its first
// arc and are masked), so the 8 id lookups per lane are in flight together
// instead of one after the other.
//
// SCAN (long rows copied slice by slice): the ids are not looked up here;
// instead bnd[0..S] receive where each slice of the caller's id space starts
// in the segment (bnd[S] = len), or bnd[0] = kSliceNone when the segment is
// not sorted, and *src_out the segment's first arc in the caller's CSR.
template <int A = kWaveArcs / 64, bool SCAN = false>
__device__ __forceinline__ uint32_t relabel_segment(const RelabelArgs &a, uint32_t r, uint64_t b0, uint64_t len,
                                                    u64 &best, u64 &own_w, uint32_t &own_hit, u64 &wsum,
                                                    uint16_t *bnd = nullptr, uint32_t S = 0,
                                                    uint64_t *src_out = nullptr) {
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t v = a.old_of[r];
    const uint64_t rs = a.g.rp[v];
    const uint64_t off = b0 - a.rp2[r];  // offset of the segment inside the row
    const uint64_t src = rs + off;
    uint32_t u[A], wv[A];
    uint32_t m = 0;
#pragma unroll
    for (int j = 0; j < A; ++j) {
        const uint64_t k = lane + 64ull * j;
        const bool in = k < len;
        m |= (uint32_t)in << j;
        const uint32_t x = a.g.col[src + (in ? k : 0)];
        u[j] = in ? x : 0u;
    }
    if (a.g.w) {
#pragma unroll
        for (int j = 0; j < A; ++j) {
            const uint64_t k = lane + 64ull * j;
            const uint32_t x = a.g.w[src + ((m >> j & 1u) ? k : 0)];
            wv[j] = (m >> j & 1u) ? x : 0u;
        }
    } else {
#pragma unroll
        for (int j = 0; j < A; ++j) wv[j] = m >> j & 1u;
    }
    // the arc before the segment (the row's previous segment), for the order test
    const uint32_t before = a.g.col[src > rs ? src - 1 : src];
    bool bad = false;
#pragma unroll
    for (int j = 0; j < A; ++j) bad |= (m >> j & 1u) && u[j] >= a.g.n;
    if (bad) atomicOr(a.err, ERR_COL);
    // strictly increasing: compare each arc with the one before it (the lane
    // below, or lane 63 of the previous column, or the arc before the segment)
    uint32_t ok = 1, sorted_in = 1;
    uint32_t prev[A];  // the arc before each one inside the segment (SCAN)
#pragma unroll
    for (int j = 0; j < A; ++j) {
        const uint32_t up = __shfl_up(u[j], 1, 64);
        const uint32_t wrap = j ? __shfl(u[j ? j - 1 : 0], 63, 64) : before;
        const uint32_t pv = lane ? up : wrap;
        const uint64_t k = lane + 64ull * j;
        const bool has_prev = k > 0 || src > rs;
        if ((m >> j & 1u) && has_prev && !(pv < u[j])) ok = 0;
        if ((m >> j & 1u) && k > 0 && pv > u[j]) sorted_in = 0;
        prev[j] = pv;
    }
#pragma unroll
    for (int j = 0; j < A; ++j) u[j] = u[j] >= a.g.n ? 0u : u[j];
    if (!SCAN) {
        uint32_t nid[A];
#pragma unroll
        for (int j = 0; j < A; ++j) nid[j] = a.new_of[u[j]];
#pragma unroll
        for (int j = 0; j < A; ++j) {
            const uint64_t k = lane + 64ull * j;
            if (m >> j & 1u) {
                a.col2[b0 + k] = nid[j];
                if (a.w2) a.w2[b0 + k] = wv[j];
            }
        }
    } else {
        if (a.w2) {
#pragma unroll
            for (int j = 0; j < A; ++j)
                if (m >> j & 1u) a.w2[b0 + lane + 64ull * j] = wv[j];
        }
        if (lane == 0) *src_out = src;
        if (__ballot(!sorted_in) == 0) {
            // each slice's first arc: arc k opens the slices after its
            // predecessor's up to its own; the last arc closes the rest
#pragma unroll
            for (int j = 0; j < A; ++j) {
                const uint32_t k = lane + 64u * j;
                if (!(m >> j & 1u)) continue;
                const uint32_t sl = u[j] >> kSliceShift;
                const uint32_t p = prev[j] < a.g.n ? prev[j] : 0u;
                const uint32_t s0 = k ? (p >> kSliceShift) + 1 : 0u;
                for (uint32_t s = s0; s <= sl && s <= S; ++s) bnd[s] = (uint16_t)k;
                if (k + 1 == len)
                    for (uint32_t s = sl + 1; s <= S; ++s) bnd[s] = (uint16_t)len;
            }
        } else if (lane == 0) {
            bnd[0] = kSliceNone;
        }
    }
    if (a.L1) {
        round1_keys<A>(u, wv, m, v, best, own_w, own_hit, wsum);
        best = wave_max64(best);
        own_w = wave_sum(own_w);
        own_hit = __ballot(own_hit != 0) != 0;
        wsum = wave_sum(wsum);
    }
    return __ballot(!ok) == 0 ? 1u : 0u;
}

// Rows of 33..512 arcs, one wavefront each.
// A arcs per lane: 8 for rows of up to 512 arcs, 2 for rows of up to 128
// (every lane issues all A loads, so a small A keeps short rows cheap).
template <int A>
__global__ __launch_bounds__(256) void relabel_wave_k(RelabelArgs a, uint8_t *rowflag, uint32_t lo, uint32_t cnt) {
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    u64 chg = 0;
    for (uint32_t i = blockIdx.x * 4 + wave; i < cnt; i += gridDim.x * 4) {
        const uint32_t r = lo + i;
        const uint64_t b0 = a.rp2[r], b1 = a.rp2[r + 1];
        u64 best = 0, own_w = 0, rs = 0;
        uint32_t own_hit = 0;
        const uint32_t ok = relabel_segment<A>(a, r, b0, b1 - b0, best, own_w, own_hit, rs);
        if ((threadIdx.x & 63) == 0) {
            rowflag[r] = ok ? ROW_DISTINCT : 0;
            if (a.L1 && ok) {
                const uint32_t v = a.old_of[r];
                if (own_hit || a.sw) best = umax64(best, vote_key(kStrict, v, own_w + a.sw));
                const uint32_t nl = best ? key_label(kStrict, best) : v;
                a.L1[r] = nl;
                chg += nl != v;
                if (rs + a.sw > 0xFFFFFFFFull) atomicOr(a.err, ERR_WOVF);
            } else if (a.L1) {
                queue_rest(a, r);
            }
        }
    }
    if (a.L1) block_count(chg, a.changed);
}

// Long rows: one wavefront per work item; a segment with a repeated or
// decreasing id marks the row HUB_REPEATS.
__global__ __launch_bounds__(256) void relabel_hub_k(RelabelArgs a, const HubItem *__restrict__ items,
                                                     uint32_t count, uint32_t *hub_flags) {
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (uint32_t it = blockIdx.x * 4 + wave; it < count; it += gridDim.x * 4) {
        const HubItem item = items[it];
        u64 best = 0, own_w = 0, rs = 0;
        uint32_t own_hit = 0;
        const uint32_t ok = relabel_segment(a, item.r, item.b0, item.b1 - item.b0, best, own_w, own_hit, rs);
        if ((threadIdx.x & 63) == 0) {
            if (!ok) {
                atomicOr(&hub_flags[item.r], HUB_REPEATS);
                if (a.L1) atomicAdd(a.hs.repeats, 1u);
            }
            if (a.L1) {  // the row's round-1 partials, as the direct long-row vote gathers them
                const uint32_t h = item.r;
                if (best) atomicMax(&a.hs.best[h], best);
                if (own_w) atomicAdd(&a.hs.own_sum[h], own_w);
                if (own_hit) atomicOr(&a.hs.flags[h], HUB_OWN_SEEN);
                atomicAdd(&a.hs.rowsum[h], rs);
            }
        }
    }
}

// ---------------------------------------------- long rows, slice by slice --
//
// The long rows hold most arcs, and their relabel is a random 4-byte gather
// into the n-entry id map (64 MB at 2^24 vertices), which runs at the memory
// system's random-request rate.  Taken slice by slice of the caller's id
// space (4 MB of the map per slice) the same gathers mostly hit L2: the scan pass
// (relabel_segment in SCAN mode, one wavefront per 512-arc segment) checks
// the segment, votes round 1 (whose labels are the caller's ids themselves)
// and records where each slice starts in it, as the segment is sorted; then
// one launch ordered slice-major copies the segments' arcs of one slice at a
// time (relabel_hub_slices_k), and the blocks after the last slice copy the
// segments that are not sorted the direct way.
__global__ __launch_bounds__(256) void relabel_hub_scan_k(RelabelArgs a, const HubItem *__restrict__ items,
                                                          uint32_t count, uint32_t *hub_flags, uint32_t S,
                                                          uint16_t *bnd, uint64_t *isrc) {
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (uint32_t it = blockIdx.x * 4 + wave; it < count; it += gridDim.x * 4) {
        const HubItem item = items[it];
        u64 best = 0, own_w = 0, rs = 0;
        uint32_t own_hit = 0;
        const uint32_t ok = relabel_segment<kWaveArcs / 64, true>(a, item.r, item.b0, item.b1 - item.b0, best, own_w,
                                                                  own_hit, rs, bnd + (size_t)it * (S + 1), S,
                                                                  isrc + it);
        if ((threadIdx.x & 63) == 0) {
            if (!ok) {
                atomicOr(&hub_flags[item.r], HUB_REPEATS);
                if (a.L1) atomicAdd(a.hs.repeats, 1u);
            }
            if (a.L1) {
                const uint32_t h = item.r;
                if (best) atomicMax(&a.hs.best[h], best);
                if (own_w) atomicAdd(&a.hs.own_sum[h], own_w);
                if (own_hit) atomicOr(&a.hs.flags[h], HUB_OWN_SEEN);
                atomicAdd(&a.hs.rowsum[h], rs);
            }
        }
    }
}

// The copy: one wavefront per 64 segments and one slice.  Lane l takes
// segment l's arcs of the slice; the wavefront then copies the 64 ranges as
// one flattened list (an exclusive scan of their lengths), 4 x 64 arcs per
// step with all their loads in flight, each lane finding the range of its
// arc by a binary search over the lanes' offsets.
constexpr uint32_t kSliceItems = 256;  // segments per block (4 wavefronts x 64)
__global__ __launch_bounds__(256) void relabel_hub_slices_k(RelabelArgs a, const HubItem *__restrict__ items,
                                                            uint32_t count, uint32_t S,
                                                            const uint16_t *__restrict__ bnd,
                                                            const uint64_t *__restrict__ isrc) {
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t per_slice = (count + kSliceItems - 1) / kSliceItems;
    const uint32_t s = blockIdx.x / per_slice;  // slice-major: blocks start in order
    const uint32_t it = (blockIdx.x - s * per_slice) * kSliceItems + wave * 64 + lane;
    uint32_t k0 = 0, k1 = 0;
    uint64_t src = 0, dst = 0;
    if (it < count) {
        const uint16_t *bi = bnd + (size_t)it * (S + 1);
        const HubItem item = items[it];
        const uint32_t len = (uint32_t)(item.b1 - item.b0);
        const bool unsorted = bi[0] == kSliceNone;
        if (s < S) {  // this slice's arcs of a sorted segment
            if (!unsorted) {
                // clamped: with an id out of range (reported by the scan)
                // the boundaries need not be consistent
                k1 = bi[s + 1] < len ? bi[s + 1] : len;
                k0 = bi[s] < k1 ? bi[s] : k1;
            }
        } else if (unsorted) {  // after the last slice: whole unsorted segments
            k1 = len;
        }
        src = isrc[it] + k0;
        dst = item.b0 + k0;
    }
    const uint32_t c = k1 - k0;
    uint32_t incl = c;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(incl, off, 64);
        if ((int)lane >= off) incl += y;
    }
    const uint32_t excl = incl - c;
    const uint32_t T = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
    const uint32_t *__restrict__ col = a.g.col;
    const uint32_t *__restrict__ nmap = a.new_of;
    uint32_t *__restrict__ out = a.col2;
    for (uint32_t t0 = 0; t0 < T; t0 += 256) {
        uint64_t from[4], to[4];
        bool in[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t t = t0 + 64u * q + lane;
            in[q] = t < T;
            const uint32_t tc = in[q] ? t : 0u;  // T > 0: arc 0 exists
            uint32_t lo = 0, hi = 64;            // the last lane whose range starts at or before tc
#pragma unroll
            for (int step = 0; step < 6; ++step) {
                const uint32_t mid = (lo + hi) >> 1;
                if ((uint32_t)__shfl((int)excl, (int)mid, 64) <= tc)
                    lo = mid;
                else
                    hi = mid;
            }
            const uint32_t d = tc - (uint32_t)__shfl((int)excl, (int)lo, 64);
            from[q] = __shfl(src, (int)lo, 64) + d;
            to[q] = __shfl(dst, (int)lo, 64) + d;
        }
        uint32_t x[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) x[q] = col[from[q]];
        uint32_t y[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) y[q] = nmap[x[q] < a.g.n ? x[q] : 0u];  // a bad id was reported by the scan
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (in[q]) out[to[q]] = y[q];
    }
}

// Rows whose segments turned out not to list each neighbour once are voted
// by the regular round-1 kernels: drop the partials the copy gathered.
__global__ void hub_unfuse_k(HubState hs, uint32_t H) {
    for (uint32_t h = blockIdx.x * blockDim.x + threadIdx.x; h < H; h += gridDim.x * blockDim.x) {
        const uint32_t f = hs.flags[h];
        if (f & HUB_REPEATS) {
            hs.best[h] = 0;
            hs.own_sum[h] = 0;
            hs.rowsum[h] = 0;
            hs.flags[h] = f & ~HUB_OWN_SEEN;
        }
    }
}

hipError_t launch_relabel_rows(const Graph &g, const uint32_t *old_of, const uint32_t *new_of, const uint64_t *rp2,
                               uint32_t *col2, uint32_t *w2, uint8_t *rowflag, uint32_t lo, uint32_t cnt,
                               uint32_t split, int bin_a, int bin_b, int per_wave, uint32_t *err,
                               const Round1Fuse *f, hipStream_t s) {
    if (cnt == 0) return hipSuccess;
    RelabelArgs a{g, old_of, new_of, rp2, col2, w2, err, nullptr, nullptr, 0, HubState{},
                  nullptr, nullptr, lo, split, bin_a, bin_b};
    if (f) {
        a.L1 = f->L1;
        a.changed = f->changed;
        a.sw = f->sw;
        a.rest_list = f->rest_list;
        a.rest_n = f->rest_n;
    }
    if (per_wave) {
        // rows [lo, split) have at most 512 arcs, rows [split, lo + cnt) at most 128
        const uint32_t c1 = split - lo, c2 = lo + cnt - split;
        if (c1) relabel_wave_k<kWaveArcs / 64><<<grid_for(c1, 4, 8192), 256, 0, s>>>(a, rowflag, lo, c1);
        if (c2) relabel_wave_k<kWaveArcsSmall / 64><<<grid_for(c2, 4, 8192), 256, 0, s>>>(a, rowflag, split, c2);
    } else {
        relabel_thread_k<<<grid_for(cnt, 256, 8192), 256, 0, s>>>(a, rowflag, lo, cnt);
    }
    return hipGetLastError();
}
uint32_t relabel_slices(uint32_t n) {
    const uint32_t S = (uint32_t)(((uint64_t)n + (1u << kSliceShift) - 1) >> kSliceShift);
    return (S >= kSliceMin && S <= kSliceMax) ? S : 0u;
}

hipError_t launch_relabel_hub(const Graph &g, const uint32_t *old_of, const uint32_t *new_of, const uint64_t *rp2,
                              uint32_t *col2, uint32_t *w2, const HubItem *items, uint32_t count,
                              uint32_t *hub_flags, uint32_t *err, const Round1Fuse *f, const HubState *hs,
                              uint32_t H, uint16_t *bnd, uint64_t *isrc, hipStream_t s) {
    if (count == 0) return hipSuccess;
    RelabelArgs a{g, old_of, new_of, rp2, col2, w2, err, nullptr, nullptr, 0, HubState{},
                  nullptr, nullptr, 0, 0, 0, 0};
    if (f) {
        a.L1 = f->L1;
        a.changed = f->changed;
        a.sw = f->sw;
        a.hs = *hs;
    }
    const uint32_t S = relabel_slices(g.n);
    if (S && bnd && isrc) {
        relabel_hub_scan_k<<<grid_for(count, 4, 8192), 256, 0, s>>>(a, items, count, hub_flags, S, bnd, isrc);
        const uint64_t per_slice = (count + kSliceItems - 1) / kSliceItems;
        relabel_hub_slices_k<<<(unsigned)(per_slice * (S + 1)), 256, 0, s>>>(a, items, count, S, bnd, isrc);
    } else {
        relabel_hub_k<<<grid_for(count, 4, 8192), 256, 0, s>>>(a, items, count, hub_flags);
    }
    if (f && H) hub_unfuse_k<<<grid_for(H, 256, 1024), 256, 0, s>>>(a.hs, H);
    return hipGetLastError();
}

// ---------------------------------------------------------- labels in/out --

// Both label buffers: vertices without arcs are never voted and keep their
// label in whichever buffer a round reads.
__global__ void init_labels_k(uint32_t *La, uint32_t *Lb, const uint32_t *old_of, const uint32_t *labels_in,
                              uint32_t n) {
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
        const uint32_t v = old_of[r];
        const uint32_t l = labels_in ? labels_in[v] : v;
        La[r] = l;
        if (Lb) Lb[r] = l;
    }
}
__global__ void scatter_labels_k(uint32_t *out, const uint32_t *old_of, const uint32_t *L, uint32_t n_int) {
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < n_int; r += gridDim.x * blockDim.x)
        out[old_of[r]] = L[r];
}

hipError_t launch_init_labels(uint32_t *La, uint32_t *Lb, const uint32_t *old_of, const uint32_t *labels_in,
                              uint32_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    init_labels_k<<<grid_for(n, 256, 8192), 256, 0, s>>>(La, Lb, old_of, labels_in, n);
    return hipGetLastError();
}
hipError_t launch_scatter_labels(uint32_t *out, const uint32_t *old_of, const uint32_t *L, uint32_t n_int,
                                 hipStream_t s) {
    if (n_int == 0) return hipSuccess;
    scatter_labels_k<<<grid_for(n_int, 256, 8192), 256, 0, s>>>(out, old_of, L, n_int);
    return hipGetLastError();
}

}  // namespace lpa
