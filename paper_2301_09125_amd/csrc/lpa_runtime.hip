// lpa_runtime.hip -- host side of the C ABI declared in include/lpa.h.
//
// lpa_run (arXiv 2301.09125, Section 3.2):
//   1. validate arguments on the host; bin vertices by degree on the device
//      (this pass also checks row_ptr) and lay out work for the long rows;
//   2. L0(v) = v in both label buffers (or the caller's labels to resume);
//   3. per round: the vote kernels of every non-empty bin read L_old and
//      write L_new, each adding its changed vertices to this round's device
//      counter; 8 bytes come back to the host, which applies the tolerance
//      test changed_t <= floor(tol * n) (Sections 3.2 and 4) and swaps the
//      buffers;
//   4. the final buffer is copied to labels_out if it is not already there.
// lpa_modularity evaluates the Section 1 quality measure with exact integer
// sums on the device.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "lpa.h"
#include "lpa_internal.h"

using namespace lpa;
typedef unsigned long long u64;

namespace {

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    template <typename T>
    T *as() const {
        return static_cast<T *>(p);
    }
    hipError_t ensure(size_t want) {
        if (want == 0) want = 8;
        if (bytes >= want) return hipSuccess;
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
        hipError_t e = hipMalloc(&p, want);
        if (e == hipSuccess) bytes = want;
        return e;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
};

enum KernelId { K_THREAD, K_GROUP, K_WAVE, K_HUB, K_HUB_REDUCE, K_HUB_FINAL, K_COUNT };
const char *kKernelNames[K_COUNT] = {"vote_thread", "vote_group", "vote_wave",
                                     "vote_hub",    "hub_reduce", "hub_final"};

struct Pending {
    int kid;
    hipEvent_t a, b;
    uint64_t bytes, arcs;
};

// Degree binning and long-row layout of one CSR.
struct Plan {
    uint32_t cnt[NBINS] = {0, 0, 0, 0, 0};
    uint64_t arcs[NBINS] = {0, 0, 0, 0, 0};
    uint32_t off[NBINS] = {0, 0, 0, 0, 0};
    uint32_t n_items = 0;   // hub work items (single-chunk rows + chunks of long rows)
    uint32_t n_multi = 0;   // rows longer than one chunk
    uint32_t n_ritems = 0;  // phase-2 items
};

}  // namespace

struct lpa_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    lpa_options opt{};
    int num_cu = 256;

    DevBuf labels_b, order, blk_counts, blk_arcs, small;  // small: totals + arc totals
    DevBuf counters;                                     // u64[max_iter] + error word
    DevBuf hub_rows, items, ritems;
    DevBuf hub_vertex, slab_off, slab_mask, touched_off, tcount, best, own_sum, own_seen, rowsum;
    DevBuf slab, touched;
    DevBuf K, mod_sums, partials;
    uint64_t *pinned = nullptr;  // host pinned scratch for small read-backs
    size_t pinned_words = 0;

    hipEvent_t round_a = nullptr, round_b = nullptr;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<Pending> pending;
    lpa_kernel_prof prof[K_COUNT];
};

namespace {

lpa_status dev_status(hipError_t e) {
    if (e == hipSuccess) return LPA_OK;
    if (e == hipErrorOutOfMemory) return LPA_ENOMEM;
    return LPA_EDEVICE;
}

#define HIP_TRY(expr)                                   \
    do {                                                \
        hipError_t _e = (expr);                         \
        if (_e != hipSuccess) return dev_status(_e);    \
    } while (0)

#define LPA_TRY(expr)                                   \
    do {                                                \
        lpa_status _s = (expr);                         \
        if (_s != LPA_OK) return _s;                    \
    } while (0)

lpa_status err_status(uint32_t bits) {
    if (bits & (ERR_COL | ERR_ROWPTR | ERR_LABEL)) return LPA_EINVAL;
    if (bits & ERR_WOVF) return LPA_EOVERFLOW;
    return LPA_OK;
}

uint32_t pow2_ceil(uint64_t x) {
    uint64_t p = 1;
    while (p < x) p <<= 1;
    return (uint32_t)p;
}

lpa_status check_options(const lpa_options &o) {
    if (o.thread_max < 1 || o.thread_max > (uint32_t)kThreadMaxCap) return LPA_EINVAL;
    if (o.group_max < o.thread_max || o.group_max > (uint32_t)kGroupSlots / 2) return LPA_EINVAL;
    if (o.wave_max < o.group_max || o.wave_max > (uint32_t)kWaveSlots / 2) return LPA_EINVAL;
    if (o.chunk < 256 || o.chunk > (uint32_t)kChunkSlotsMax / 2 || (o.chunk & (o.chunk - 1))) return LPA_EINVAL;
    return LPA_OK;
}

lpa_status ensure_pinned(lpa_ctx *c, size_t words) {
    if (c->pinned_words >= words) return LPA_OK;
    if (c->pinned) (void)hipHostFree(c->pinned);
    c->pinned = nullptr;
    c->pinned_words = 0;
    void *p = nullptr;
    HIP_TRY(hipHostMalloc(&p, words * sizeof(uint64_t), hipHostMallocDefault));
    c->pinned = static_cast<uint64_t *>(p);
    c->pinned_words = words;
    return LPA_OK;
}

hipEvent_t take_event(lpa_ctx *c) {
    if (c->ev_used == c->ev_pool.size()) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        c->ev_pool.push_back(e);
    }
    return c->ev_pool[c->ev_used++];
}

// Launch wrapper: brackets the launch with events when profiling.
template <typename F>
lpa_status timed(lpa_ctx *c, int kid, uint64_t bytes, uint64_t arcs, F &&launch) {
    hipEvent_t a = nullptr, b = nullptr;
    if (c->opt.profile) {
        a = take_event(c);
        b = take_event(c);
        if (!a || !b) return LPA_EDEVICE;
        HIP_TRY(hipEventRecord(a, c->stream));
    }
    HIP_TRY(launch());
    if (c->opt.profile) {
        HIP_TRY(hipEventRecord(b, c->stream));
        c->pending.push_back(Pending{kid, a, b, bytes, arcs});
    }
    return LPA_OK;
}

// After a stream synchronisation: fold the pending launch timings in.
void collect_profile(lpa_ctx *c) {
    for (const Pending &p : c->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            lpa_kernel_prof &r = c->prof[p.kid];
            r.launches += 1;
            r.ms += ms;
            r.bytes += p.bytes;
            r.arcs += p.arcs;
        }
    }
    c->pending.clear();
    c->ev_used = 0;
}

Graph make_graph(const lpa_csr *g) { return Graph{g->row_ptr, g->col, g->w, g->n, g->m}; }

lpa_status check_csr_args(const lpa_csr *g) {
    if (!g) return LPA_EINVAL;
    if (g->n > 0xFFFFFFFEu) return LPA_EINVAL;
    if (!g->row_ptr) return LPA_EINVAL;
    if (g->m > 0 && !g->col) return LPA_EINVAL;
    if (g->n == 0 && g->m != 0) return LPA_EINVAL;
    return LPA_OK;
}

// Bin the vertices, validate row_ptr, and lay out the long rows.
lpa_status prepare(lpa_ctx *c, const lpa_csr *g, Plan &P, uint32_t *err_dev, bool hub_state) {
    const hipStream_t s = c->stream;
    const Graph G = make_graph(g);
    const uint32_t n = g->n;
    const uint32_t nblk = (n + 255) / 256;
    HIP_TRY(c->blk_counts.ensure((size_t)NBINS * nblk * sizeof(uint32_t)));
    HIP_TRY(c->blk_arcs.ensure((size_t)NBINS * nblk * sizeof(u64)));
    HIP_TRY(c->order.ensure((size_t)n * sizeof(uint32_t)));
    HIP_TRY(c->small.ensure(NBINS * (sizeof(uint32_t) + sizeof(u64)) + 64));
    uint32_t *totals = c->small.as<uint32_t>();
    u64 *arc_totals = reinterpret_cast<u64 *>(c->small.as<char>() + 32);
    const lpa_options &o = c->opt;
    HIP_TRY(launch_bin_count(G, o.thread_max, o.group_max, o.wave_max, c->blk_counts.as<uint32_t>(),
                             c->blk_arcs.as<u64>(), nblk, err_dev, s));
    HIP_TRY(launch_bin_scan(c->blk_counts.as<uint32_t>(), c->blk_arcs.as<u64>(), nblk, totals, arc_totals, s));
    HIP_TRY(launch_bin_scatter(G, o.thread_max, o.group_max, o.wave_max, c->blk_counts.as<uint32_t>(), nblk,
                               c->order.as<uint32_t>(), s));
    LPA_TRY(ensure_pinned(c, 16));
    uint32_t *h32 = reinterpret_cast<uint32_t *>(c->pinned);
    HIP_TRY(hipMemcpyAsync(c->pinned, c->small.p, 32 + NBINS * sizeof(u64), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(c->pinned + 12, err_dev, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const uint32_t errbits = reinterpret_cast<uint32_t *>(c->pinned + 12)[0];
    if (errbits) return err_status(errbits);
    uint32_t run = 0;
    for (int b = 0; b < NBINS; ++b) {
        P.cnt[b] = h32[b];
        P.arcs[b] = c->pinned[4 + b];
        P.off[b] = run;
        run += P.cnt[b];
    }
    P.n_items = P.n_multi = P.n_ritems = 0;
    const uint32_t H = P.cnt[BIN_HUB];
    if (H == 0) return LPA_OK;

    // Long rows: fetch (vertex, row begin, row end) and build the work items.
    HIP_TRY(c->hub_rows.ensure((size_t)H * 2 * sizeof(uint64_t)));
    const uint32_t *hub_list = c->order.as<uint32_t>() + P.off[BIN_HUB];
    HIP_TRY(launch_gather_rows(g->row_ptr, hub_list, H, c->hub_rows.as<uint64_t>(), s));
    std::vector<uint32_t> verts(H);
    std::vector<uint64_t> rows((size_t)H * 2);
    HIP_TRY(hipMemcpyAsync(verts.data(), hub_list, (size_t)H * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(rows.data(), c->hub_rows.p, (size_t)H * 2 * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));

    const uint64_t C = o.chunk;
    std::vector<HubItem> items;
    std::vector<ReduceItem> ritems;
    std::vector<uint32_t> hv;
    std::vector<uint64_t> soff, toff;
    std::vector<uint32_t> smask;
    uint64_t slab_total = 0, touched_total = 0;
    std::vector<HubItem> singles;
    for (uint32_t i = 0; i < H; ++i) {
        const uint64_t b = rows[2 * i], e = rows[2 * i + 1], d = e - b;
        if (d <= C) {
            singles.push_back(HubItem{verts[i], kNoHub, b, e});
            continue;
        }
        const uint32_t h = (uint32_t)hv.size();
        hv.push_back(verts[i]);
        const uint64_t slots = pow2_ceil(2 * d);
        soff.push_back(slab_total);
        smask.push_back((uint32_t)(slots - 1));
        toff.push_back(touched_total);
        slab_total += slots;
        touched_total += d;
        uint32_t ci = 0;
        for (uint64_t x = b; x < e; x += C, ++ci) {
            items.push_back(HubItem{verts[i], h, x, std::min(e, x + C)});
            ritems.push_back(ReduceItem{h, (uint32_t)(ci * C), (uint32_t)((ci + 1) * C), 0});
        }
    }
    // long rows first: their chunks are the largest units of work
    items.insert(items.end(), singles.begin(), singles.end());
    P.n_items = (uint32_t)items.size();
    P.n_multi = (uint32_t)hv.size();
    P.n_ritems = (uint32_t)ritems.size();
    HIP_TRY(c->items.ensure(items.size() * sizeof(HubItem)));
    HIP_TRY(hipMemcpyAsync(c->items.p, items.data(), items.size() * sizeof(HubItem), hipMemcpyHostToDevice, s));
    if (!hub_state || P.n_multi == 0) {
        HIP_TRY(hipStreamSynchronize(s));
        return LPA_OK;
    }
    const uint32_t M = P.n_multi;
    HIP_TRY(c->ritems.ensure(ritems.size() * sizeof(ReduceItem)));
    HIP_TRY(c->hub_vertex.ensure(M * sizeof(uint32_t)));
    HIP_TRY(c->slab_off.ensure(M * sizeof(uint64_t)));
    HIP_TRY(c->slab_mask.ensure(M * sizeof(uint32_t)));
    HIP_TRY(c->touched_off.ensure(M * sizeof(uint64_t)));
    HIP_TRY(c->tcount.ensure(M * sizeof(uint32_t)));
    HIP_TRY(c->best.ensure(M * sizeof(u64)));
    HIP_TRY(c->own_sum.ensure(M * sizeof(u64)));
    HIP_TRY(c->own_seen.ensure(M * sizeof(uint32_t)));
    HIP_TRY(c->rowsum.ensure(M * sizeof(u64)));
    HIP_TRY(c->touched.ensure(touched_total * sizeof(uint32_t)));
    const size_t old_slab = c->slab.bytes;
    HIP_TRY(c->slab.ensure(slab_total * sizeof(u64)));
    if (c->slab.bytes != old_slab || old_slab == 0)  // fresh allocation: every slot EMPTY
        HIP_TRY(launch_fill_u64(c->slab.as<u64>(), 0xFFFFFFFF00000000ull, c->slab.bytes / sizeof(u64), s));
    HIP_TRY(hipMemcpyAsync(c->ritems.p, ritems.data(), ritems.size() * sizeof(ReduceItem), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(c->hub_vertex.p, hv.data(), M * sizeof(uint32_t), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(c->slab_off.p, soff.data(), M * sizeof(uint64_t), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(c->slab_mask.p, smask.data(), M * sizeof(uint32_t), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(c->touched_off.p, toff.data(), M * sizeof(uint64_t), hipMemcpyHostToDevice, s));
    HIP_TRY(launch_fill_u32(c->tcount.as<uint32_t>(), 0, M, s));
    HIP_TRY(launch_fill_u64(c->best.as<u64>(), 0, M, s));
    HIP_TRY(launch_fill_u64(c->own_sum.as<u64>(), 0, M, s));
    HIP_TRY(launch_fill_u32(c->own_seen.as<uint32_t>(), 0, M, s));
    HIP_TRY(launch_fill_u64(c->rowsum.as<u64>(), 0, M, s));
    // the host vectors must outlive the asynchronous copies
    HIP_TRY(hipStreamSynchronize(s));
    return LPA_OK;
}

HubState hub_state(lpa_ctx *c) {
    HubState h;
    h.vertex = c->hub_vertex.as<uint32_t>();
    h.slab_off = c->slab_off.as<uint64_t>();
    h.slab_mask = c->slab_mask.as<uint32_t>();
    h.touched_off = c->touched_off.as<uint64_t>();
    h.slab = c->slab.as<u64>();
    h.touched = c->touched.as<uint32_t>();
    h.tcount = c->tcount.as<uint32_t>();
    h.best = c->best.as<u64>();
    h.own_sum = c->own_sum.as<u64>();
    h.own_seen = c->own_seen.as<uint32_t>();
    h.rowsum = c->rowsum.as<u64>();
    return h;
}

// Enqueue every vote kernel of one round.
lpa_status enqueue_round(lpa_ctx *c, const Plan &P, const RoundArgs &ra, const HubState &hs, bool weighted) {
    const hipStream_t s = c->stream;
    const uint32_t *order = c->order.as<uint32_t>();
    const uint64_t ab = weighted ? 12 : 8;  // algorithmic bytes per arc: col, w, gathered label
    const int cap = c->num_cu * 8;
    LPA_TRY(timed(c, K_THREAD, ab * P.arcs[BIN_THREAD] + 16ull * P.cnt[BIN_THREAD], P.arcs[BIN_THREAD], [&] {
        return launch_vote_thread(ra, order + P.off[BIN_THREAD], P.cnt[BIN_THREAD], cap, s);
    }));
    LPA_TRY(timed(c, K_GROUP, ab * P.arcs[BIN_GROUP] + 16ull * P.cnt[BIN_GROUP], P.arcs[BIN_GROUP], [&] {
        return launch_vote_group(ra, order + P.off[BIN_GROUP], P.cnt[BIN_GROUP], cap, s);
    }));
    LPA_TRY(timed(c, K_WAVE, ab * P.arcs[BIN_WAVE] + 16ull * P.cnt[BIN_WAVE], P.arcs[BIN_WAVE], [&] {
        return launch_vote_wave(ra, order + P.off[BIN_WAVE], P.cnt[BIN_WAVE], cap, s);
    }));
    if (P.n_items) {
        LPA_TRY(timed(c, K_HUB, ab * P.arcs[BIN_HUB] + 16ull * P.cnt[BIN_HUB], P.arcs[BIN_HUB], [&] {
            return launch_vote_hub(ra, c->items.as<HubItem>(), P.n_items, c->opt.chunk, hs, s);
        }));
    }
    if (P.n_multi) {
        LPA_TRY(timed(c, K_HUB_REDUCE, 0, 0, [&] {
            return launch_hub_reduce(hs, c->ritems.as<ReduceItem>(), P.n_ritems, s);
        }));
        LPA_TRY(timed(c, K_HUB_FINAL, 0, 0, [&] { return launch_hub_final(ra, hs, P.n_multi, s); }));
    }
    return LPA_OK;
}

lpa_status run_impl(lpa_ctx *c, const lpa_csr *g, uint32_t *labels, double tol, uint32_t max_iter,
                    lpa_stats *stats, bool resume) {
    const auto t_start = std::chrono::steady_clock::now();
    if (!c) return LPA_EINVAL;
    LPA_TRY(check_csr_args(g));
    if (!labels && g->n) return LPA_EINVAL;
    if (!(tol >= 0.0 && tol <= 1.0)) return LPA_EINVAL;
    HIP_TRY(hipSetDevice(c->device));
    const hipStream_t s = c->stream;
    const uint32_t n = g->n;
    if (stats) {
        stats->iterations = 0;
        stats->converged = 0;
        stats->changed_last = 0;
        stats->arcs_processed = 0;
        stats->ms_rounds = 0;
        stats->ms_total = 0;
    }
    // counters: one u64 per round, then the error word
    HIP_TRY(c->counters.ensure(((size_t)max_iter + 2) * sizeof(u64)));
    u64 *counters = c->counters.as<u64>();
    uint32_t *err_dev = reinterpret_cast<uint32_t *>(counters + max_iter + 1);
    HIP_TRY(launch_fill_u64(counters, 0, (size_t)max_iter + 2, s));
    LPA_TRY(ensure_pinned(c, 16));

    if (resume && n) {
        HIP_TRY(launch_check_labels(labels, n, err_dev, s));
    }
    Plan P;
    if (n) LPA_TRY(prepare(c, g, P, err_dev, true));
    HIP_TRY(c->labels_b.ensure((size_t)n * sizeof(uint32_t)));
    uint32_t *A = labels, *B = c->labels_b.as<uint32_t>();
    if (resume) {
        HIP_TRY(launch_copy_u32(B, A, n, s));
    } else {
        HIP_TRY(launch_fill_u32_iota(A, B, n, s));
    }
    const uint64_t thr = (uint64_t)std::floor(tol * (double)n);
    const bool weighted = g->w != nullptr;
    const HubState hs = hub_state(c);
    const uint64_t voted_arcs = P.arcs[BIN_THREAD] + P.arcs[BIN_GROUP] + P.arcs[BIN_WAVE] + P.arcs[BIN_HUB];
    if (!c->round_a) HIP_TRY(hipEventCreate(&c->round_a));
    if (!c->round_b) HIP_TRY(hipEventCreate(&c->round_b));

    uint32_t *L_old = A, *L_new = B;
    lpa_status st = LPA_OK;
    uint32_t it = 0;
    int converged = 0;
    u64 changed = 0;
    double ms_rounds = 0;
    for (uint32_t t = 1; t <= max_iter && n; ++t) {
        RoundArgs ra;
        ra.g = make_graph(g);
        ra.L_old = L_old;
        ra.L_new = L_new;
        ra.sw = c->opt.self_weight;
        ra.check = (t == 1);
        ra.changed = counters + (t - 1);
        ra.err = err_dev;
        HIP_TRY(hipEventRecord(c->round_a, s));
        st = enqueue_round(c, P, ra, hs, weighted);
        if (st != LPA_OK) break;
        HIP_TRY(hipEventRecord(c->round_b, s));
        HIP_TRY(hipMemcpyAsync(c->pinned, counters + (t - 1), sizeof(u64), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(c->pinned + 1, err_dev, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (c->opt.profile) collect_profile(c);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, c->round_a, c->round_b);
        ms_rounds += ms;
        const uint32_t errbits = reinterpret_cast<uint32_t *>(c->pinned + 1)[0];
        if (errbits) {
            st = err_status(errbits);
            break;
        }
        changed = c->pinned[0];
        it = t;
        if (stats) {
            if (stats->changed_per_iter && t <= stats->cap) stats->changed_per_iter[t - 1] = changed;
            if (stats->ms_per_iter && t <= stats->cap) stats->ms_per_iter[t - 1] = ms;
        }
        std::swap(L_old, L_new);
        if (changed <= thr) {
            converged = 1;
            break;
        }
    }
    if (st != LPA_OK) return st;
    if (L_old != labels) HIP_TRY(launch_copy_u32(labels, L_old, n, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (stats) {
        stats->iterations = it;
        stats->converged = converged;
        stats->changed_last = changed;
        stats->arcs_processed = voted_arcs * it;
        stats->ms_rounds = ms_rounds;
        stats->ms_total =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    }
    return LPA_OK;
}

}  // namespace

extern "C" {

void lpa_default_options(lpa_options *opt) {
    if (!opt) return;
    opt->self_weight = 1;
    opt->thread_max = 8;
    opt->group_max = 32;
    opt->wave_max = 256;
    opt->chunk = 2048;
    opt->profile = 0;
}

lpa_status lpa_init(lpa_ctx **ctx, int device, void *stream, const lpa_options *opt) {
    if (!ctx) return LPA_EINVAL;
    *ctx = nullptr;
    lpa_options o;
    lpa_default_options(&o);
    if (opt) {
        o = *opt;
        lpa_options d;
        lpa_default_options(&d);
        if (!o.thread_max) o.thread_max = d.thread_max;
        if (!o.group_max) o.group_max = d.group_max;
        if (!o.wave_max) o.wave_max = d.wave_max;
        if (!o.chunk) o.chunk = d.chunk;
    }
    LPA_TRY(check_options(o));
    int ndev = 0;
    HIP_TRY(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return LPA_EINVAL;
    HIP_TRY(hipSetDevice(device));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, device));
    lpa_ctx *c = new (std::nothrow) lpa_ctx();
    if (!c) return LPA_ENOMEM;
    c->device = device;
    c->stream = static_cast<hipStream_t>(stream);
    c->opt = o;
    c->num_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    for (int k = 0; k < K_COUNT; ++k) {
        std::memset(&c->prof[k], 0, sizeof(lpa_kernel_prof));
        std::snprintf(c->prof[k].name, sizeof(c->prof[k].name), "%s", kKernelNames[k]);
    }
    *ctx = c;
    return LPA_OK;
}

lpa_status lpa_run(lpa_ctx *ctx, const lpa_csr *g, uint32_t *labels_out, double tol, uint32_t max_iter,
                   lpa_stats *stats) {
    return run_impl(ctx, g, labels_out, tol, max_iter, stats, false);
}

lpa_status lpa_run_resume(lpa_ctx *ctx, const lpa_csr *g, uint32_t *labels_inout, double tol, uint32_t max_iter,
                          lpa_stats *stats) {
    return run_impl(ctx, g, labels_inout, tol, max_iter, stats, true);
}

lpa_status lpa_modularity(lpa_ctx *c, const lpa_csr *g, const uint32_t *labels, double *q_out, uint64_t *terms) {
    if (!c || !q_out) return LPA_EINVAL;
    LPA_TRY(check_csr_args(g));
    if (g->n && !labels) return LPA_EINVAL;
    HIP_TRY(hipSetDevice(c->device));
    const hipStream_t s = c->stream;
    const uint32_t n = g->n;
    *q_out = 0.0;
    if (terms) std::memset(terms, 0, 4 * sizeof(uint64_t));
    if (n == 0) return LPA_OK;
    HIP_TRY(c->counters.ensure(4 * sizeof(u64)));
    u64 *counters = c->counters.as<u64>();
    uint32_t *err_dev = reinterpret_cast<uint32_t *>(counters);
    HIP_TRY(launch_fill_u64(counters, 0, 1, s));
    HIP_TRY(launch_check_labels(labels, n, err_dev, s));
    Plan P;
    LPA_TRY(prepare(c, g, P, err_dev, false));
    const uint32_t nparts = 1024;
    HIP_TRY(c->K.ensure((size_t)n * sizeof(u64)));
    HIP_TRY(c->mod_sums.ensure(2 * sizeof(u64)));
    HIP_TRY(c->partials.ensure(2 * nparts * sizeof(u64)));
    HIP_TRY(launch_fill_u64(c->K.as<u64>(), 0, n, s));
    HIP_TRY(launch_fill_u64(c->mod_sums.as<u64>(), 0, 2, s));
    ModArgs ma;
    ma.g = make_graph(g);
    ma.labels = labels;
    ma.K = c->K.as<u64>();
    ma.sums = c->mod_sums.as<u64>();
    ma.err = err_dev;
    const uint32_t *order = c->order.as<uint32_t>();
    HIP_TRY(launch_mod_small(ma, order + P.off[BIN_THREAD], P.cnt[BIN_THREAD] + P.cnt[BIN_GROUP], s));
    HIP_TRY(launch_mod_wave(ma, order + P.off[BIN_WAVE], P.cnt[BIN_WAVE], s));
    HIP_TRY(launch_mod_hub(ma, c->items.as<HubItem>(), P.n_items, s));
    HIP_TRY(launch_mod_sumsq(c->K.as<u64>(), n, c->partials.as<u64>(), nparts, s));
    std::vector<u64> parts(2 * nparts);
    u64 sums[2];
    uint32_t errbits = 0;
    HIP_TRY(hipMemcpyAsync(parts.data(), c->partials.p, 2 * nparts * sizeof(u64), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(sums, c->mod_sums.p, 2 * sizeof(u64), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&errbits, err_dev, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (errbits) return err_status(errbits);
    unsigned __int128 sk2 = 0;
    for (uint32_t i = 0; i < nparts; ++i)
        sk2 += ((unsigned __int128)parts[2 * i + 1] << 64) | (unsigned __int128)parts[2 * i];
    const u64 two_m = sums[0], sigma_in = sums[1];
    double q = 0.0;
    if (two_m > 0) {
        const double W = (double)two_m;
        q = (double)sigma_in / W - (double)sk2 / (W * W);
    }
    *q_out = q;
    if (terms) {
        terms[0] = two_m;
        terms[1] = sigma_in;
        terms[2] = (u64)sk2;
        terms[3] = (u64)(sk2 >> 64);
    }
    return LPA_OK;
}

lpa_status lpa_profile_get(lpa_ctx *c, lpa_kernel_prof *out, uint32_t cap, uint32_t *count) {
    if (!c || !count || (cap && !out)) return LPA_EINVAL;
    *count = K_COUNT;
    for (uint32_t k = 0; k < cap && k < (uint32_t)K_COUNT; ++k) out[k] = c->prof[k];
    return LPA_OK;
}

lpa_status lpa_profile_reset(lpa_ctx *c) {
    if (!c) return LPA_EINVAL;
    for (int k = 0; k < K_COUNT; ++k) {
        c->prof[k].launches = 0;
        c->prof[k].ms = 0;
        c->prof[k].bytes = 0;
        c->prof[k].arcs = 0;
    }
    return LPA_OK;
}

void lpa_destroy(lpa_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    DevBuf *bufs[] = {&c->labels_b, &c->order,    &c->blk_counts, &c->blk_arcs,  &c->small,     &c->counters,
                      &c->hub_rows, &c->items,    &c->ritems,     &c->hub_vertex, &c->slab_off, &c->slab_mask,
                      &c->touched_off, &c->tcount, &c->best,      &c->own_sum,   &c->own_seen,  &c->rowsum,
                      &c->slab,     &c->touched,  &c->K,          &c->mod_sums,  &c->partials};
    for (DevBuf *b : bufs) b->release();
    if (c->pinned) (void)hipHostFree(c->pinned);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    if (c->round_a) (void)hipEventDestroy(c->round_a);
    if (c->round_b) (void)hipEventDestroy(c->round_b);
    delete c;
}

const char *lpa_strerror(lpa_status s) {
    switch (s) {
        case LPA_OK: return "success";
        case LPA_EINVAL: return "invalid argument, malformed CSR or label out of range";
        case LPA_EOVERFLOW: return "a weighted degree plus self weight does not fit 32 bits";
        case LPA_ENOMEM: return "out of memory";
        case LPA_EDEVICE: return "HIP runtime error";
        case LPA_EUNSUPPORTED: return "unsupported option or size";
    }
    return "unknown status";
}

}  // extern "C"
