// lpa_runtime.hip -- host side of the C ABI declared in include/lpa.h.
//
// lpa_run (arXiv 2301.09125, Section 3.2):
//   1. validate arguments on the host; bin the vertices by degree on the
//      device (this pass also checks row_ptr) and build the relabelled
//      internal CSR (lpa_internal.h), which also checks every col value;
//   2. L0(v) = v in both label buffers (or the caller's labels to resume);
//   3. per round: the vote kernel of every non-empty bin reads L_old and
//      writes L_new, adding its changed vertices to this round's device
//      counter words; 4 KB come back to the host, which applies the
//      tolerance test changed_t <= floor(tol * n) (Sections 3.2 and 4) and
//      swaps the buffers;
//   4. the final labels are scattered back to the caller's vertex order, and
//      optionally their modularity (Section 1) is computed on the same
//      internal graph.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "lpa.h"
#include "lpa_internal.h"
#include "lpa_copra.h"
#include "lpa_sortnet.h"

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

enum KernelId {
    K_THREAD, K_GROUP, K_WAVE, K_WIDE, K_HUB, K_HUB1, K_MERGE, K_FALLBACK, K_REDUCE, K_FINAL, K_MOD,
    K_PREDICT, K_PUSH, K_LISTED, K_COPRA, K_COPRA_GLOBAL, K_COUNT
};
// vote_round1_rest: round-1 votes of the rows the relabel pass could not
// decide (repeated neighbours), no algorithmic bytes counted;
// predict / push: candidate selection and frontier stamps of frontier runs;
// vote_listed: the short-row votes of a round driven by candidate lists
const char *kKernelNames[K_COUNT] = {"vote_thread",  "vote_group", "vote_wave",    "vote_wide",
                                     "vote_hub",     "vote_round1_rest", "hub_merge", "hub_fallback",
                                     "hub_reduce",   "hub_final",  "modularity", "predict", "push",
                                     "vote_listed", "copra", "copra_global"};

struct Pending {
    int kid;
    hipEvent_t a, b;
    uint64_t bytes, arcs;
};

// Bins and long-row work of one CSR.
struct Plan {
    Bins bins;
    uint32_t H = 0;         // long rows (internal ids 0..H-1)
    uint32_t n_items = 0;   // wavefront segments of long rows
    uint32_t n_ritems = 0;  // phase-2 items
    uint32_t n_mwave = 0;   // rows merged by one wavefront
    uint32_t n_mblock = 0;  // rows merged by one block
};

}  // namespace

struct lpa_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    lpa_options opt{};
    int num_cu = 256;

    DevBuf blk_counts, blk_arcs, small;
    DevBuf old_of, new_of, rp2, col2, w2, rowflag, La, Lb;
    DevBuf counters;  // kCountWords u64 per round, then the error word
    DevBuf items, ritems, slab_off, slab_mask, touched_off, tcount, best, own_sum, hflags, rowsum, slab, touched;
    DevBuf cand, thr, item_lo, mrows, slab_pending, hub_tmp, r1_rows, r1_cnt;
    DevBuf hub_bnd, hub_src;  // long-row relabel by slices: slice starts per segment, segment sources
    DevBuf K, mod_sums, partials;
    DevBuf gid, gvd, bstate, bseg;  // batched run
    DevBuf f_top1, f_top2, f_kw, f_last, f_front, f_stale, f_lists, f_small, f_model;  // frontier runs
    DevBuf t_w, t_m, t_v, t_part, t_grad, t_loss, t_z;                               // training
    DevBuf tune_labels, tune_hist;                                                    // autotuner
    DevBuf cp_rec[2], cp_rows, cp_ovf, cp_off, cp_key, cp_tal;  // COPRA
    DevBuf cp_first, cp_pieces, cp_total, cp_rows1, cp_rows2, cp_rows3, cp_distinct, cp_sfirst, cp_slices, cp_rowstate,
        cp_wsum;
    std::map<std::vector<int>, lpa_options> tune_cache;
    // the CSR and thresholds the internal copy was last built for by a
    // prepare() that also set up the long-row state (empty = none)
    std::vector<uint64_t> prep_key;
    std::vector<uint64_t> bprep_key;  // prep_key, G and graph_vptr of the batch whose gid/segments are built
    Plan prep_plan;
    bool slab_dirty = false;      // slab may hold entries (set after a timed-out batch)
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t bexec = nullptr;
    std::vector<unsigned char> bkey;  // launch parameters the captured graph was made with
    uint64_t *pinned = nullptr;  // host pinned scratch for small read-backs
    size_t pinned_words = 0;

    hipEvent_t round_a = nullptr, round_b = nullptr, prep_a = nullptr, prep_b = nullptr;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<Pending> pending;
    lpa_kernel_prof prof[K_COUNT];
};

namespace lpa {
int ctx_device(const lpa_ctx *c) { return c->device; }
hipStream_t ctx_stream(const lpa_ctx *c) { return c->stream; }
}  // namespace lpa

namespace {

lpa_status dev_status(hipError_t e) {
    if (e == hipSuccess) return LPA_OK;
    if (e == hipErrorOutOfMemory) return LPA_ENOMEM;
    return LPA_EDEVICE;
}

#define HIP_TRY(expr)                                \
    do {                                             \
        hipError_t _e = (expr);                      \
        if (_e != hipSuccess) return dev_status(_e); \
    } while (0)

#define LPA_TRY(expr)                \
    do {                             \
        lpa_status _s = (expr);      \
        if (_s != LPA_OK) return _s; \
    } while (0)

lpa_status err_status(uint32_t bits) {
    if (bits & (ERR_COL | ERR_ROWPTR | ERR_LABEL | ERR_GRAPH)) return LPA_EINVAL;
    if (bits & ERR_TIMEOUT) return LPA_ETIMEDOUT;
    if (bits & ERR_WOVF) return LPA_EOVERFLOW;
    if (bits & ERR_TABLE) return LPA_EDEVICE;
    return LPA_OK;
}

lpa_status check_options(const lpa_options &o) {
    if (o.thread_max < 1 || o.thread_max > (uint32_t)kThreadMaxCap) return LPA_EINVAL;
    if (o.group_max < o.thread_max || o.group_max > (uint32_t)kGroupSlots / 2) return LPA_EINVAL;
    if (o.wave_max < o.group_max || o.wave_max > (uint32_t)kWaveArcsSmall) return LPA_EINVAL;
    if (o.wide_max < o.wave_max || o.wide_max > (uint32_t)kWaveArcs) return LPA_EINVAL;
    if (o.merge_max < 1 || o.merge_max > (uint32_t)kMergeBlockSegs) return LPA_EINVAL;
    if (o.frontier > 1) return LPA_EINVAL;
    if (o.order > LPA_ORDER_SEMISYNC || o.tie > LPA_TIE_HASH) return LPA_EINVAL;
    if (o.frontier && (o.order || o.tie)) return LPA_EUNSUPPORTED;
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

lpa_status check_csr_args(const lpa_csr *g) {
    if (!g) return LPA_EINVAL;
    if (g->n > 0xFFFFFFFEu) return LPA_EINVAL;
    if (!g->row_ptr) return LPA_EINVAL;
    if (g->m > 0 && !g->col) return LPA_EINVAL;
    if (g->n == 0 && g->m != 0) return LPA_EINVAL;
    return LPA_OK;
}

Graph internal_graph(lpa_ctx *c, const lpa_csr *g) {
    return Graph{c->rp2.as<uint64_t>(), c->col2.as<uint32_t>(), g->w ? c->w2.as<uint32_t>() : nullptr, g->n, g->m};
}

HubState hub_state(lpa_ctx *c) {
    HubState h;
    h.slab_off = c->slab_off.as<uint64_t>();
    h.slab_mask = c->slab_mask.as<uint32_t>();
    h.touched_off = c->touched_off.as<uint64_t>();
    h.slab = c->slab.as<u64>();
    h.touched = c->touched.as<uint32_t>();
    h.tcount = c->tcount.as<uint32_t>();
    h.best = c->best.as<u64>();
    h.own_sum = c->own_sum.as<u64>();
    h.flags = c->hflags.as<uint32_t>();
    h.rowsum = c->rowsum.as<u64>();
    h.cand = c->cand.as<u64>();
    h.thr = c->thr.as<uint32_t>();
    h.item_lo = c->item_lo.as<uint32_t>();
    h.pending = c->slab_pending.as<uint32_t>();
    h.repeats = h.pending ? h.pending + 1 : nullptr;
    return h;
}

// What an internal copy depends on: the CSR arrays, sizes and bin thresholds.
std::vector<uint64_t> csr_key(const lpa_ctx *c, const lpa_csr *g) {
    const lpa_options &o = c->opt;
    return {(uint64_t)(uintptr_t)g->row_ptr, (uint64_t)(uintptr_t)g->col, (uint64_t)(uintptr_t)g->w, g->n, g->m,
            o.thread_max, o.group_max, o.wave_max, o.wide_max, o.merge_max};
}

// Bin the vertices, validate row_ptr, build the internal CSR and lay out the
// long rows.  with_slab: also prepare the global slabs used by the vote (and
// remember the copy under csr_key for reuse_csr).  fuse: also run round 1
// from the unique labels inside the relabel pass (rows that list each
// neighbour once); La/fuse->L1 then get their initial labels here.
lpa_status prepare(lpa_ctx *c, const lpa_csr *g, Plan &P, uint32_t *err_dev, bool with_slab,
                   const Round1Fuse *fuse = nullptr, uint32_t *La = nullptr) {
    const hipStream_t s = c->stream;
    const Graph G{g->row_ptr, g->col, g->w, g->n, g->m};
    const uint32_t n = g->n;
    const uint32_t nblk = bin_blocks(n);
    const lpa_options &o = c->opt;
    c->prep_key.clear();  // the internal copy is rebuilt below
    c->bprep_key.clear();
    HIP_TRY(c->blk_counts.ensure((size_t)NBINS * nblk * sizeof(uint32_t)));
    HIP_TRY(c->blk_arcs.ensure((size_t)NBINS * nblk * sizeof(u64)));
    HIP_TRY(c->small.ensure(128));
    HIP_TRY(c->old_of.ensure((size_t)n * sizeof(uint32_t)));
    HIP_TRY(c->new_of.ensure((size_t)n * sizeof(uint32_t)));
    HIP_TRY(c->rp2.ensure(((size_t)n + 1) * sizeof(uint64_t)));
    HIP_TRY(c->col2.ensure(((size_t)g->m + kLaneArcPad) * sizeof(uint32_t)));
    if (g->w) HIP_TRY(c->w2.ensure(((size_t)g->m + kLaneArcPad) * sizeof(uint32_t)));
    HIP_TRY(c->rowflag.ensure((size_t)n));
    uint32_t *totals = c->small.as<uint32_t>();
    u64 *arc_totals = reinterpret_cast<u64 *>(c->small.as<char>() + 32);
    const BinCfg cfg{o.thread_max, o.group_max, o.wave_max, o.wide_max};
    HIP_TRY(launch_bin_count(G, cfg, c->blk_counts.as<uint32_t>(), c->blk_arcs.as<u64>(), nblk, err_dev, s));
    HIP_TRY(launch_bin_scan(c->blk_counts.as<uint32_t>(), c->blk_arcs.as<u64>(), nblk, totals, arc_totals, s));
    HIP_TRY(launch_bin_scatter(G, cfg, c->blk_counts.as<uint32_t>(), c->blk_arcs.as<u64>(), totals, arc_totals,
                               nblk, c->old_of.as<uint32_t>(), c->new_of.as<uint32_t>(), c->rp2.as<uint64_t>(), s));
    HIP_TRY(launch_fill_u64(reinterpret_cast<u64 *>(c->rp2.as<uint64_t>() + n), g->m, 1, s));
    LPA_TRY(ensure_pinned(c, 16));
    HIP_TRY(hipMemcpyAsync(c->pinned, c->small.p, 32 + NBINS * sizeof(u64), hipMemcpyDeviceToHost, s));
    static_assert(NBINS <= 8 && 4 + NBINS <= 12, "bin totals must fit the read-back layout");
    HIP_TRY(hipMemcpyAsync(c->pinned + 12, err_dev, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const uint32_t errbits = reinterpret_cast<uint32_t *>(c->pinned + 12)[0];
    if (errbits) return err_status(errbits);
    const uint32_t *h32 = reinterpret_cast<const uint32_t *>(c->pinned);
    uint32_t run = 0;
    for (int b = 0; b < NBINS; ++b) {
        P.bins.cnt[b] = h32[b];
        P.bins.arcs[b] = c->pinned[4 + b];
        P.bins.lo[b] = run;
        run += P.bins.cnt[b];
    }
    P.H = P.bins.cnt[BIN_HUB];
    P.n_items = P.n_ritems = 0;
    uint64_t slab_total = 0, touched_total = 0;

    // long rows: wavefront segments, merge lists, slab and touched-list
    // offsets, planned on the device
    if (P.H) {
        const uint32_t H = P.H;
        const uint32_t nb = (H + 1023) / 1024;
        HIP_TRY(c->item_lo.ensure(((size_t)H + 1) * sizeof(uint32_t)));
        HIP_TRY(c->slab_off.ensure(H * sizeof(uint64_t)));
        HIP_TRY(c->touched_off.ensure(H * sizeof(uint64_t)));
        HIP_TRY(c->slab_mask.ensure(H * sizeof(uint32_t)));
        HIP_TRY(c->hflags.ensure(H * sizeof(uint32_t)));
        HIP_TRY(c->hub_tmp.ensure(((size_t)nb * 6 + 8) * sizeof(u64)));
        u64 *blk = c->hub_tmp.as<u64>(), *plan = blk + (size_t)nb * 6;
        HIP_TRY(launch_hub_plan(c->rp2.as<uint64_t>(), H, o.merge_max, blk, plan, s));
        HIP_TRY(hipMemcpyAsync(c->pinned, plan, 6 * sizeof(u64), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        P.n_items = (uint32_t)c->pinned[0];
        slab_total = c->pinned[1];
        touched_total = c->pinned[2];
        P.n_ritems = (uint32_t)c->pinned[3];
        P.n_mwave = (uint32_t)c->pinned[4];
        P.n_mblock = (uint32_t)c->pinned[5];
        HIP_TRY(c->items.ensure((size_t)P.n_items * sizeof(HubItem)));
        HIP_TRY(c->ritems.ensure((size_t)P.n_ritems * sizeof(ReduceItem)));
        HIP_TRY(c->mrows.ensure(((size_t)P.n_mwave + P.n_mblock) * sizeof(uint32_t)));
        HIP_TRY(launch_hub_fill(c->rp2.as<uint64_t>(), H, o.merge_max, blk, plan, c->item_lo.as<uint32_t>(),
                                c->slab_off.as<uint64_t>(), c->touched_off.as<uint64_t>(), c->items.as<HubItem>(),
                                c->ritems.as<ReduceItem>(), c->hflags.as<uint32_t>(), c->slab_mask.as<uint32_t>(),
                                c->mrows.as<uint32_t>(), s));
    }

    if (with_slab && P.H) {
        const uint32_t H = P.H;
        HIP_TRY(c->tcount.ensure(H * sizeof(uint32_t)));
        HIP_TRY(c->best.ensure(H * sizeof(u64)));
        HIP_TRY(c->own_sum.ensure(H * sizeof(u64)));
        HIP_TRY(c->rowsum.ensure(H * sizeof(u64)));
        HIP_TRY(c->touched.ensure(touched_total * sizeof(uint32_t)));
        const size_t old_slab = c->slab.bytes;
        HIP_TRY(c->slab.ensure(slab_total * sizeof(u64)));
        if (c->slab.bytes != old_slab || old_slab == 0 || c->slab_dirty) {  // every slot EMPTY
            HIP_TRY(launch_fill_u64(c->slab.as<u64>(), 0xFFFFFFFF00000000ull, c->slab.bytes / sizeof(u64), s));
            c->slab_dirty = false;
        }
        HIP_TRY(c->slab_pending.ensure(2 * sizeof(uint32_t)));  // pending, repeats
        HIP_TRY(launch_fill_u32(c->slab_pending.as<uint32_t>(), 0, 2, s));
        HIP_TRY(c->cand.ensure((size_t)P.n_items * kTopK * sizeof(u64)));
        HIP_TRY(c->thr.ensure((size_t)P.n_items * sizeof(uint32_t)));
        HIP_TRY(launch_fill_u32(c->tcount.as<uint32_t>(), 0, H, s));
        HIP_TRY(launch_fill_u64(c->best.as<u64>(), 0, H, s));
        HIP_TRY(launch_fill_u64(c->own_sum.as<u64>(), 0, H, s));
        HIP_TRY(launch_fill_u64(c->rowsum.as<u64>(), 0, H, s));
    }

    // internal CSR
    uint32_t *w2 = g->w ? c->w2.as<uint32_t>() : nullptr;
    const Bins &B = P.bins;
    if (fuse) HIP_TRY(launch_init_labels(La, fuse->L1, c->old_of.as<uint32_t>(), nullptr, n, s));
    if (fuse && fuse->rest_n) HIP_TRY(launch_fill_u32(fuse->rest_n, 0, NBINS, s));
    const HubState hs = hub_state(c);
    uint16_t *bnd = nullptr;
    uint64_t *isrc = nullptr;
    if (const uint32_t S = relabel_slices(n); S && P.n_items) {
        HIP_TRY(c->hub_bnd.ensure((size_t)P.n_items * (S + 1) * sizeof(uint16_t)));
        HIP_TRY(c->hub_src.ensure((size_t)P.n_items * sizeof(uint64_t)));
        bnd = c->hub_bnd.as<uint16_t>();
        isrc = c->hub_src.as<uint64_t>();
    }
    HIP_TRY(launch_relabel_hub(G, c->old_of.as<uint32_t>(), c->new_of.as<uint32_t>(), c->rp2.as<uint64_t>(),
                               c->col2.as<uint32_t>(), w2, c->items.as<HubItem>(), P.n_items,
                               c->hflags.as<uint32_t>(), err_dev, (fuse && with_slab) ? fuse : nullptr, &hs, P.H,
                               bnd, isrc, s));
    HIP_TRY(launch_relabel_rows(G, c->old_of.as<uint32_t>(), c->new_of.as<uint32_t>(), c->rp2.as<uint64_t>(),
                                c->col2.as<uint32_t>(), w2, c->rowflag.as<uint8_t>(), B.lo[BIN_WIDE],
                                B.cnt[BIN_WIDE] + B.cnt[BIN_WAVE], B.lo[BIN_WAVE], BIN_WIDE, BIN_WAVE, 1, err_dev,
                                fuse, s));
    HIP_TRY(launch_relabel_rows(G, c->old_of.as<uint32_t>(), c->new_of.as<uint32_t>(), c->rp2.as<uint64_t>(),
                                c->col2.as<uint32_t>(), w2, c->rowflag.as<uint8_t>(), B.lo[BIN_GROUP],
                                B.cnt[BIN_GROUP] + B.cnt[BIN_THREAD], B.lo[BIN_THREAD], BIN_GROUP, BIN_THREAD, 0,
                                err_dev, fuse, s));
    if (with_slab) {
        c->prep_key = csr_key(c, g);
        c->prep_plan = P;
    }
    return LPA_OK;
}

// Per-run state of the long rows, as prepare() leaves it (with_slab).
lpa_status reset_hub_state(lpa_ctx *c, const Plan &P) {
    const hipStream_t s = c->stream;
    if (!P.H) return LPA_OK;
    if (c->slab_dirty) {
        HIP_TRY(launch_fill_u64(c->slab.as<u64>(), 0xFFFFFFFF00000000ull, c->slab.bytes / sizeof(u64), s));
        c->slab_dirty = false;
    }
    HIP_TRY(launch_fill_u32(c->slab_pending.as<uint32_t>(), 0, 2, s));
    HIP_TRY(launch_fill_u32(c->tcount.as<uint32_t>(), 0, P.H, s));
    HIP_TRY(launch_fill_u64(c->best.as<u64>(), 0, P.H, s));
    HIP_TRY(launch_fill_u64(c->own_sum.as<u64>(), 0, P.H, s));
    HIP_TRY(launch_fill_u64(c->rowsum.as<u64>(), 0, P.H, s));
    return LPA_OK;
}

// Enqueue every vote kernel of one round.  first = round 1 from L0(v) = v.
lpa_status enqueue_round(lpa_ctx *c, const Plan &P, const RoundArgs &ra, const HubState &hs, bool weighted,
                         int first, int feat = 0, uint32_t *const *lists = nullptr,
                         const uint32_t *list_n = nullptr) {
    const hipStream_t s = c->stream;
    // algorithmic bytes: per arc col, weight, gathered label; per vertex
    // row_ptr, own label read, new label write (rows of a list: unknown here)
    const uint64_t ab = weighted ? 12 : 8;
    const Bins &B = P.bins;
    const int cap = c->num_cu;  // the launchers size grids from it
    const bool rest = ra.skip_distinct != 0;  // round 1 after the relabel pass voted the distinct rows
    auto bytes = [&](int b) { return (lists || rest) ? 0ull : ab * B.arcs[b] + 16ull * B.cnt[b]; };
    auto args = [&](int b) {
        RoundArgs r = ra;
        if (lists) {
            r.list = lists[b];
            r.list_n = list_n + b;
        }
        return r;
    };
    auto kid = [&](int k) { return rest ? (int)K_HUB1 : (lists ? (int)K_LISTED : k); };
    LPA_TRY(timed(c, kid(K_THREAD), bytes(BIN_THREAD), B.arcs[BIN_THREAD], [&] {
        return launch_vote_thread(args(BIN_THREAD), B.lo[BIN_THREAD], B.cnt[BIN_THREAD], first, feat, cap, s);
    }));
    LPA_TRY(timed(c, kid(K_GROUP), bytes(BIN_GROUP), B.arcs[BIN_GROUP], [&] {
        return launch_vote_group(args(BIN_GROUP), B.lo[BIN_GROUP], B.cnt[BIN_GROUP], first, feat, cap, s);
    }));
    LPA_TRY(timed(c, kid(K_WAVE), bytes(BIN_WAVE), B.arcs[BIN_WAVE], [&] {
        return launch_vote_wave(args(BIN_WAVE), B.lo[BIN_WAVE], B.cnt[BIN_WAVE], 0, first, feat, cap, s);
    }));
    LPA_TRY(timed(c, kid(K_WIDE), bytes(BIN_WIDE), B.arcs[BIN_WIDE], [&] {
        return launch_vote_wave(args(BIN_WIDE), B.lo[BIN_WIDE], B.cnt[BIN_WIDE], 1, first, feat, cap, s);
    }));
    if (P.H) {
        const uint32_t *mrows = c->mrows.as<uint32_t>();
        LPA_TRY(timed(c, (first && rest) ? K_HUB1 : K_HUB, bytes(BIN_HUB), B.arcs[BIN_HUB], [&] {
            return launch_vote_hub(ra, c->items.as<HubItem>(), P.n_items, hs, first, ra.skip_distinct ? 1 : 0,
                                   cap, s);
        }));
        LPA_TRY(timed(c, K_MERGE, 0, 0, [&] {
            hipError_t e = launch_hub_merge(ra, hs, mrows, P.n_mwave, 0, first, s);
            if (e == hipSuccess) e = launch_hub_merge(ra, hs, mrows + P.n_mwave, P.n_mblock, 1, first, s);
            return e;
        }));
        LPA_TRY(timed(c, K_FALLBACK, 0, 0, [&] {
            return launch_hub_fallback(ra, c->items.as<HubItem>(), P.n_items, hs, cap, s);
        }));
        LPA_TRY(timed(c, K_REDUCE, 0, 0, [&] {
            return launch_hub_reduce(ra, hs, c->ritems.as<ReduceItem>(), P.n_ritems, s);
        }));
        LPA_TRY(timed(c, K_FINAL, 0, 0, [&] { return launch_hub_final(ra, hs, P.H, first, s); }));
    }
    return LPA_OK;
}

// Modularity of the internal labels L on the internal graph.  With L_prev
// (the labels before the last round of a plain run, every row voted in it)
// and insum (that round's own-label weight sum = Sigma_in of L_prev), only the
// arcs of rows whose label changed in the last round are read.
lpa_status modularity_internal(lpa_ctx *c, const lpa_csr *g, const Plan &P, const uint32_t *L, uint32_t *err_dev,
                               double *q_out, uint64_t *terms, const uint32_t *L_prev = nullptr,
                               u64 insum = 0) {
    const hipStream_t s = c->stream;
    const uint32_t n = g->n;
    const uint32_t nparts = 1024;
    HIP_TRY(c->K.ensure((size_t)n * sizeof(u64)));
    HIP_TRY(c->mod_sums.ensure(2 * sizeof(u64)));
    HIP_TRY(c->partials.ensure(2 * nparts * sizeof(u64)));
    const Bins &B = P.bins;
    const uint64_t wb = g->w ? 12 : 8;
    LPA_TRY(timed(c, K_MOD, L_prev ? 0ull : wb * g->m + 28ull * n, L_prev ? 0ull : g->m, [&]() -> hipError_t {
        hipError_t e = launch_fill_u64(c->K.as<u64>(), 0, n, s);
        if (e == hipSuccess) e = launch_fill_u64(c->mod_sums.as<u64>(), 0, 2, s);
        ModArgs ma;
        ma.g = internal_graph(c, g);
        ma.labels = L;
        ma.K = c->K.as<u64>();
        ma.sums = c->mod_sums.as<u64>();
        ma.err = err_dev;
        ma.labels_prev = L_prev;
        if (e == hipSuccess)
            e = launch_mod_rows(ma, B.lo[BIN_GROUP], B.cnt[BIN_GROUP] + B.cnt[BIN_THREAD], 0, s);
        if (e == hipSuccess) e = launch_mod_rows(ma, B.lo[BIN_WIDE], B.cnt[BIN_WIDE] + B.cnt[BIN_WAVE], 1, s);
        if (e == hipSuccess) e = launch_mod_hub(ma, c->items.as<HubItem>(), P.n_items, s);
        if (e == hipSuccess) e = launch_mod_sumsq(c->K.as<u64>(), n, c->partials.as<u64>(), nparts, s);
        return e;
    }));
    // read back into pinned memory (no staging copy): the block partials,
    // the two sums, the error word
    LPA_TRY(ensure_pinned(c, 16 + 2 * (size_t)nparts + 2));
    const uint64_t *parts = c->pinned + 16;
    const uint64_t *sums = parts + 2 * nparts;
    HIP_TRY(hipMemcpyAsync(c->pinned + 16, c->partials.p, 2 * nparts * sizeof(u64), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(c->pinned + 16 + 2 * nparts, c->mod_sums.p, 2 * sizeof(u64), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(c->pinned + 1, err_dev, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (c->opt.profile) collect_profile(c);
    const uint32_t errbits = reinterpret_cast<const uint32_t *>(c->pinned + 1)[0];
    if (errbits) return err_status(errbits);
    unsigned __int128 sk2 = 0;
    for (uint32_t i = 0; i < nparts; ++i)
        sk2 += ((unsigned __int128)parts[2 * i + 1] << 64) | (unsigned __int128)parts[2 * i];
    const u64 two_m = sums[0], sigma_in = L_prev ? insum + sums[1] : sums[1];  // mod 2^64: the change may be negative
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

void clear_stats(lpa_stats *stats) {
    if (!stats) return;
    stats->iterations = 0;
    stats->converged = 0;
    stats->changed_last = 0;
    stats->arcs_processed = 0;
    stats->ms_total = 0;
    stats->ms_rounds = 0;
    stats->ms_prepare = 0;
    stats->modularity = 0;
    for (int i = 0; i < 4; ++i) stats->mod_terms[i] = 0;
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
    clear_stats(stats);
    if (n == 0) return LPA_OK;

    // semi-synchronous rounds and hashed ties: every row is voted by the
    // round kernels (no round 1 in the relabel pass, which votes strictly
    // from the unique labels) and, for semi-synchronous rounds, modularity
    // by the full pass (a round's own-label sums mix two labelings)
    const bool semi = c->opt.order == LPA_ORDER_SEMISYNC;
    const bool plain_order = !semi && c->opt.tie == LPA_TIE_LOWEST;
    // per round: changed counter words, then (with modularity) own-label
    // weight sums; one word of error bits after them
    const bool want_insum = c->opt.modularity != 0 && !semi;
    const size_t rwords = (size_t)max_iter * kCountWords;
    const size_t cwords = rwords * (want_insum ? 2 : 1) + 1;
    HIP_TRY(c->counters.ensure(cwords * sizeof(u64)));
    u64 *counters = c->counters.as<u64>();
    u64 *insums = want_insum ? counters + rwords : nullptr;
    uint32_t *err_dev = reinterpret_cast<uint32_t *>(counters + cwords - 1);
    HIP_TRY(launch_fill_u64(counters, 0, cwords, s));
    LPA_TRY(ensure_pinned(c, 2 * kCountWords + 16));  // round counts and own-label sums
    if (resume) HIP_TRY(launch_check_labels(labels, n, err_dev, s));

    Plan P;
    HIP_TRY(c->La.ensure((size_t)n * sizeof(uint32_t)));
    HIP_TRY(c->Lb.ensure((size_t)n * sizeof(uint32_t)));
    // the internal copy of this CSR, kept from an earlier call
    const bool reuse = c->opt.reuse_csr && !c->prep_key.empty() && c->prep_key == csr_key(c, g);
    // from the unique labels, round 1 of the rows that list each neighbour
    // once is done while the internal CSR is built
    const bool fused = !reuse && !resume && max_iter > 0 && plain_order;
    HIP_TRY(c->r1_rows.ensure((size_t)n * sizeof(uint32_t)));
    HIP_TRY(c->r1_cnt.ensure(NBINS * sizeof(uint32_t)));
    const Round1Fuse fz{c->Lb.as<uint32_t>(), counters, c->opt.self_weight, c->r1_rows.as<uint32_t>(),
                        c->r1_cnt.as<uint32_t>()};
    if (!c->round_a) HIP_TRY(hipEventCreate(&c->round_a));
    if (!c->round_b) HIP_TRY(hipEventCreate(&c->round_b));
    if (!c->prep_a) HIP_TRY(hipEventCreate(&c->prep_a));
    if (!c->prep_b) HIP_TRY(hipEventCreate(&c->prep_b));
    HIP_TRY(hipEventRecord(c->prep_a, s));
    if (reuse) {
        P = c->prep_plan;
        LPA_TRY(reset_hub_state(c, P));
    } else {
        LPA_TRY(prepare(c, g, P, err_dev, true, fused ? &fz : nullptr, c->La.as<uint32_t>()));
    }
    if (!fused)
        HIP_TRY(launch_init_labels(c->La.as<uint32_t>(), c->Lb.as<uint32_t>(), c->old_of.as<uint32_t>(),
                                   resume ? labels : nullptr, n, s));
    HIP_TRY(hipEventRecord(c->prep_b, s));  // read once the first round has synchronised

    const uint64_t thr = (uint64_t)std::floor(tol * (double)n);
    const bool weighted = g->w != nullptr;
    const HubState hs = hub_state(c);
    const Bins &B = P.bins;
    const uint64_t voted_arcs =
        B.arcs[BIN_THREAD] + B.arcs[BIN_GROUP] + B.arcs[BIN_WAVE] + B.arcs[BIN_WIDE] + B.arcs[BIN_HUB];

    uint32_t *L_old = c->La.as<uint32_t>(), *L_new = c->Lb.as<uint32_t>();
    uint32_t it = 0;
    int converged = 0;
    u64 changed = 0, insum_last = 0;
    double ms_rounds = 0;
    for (uint32_t t = 1; t <= max_iter; ++t) {
        RoundArgs ra;
        ra.g = internal_graph(c, g);
        ra.L_old = L_old;
        ra.L_new = L_new;
        ra.rowflag = c->rowflag.as<uint8_t>();
        ra.sw = c->opt.self_weight;
        ra.check = (t == 1);
        ra.changed = counters + (size_t)(t - 1) * kCountWords;
        ra.err = err_dev;
        ra.list = nullptr;
        ra.list_n = nullptr;
        ra.top1 = ra.top2 = nullptr;
        // round 1 from the unique labels (its single-occurrence shortcuts);
        // the second half of a semi-synchronous round 1 reads labels the
        // first half changed, so those rounds take the general path
        const int first = (t == 1 && !resume && plain_order) ? 1 : 0;
        ra.skip_distinct = (first && fused) ? 1 : 0;
        ra.insum = insums ? insums + (size_t)(t - 1) * kCountWords : nullptr;
        ra.half = 0;
        ra.tie = c->opt.tie;
        ra.t = t;
        ra.seed = c->opt.seed;
        ra.orig = c->old_of.as<uint32_t>();
        HIP_TRY(hipEventRecord(c->round_a, s));
        if (first && fused) {  // just the rows the relabel pass queued
            uint32_t *r1l[NBINS];
            for (int b = 0; b < NBINS; ++b) r1l[b] = c->r1_rows.as<uint32_t>() + B.lo[b];
            LPA_TRY(enqueue_round(c, P, ra, hs, weighted, first, 0, r1l, c->r1_cnt.as<uint32_t>()));
        } else if (semi) {
            // half 1 writes every row of L_new (its rows voted, the others
            // copied), half 2 reads that and writes every row of L_old; a
            // vertex votes in one half only, so both add to the same counts
            ra.half = 1;
            LPA_TRY(enqueue_round(c, P, ra, hs, weighted, 0));
            ra.half = 2;
            ra.L_old = L_new;
            ra.L_new = L_old;
            LPA_TRY(enqueue_round(c, P, ra, hs, weighted, 0));
        } else {
            LPA_TRY(enqueue_round(c, P, ra, hs, weighted, first));
        }
        HIP_TRY(hipEventRecord(c->round_b, s));
        HIP_TRY(hipMemcpyAsync(c->pinned + 16, ra.changed, kCountWords * sizeof(u64), hipMemcpyDeviceToHost, s));
        if (ra.insum)  // read with the round's counts: no extra round trip after the last round
            HIP_TRY(hipMemcpyAsync(c->pinned + 16 + kCountWords, ra.insum, kCountWords * sizeof(u64),
                                   hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(c->pinned + 1, err_dev, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        // (per-kernel timings are folded in after the run: between rounds
        // the device waits for the host)
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, c->round_a, c->round_b);
        ms_rounds += ms;
        const uint32_t errbits = reinterpret_cast<uint32_t *>(c->pinned + 1)[0];
        if (errbits) return err_status(errbits);
        changed = 0;
        insum_last = 0;
        for (int k = 0; k < kCountSlots; ++k) {
            changed += c->pinned[16 + (size_t)k * kCountStride];
            if (ra.insum) insum_last += c->pinned[16 + kCountWords + (size_t)k * kCountStride];
        }
        it = t;
        if (stats) {
            if (stats->changed_per_iter && t <= stats->cap) stats->changed_per_iter[t - 1] = changed;
            if (stats->ms_per_iter && t <= stats->cap) stats->ms_per_iter[t - 1] = ms;
        }
        if (!semi) std::swap(L_old, L_new);  // a semi-synchronous round ends in L_old
        if (changed <= thr) {
            converged = 1;
            break;
        }
    }
    HIP_TRY(launch_scatter_labels(labels, c->old_of.as<uint32_t>(), L_old, n, s));
    double q = 0;
    uint64_t terms[4] = {0, 0, 0, 0};
    if (c->opt.modularity) {
        // after round 1 every row voted in round it (round 1 may have been
        // voted by the relabel pass, which does not sum own-label weights);
        // modularity_internal ends with a synchronisation and an error check
        if (it >= 2 && !semi)
            LPA_TRY(modularity_internal(c, g, P, L_old, err_dev, &q, terms, L_new, insum_last));
        else
            LPA_TRY(modularity_internal(c, g, P, L_old, err_dev, &q, terms));
    } else {
        HIP_TRY(hipMemcpyAsync(c->pinned + 1, err_dev, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (c->opt.profile) collect_profile(c);
        const uint32_t errbits = reinterpret_cast<uint32_t *>(c->pinned + 1)[0];
        if (errbits) return err_status(errbits);
    }
    if (stats) {
        stats->iterations = it;
        stats->converged = converged;
        stats->changed_last = changed;
        stats->arcs_processed = voted_arcs * it;
        stats->ms_rounds = ms_rounds;
        float ms_prep = 0.f;
        (void)hipEventElapsedTime(&ms_prep, c->prep_a, c->prep_b);
        stats->ms_prepare = ms_prep;
        stats->modularity = q;
        for (int i = 0; i < 4; ++i) stats->mod_terms[i] = terms[i];
        stats->ms_total =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    }
    return LPA_OK;
}

// -------------------------------------------------- frontier / learned --
//
// One engine runs three kinds of run on the relabelled graph:
//   exact    rounds >= 2 vote only the vertices that can change (lossless);
//   learned  rounds >= 2 vote the candidates the network keeps, then a full
//            check round, then plain rounds if the check fails;
//   trace    every round votes every vertex; before each round t >= 2 the
//            features of the rows of at most wide_max arcs are written out,
//            after it whether they changed.
// Round 1 always votes every vertex (from the unique labels).  The vote
// kernels record each row's winning and runner-up tally (FEAT); after every
// round the push kernels stamp the rows that may change next.

uint16_t host_bf16(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
float host_bf16_float(float f) {
    const uint32_t u = (uint32_t)host_bf16(f) << 16;
    float r;
    std::memcpy(&r, &u, 4);
    return r;
}

// Model in the MFMA lane layouts (MlpDev, lpa_internal.h).
MlpDev make_mlp_dev(const lpa_mlp &m) {
    MlpDev d;
    std::memset(&d, 0, sizeof(d));
    for (int l = 0; l < 64; ++l) {
        uint64_t w = 0;
        for (int c = 0; c < 4; ++c) {
            const int k = 4 * (l / 32) + c;
            const float x = k < 6 ? m.w1[k][l % 32] : 0.f;
            w |= (uint64_t)host_bf16(x) << (16 * c);
        }
        d.a1[l] = w;
        for (int st = 0; st < 4; ++st) {
            uint64_t w2 = 0;
            for (int c = 0; c < 4; ++c) w2 |= (uint64_t)host_bf16(m.w2[8 * st + 4 * (l / 32) + c][l % 32]) << (16 * c);
            d.a2[st][l] = w2;
        }
    }
    for (int j = 0; j < 32; ++j) {
        d.b1[j] = m.b1[j];
        d.b2[j] = m.b2[j];
        d.w3[j] = host_bf16_float(m.w3[j]);
    }
    d.b3 = m.b3;
    const double tau = m.tau;
    d.zcut = tau <= 0.0 ? -INFINITY : (tau >= 1.0 ? INFINITY : (float)std::log(tau / (1.0 - tau)));
    return d;
}

enum FrontMode { F_EXACT, F_LEARNED, F_TRACE };

struct FrontRun {
    FrontMode mode = F_EXACT;
    const lpa_mlp *model = nullptr;
    uint8_t *masks = nullptr;
    uint32_t mask_rounds = 0;
    float *tX = nullptr;
    uint8_t *ty = nullptr;
    uint64_t tcap = 0, tcount = 0;
    // results
    uint32_t iterations = 0;
    int converged = 0;
    uint32_t learned_rounds = 0, check_round = 0;
    uint64_t changed_last = 0, arcs = 0;
    double ms_rounds = 0;
    std::vector<u64> changed, voted, cands;
    std::vector<float> ms;
    double q = 0;
    uint64_t terms[4] = {0, 0, 0, 0};
};

lpa_status frontier_impl(lpa_ctx *c, const lpa_csr *g, uint32_t *labels, double tol, uint32_t max_iter,
                         FrontRun &R) {
    if (c->opt.order != LPA_ORDER_SYNC || c->opt.tie != LPA_TIE_LOWEST) return LPA_EUNSUPPORTED;
    LPA_TRY(check_csr_args(g));
    if (!labels && g->n && R.mode != F_TRACE) return LPA_EINVAL;
    if (!(tol >= 0.0 && tol <= 1.0)) return LPA_EINVAL;
    HIP_TRY(hipSetDevice(c->device));
    const hipStream_t s = c->stream;
    const uint32_t n = g->n;
    if (n == 0) return LPA_OK;
    // per round: changed counter words, then (with modularity) own-label
    // weight sums of the rounds that vote every row; the error word last
    const bool want_insum = c->opt.modularity && labels;
    const size_t rwords = (size_t)std::max<uint32_t>(max_iter, 1) * kCountWords;
    const size_t cwords = rwords * (want_insum ? 2 : 1) + 1;
    HIP_TRY(c->counters.ensure(cwords * sizeof(u64)));
    u64 *counters = c->counters.as<u64>();
    u64 *insums = want_insum ? counters + rwords : nullptr;
    uint32_t *err_dev = reinterpret_cast<uint32_t *>(counters + (cwords - 1));
    HIP_TRY(launch_fill_u64(counters, 0, cwords, s));
    LPA_TRY(ensure_pinned(c, kCountWords + 32));
    Plan P;
    HIP_TRY(c->La.ensure((size_t)n * 4));
    HIP_TRY(c->Lb.ensure((size_t)n * 4));
    // round 1 of the rows that list each neighbour once is voted while the
    // internal CSR is built, as in lpa_run; it leaves no top-two tallies,
    // so round 2 votes every vertex (it changes nearly every label anyway)
    // and the first prediction uses round 2's tallies.  Traces keep round 1
    // in the vote kernels for the features of round 2.
    const bool fused = R.mode != F_TRACE && max_iter > 0;
    HIP_TRY(c->r1_rows.ensure((size_t)n * sizeof(uint32_t)));
    HIP_TRY(c->r1_cnt.ensure(NBINS * sizeof(uint32_t)));
    const Round1Fuse fz{c->Lb.as<uint32_t>(), counters, c->opt.self_weight, c->r1_rows.as<uint32_t>(),
                        c->r1_cnt.as<uint32_t>()};
    LPA_TRY(prepare(c, g, P, err_dev, true, fused ? &fz : nullptr, c->La.as<uint32_t>()));
    const Bins &B = P.bins;
    if (!fused)
        HIP_TRY(launch_init_labels(c->La.as<uint32_t>(), c->Lb.as<uint32_t>(), c->old_of.as<uint32_t>(), nullptr, n,
                                   s));
    for (DevBuf *b : {&c->f_top1, &c->f_top2, &c->f_last, &c->f_front}) HIP_TRY(b->ensure((size_t)n * 4));
    HIP_TRY(c->f_stale.ensure(n));
    HIP_TRY(c->f_lists.ensure((size_t)n * 4));
    HIP_TRY(c->f_small.ensure(64));  // list counts [8], candidates, kept arcs, expected skipped changes
    HIP_TRY(launch_fill_u32(c->f_last.as<uint32_t>(), 0, n, s));
    HIP_TRY(launch_fill_u32(c->f_front.as<uint32_t>(), 0, n, s));
    HIP_TRY(launch_fill_u32(c->f_top1.as<uint32_t>(), 0, n, s));
    HIP_TRY(launch_fill_u32(c->f_top2.as<uint32_t>(), 0, n, s));
    HIP_TRY(launch_fill_u64(reinterpret_cast<u64 *>(c->f_stale.p), 0, ((size_t)n + 7) / 8, s));
    const Graph gi = internal_graph(c, g);
    const uint32_t *kw = nullptr;
    if (g->w) {
        HIP_TRY(c->f_kw.ensure((size_t)n * 4));
        HIP_TRY(launch_row_sums(gi, c->f_kw.as<uint32_t>(), s));
        kw = c->f_kw.as<uint32_t>();
    }
    if (R.mode == F_LEARNED) {
        if (!R.model) return LPA_EINVAL;
        const MlpDev md = make_mlp_dev(*R.model);
        HIP_TRY(c->f_model.ensure(sizeof(MlpDev)));
        HIP_TRY(hipMemcpyAsync(c->f_model.p, &md, sizeof(MlpDev), hipMemcpyHostToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));  // md lives on this stack frame
    }
    // per-bin lists over the non-long bins, in one buffer
    uint32_t *lists[NBINS] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    {
        uint32_t off = 0;
        for (int b = BIN_WIDE; b <= BIN_THREAD; ++b) {
            lists[b] = c->f_lists.as<uint32_t>() + off;
            off += B.cnt[b];
        }
    }
    uint32_t *list_n = c->f_small.as<uint32_t>();                          // [NBINS]
    u64 *cand_dev = reinterpret_cast<u64 *>(c->f_small.as<char>() + 32);  // candidates
    const uint32_t nonhub_lo = B.lo[BIN_WIDE];
    const uint32_t nonhub_cnt = B.cnt[BIN_WIDE] + B.cnt[BIN_WAVE] + B.cnt[BIN_GROUP] + B.cnt[BIN_THREAD];
    const uint64_t nonisolated = (uint64_t)nonhub_cnt + B.cnt[BIN_HUB];
    const uint64_t thr = (uint64_t)std::floor(tol * (double)n);
    const bool weighted = g->w != nullptr;
    const HubState hs = hub_state(c);
    const uint64_t all_arcs = B.arcs[BIN_THREAD] + B.arcs[BIN_GROUP] + B.arcs[BIN_WAVE] + B.arcs[BIN_WIDE] +
                              B.arcs[BIN_HUB];
    // below this many changed vertices the next round's candidates are
    // tracked exactly; above it every vertex counts as a candidate
    const uint64_t push_limit = nonisolated / 4;
    if (!c->round_a) HIP_TRY(hipEventCreate(&c->round_a));
    if (!c->round_b) HIP_TRY(hipEventCreate(&c->round_b));

    uint32_t *L_old = c->La.as<uint32_t>(), *L_new = c->Lb.as<uint32_t>();
    int all_dirty = 1;
    bool last_full = false;  // the last round voted every row (incremental modularity applies)
    // learned runs predict only after a round that recorded top-two tallies
    // and changed fewer than half of the non-isolated vertices; while more
    // change, the network would keep nearly every candidate and a full round
    // (plain RAK) is cheaper
    bool feat_prev = false;
    bool quiet = false;  // the last round changed fewer than half of the non-isolated vertices
    enum { PH_LEARN, PH_CHECK, PH_PLAIN } phase = R.mode == F_LEARNED ? PH_LEARN : PH_PLAIN;
    for (uint32_t t = 1; t <= max_iter; ++t) {
        RoundArgs ra;
        ra.g = gi;
        ra.L_old = L_old;
        ra.L_new = L_new;
        ra.rowflag = c->rowflag.as<uint8_t>();
        ra.sw = c->opt.self_weight;
        ra.check = t == 1;
        ra.changed = counters + (size_t)(t - 1) * kCountWords;
        ra.err = err_dev;
        ra.list = nullptr;
        ra.list_n = nullptr;
        ra.skip_distinct = (t == 1 && fused) ? 1 : 0;
        ra.insum = nullptr;
        ra.half = 0;  // synchronous rounds, strict ties
        ra.tie = 0;
        ra.t = t;
        ra.seed = 0;
        ra.orig = nullptr;
        ra.top1 = c->f_top1.as<uint32_t>();
        ra.top2 = c->f_top2.as<uint32_t>();
        FrontArgs fa;
        fa.g = gi;
        fa.L_old = L_old;
        fa.L_new = L_new;
        fa.top1 = ra.top1;
        fa.top2 = ra.top2;
        fa.kw = kw;
        fa.lastchg = c->f_last.as<uint32_t>();
        fa.front = c->f_front.as<uint32_t>();
        fa.stale = c->f_stale.as<uint8_t>();
        fa.mask = (R.masks && t - 1 < R.mask_rounds) ? R.masks + (size_t)(t - 1) * n : nullptr;
        fa.old_of = c->old_of.as<uint32_t>();
        fa.cand_count = cand_dev;
        fa.kept_arcs = cand_dev + 1;
        fa.exp_skip = cand_dev + 2;
        fa.sw = c->opt.self_weight;
        fa.t = t;
        fa.max_iter = max_iter;
        fa.all_dirty = all_dirty;
        fa.keep_all = phase != PH_LEARN;
        // full: every non-isolated row votes, no candidate lists (round 1,
        // traces, and rounds in which every row is a candidate anyway)
        const bool learn = R.mode == F_LEARNED && phase == PH_LEARN;
        const bool full = t == 1 || R.mode == F_TRACE || (learn ? !(feat_prev && quiet) : all_dirty != 0);
        const bool learned_round = learn && !full;
        // the tallies feed the features of the next round's prediction
        const int feat = R.mode == F_TRACE || (learn && quiet && !(t == 1 && fused));
        ra.insum = (full && insums) ? insums + (size_t)(t - 1) * kCountWords : nullptr;
        last_full = full;
        uint64_t trace_base = R.tcount;
        HIP_TRY(hipEventRecord(c->round_a, s));
        if (full) {
            if (fa.mask) HIP_TRY(launch_mask_rows(fa.mask, fa.old_of, 0, n, 1, s));
            if (R.mode == F_LEARNED && R.learned_rounds)
                HIP_TRY(launch_fill_u64(reinterpret_cast<u64 *>(c->f_stale.p), 0, ((size_t)n + 7) / 8, s));
            if (R.mode == F_TRACE && t >= 2 && R.tX && trace_base + nonhub_cnt <= R.tcap)
                HIP_TRY(launch_trace_x(fa, nonhub_lo, nonhub_cnt, R.tX + trace_base * 6, s));
            if (t == 1 && fused) {  // just the rows the relabel pass queued
                uint32_t *r1l[NBINS];
                for (int b = 0; b < NBINS; ++b) r1l[b] = c->r1_rows.as<uint32_t>() + B.lo[b];
                LPA_TRY(enqueue_round(c, P, ra, hs, weighted, 1, feat, r1l, c->r1_cnt.as<uint32_t>()));
            } else {
                LPA_TRY(enqueue_round(c, P, ra, hs, weighted, t == 1 ? 1 : 0, feat));
            }
        } else {
            HIP_TRY(launch_fill_u32(list_n, 0, NBINS, s));
            HIP_TRY(launch_fill_u64(cand_dev, 0, 3, s));
            LPA_TRY(timed(c, K_PREDICT, 0, 0, [&]() -> hipError_t {
                for (int b = BIN_WIDE; b <= BIN_THREAD; ++b) {
                    const hipError_t e = launch_predict(fa, c->f_model.as<MlpDev>(), B.lo[b], B.cnt[b], lists[b],
                                                        list_n + b, c->num_cu, s);
                    if (e != hipSuccess) return e;
                }
                return hipSuccess;
            }));
            if (fa.mask) {
                HIP_TRY(launch_mask_rows(fa.mask, fa.old_of, B.lo[BIN_HUB], B.cnt[BIN_HUB], 1, s));
                HIP_TRY(launch_mask_rows(fa.mask, fa.old_of, B.lo[BIN_ZERO], B.cnt[BIN_ZERO], 0, s));
            }
            LPA_TRY(enqueue_round(c, P, ra, hs, weighted, 0, feat, lists, list_n));
        }
        HIP_TRY(hipEventRecord(c->round_b, s));
        HIP_TRY(hipMemcpyAsync(c->pinned + 16, ra.changed, kCountWords * sizeof(u64), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(c->pinned + 1, err_dev, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        if (!full) HIP_TRY(hipMemcpyAsync(c->pinned + 2, c->f_small.p, 56, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (c->opt.profile) collect_profile(c);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, c->round_a, c->round_b);
        R.ms_rounds += ms;
        const uint32_t errbits = reinterpret_cast<uint32_t *>(c->pinned + 1)[0];
        if (errbits) return err_status(errbits);
        u64 changed = 0;
        for (int k = 0; k < kCountSlots; ++k) changed += c->pinned[16 + (size_t)k * kCountStride];
        u64 voted = nonisolated, cand = nonisolated, arcs = all_arcs, expected_skipped = 0;
        if (!full) {
            const uint32_t *ln = reinterpret_cast<const uint32_t *>(c->pinned + 2);
            voted = B.cnt[BIN_HUB];
            for (int b = BIN_WIDE; b <= BIN_THREAD; ++b) voted += ln[b];
            cand = c->pinned[2 + 4] + B.cnt[BIN_HUB];
            arcs = c->pinned[2 + 5] + B.arcs[BIN_HUB];
            expected_skipped = (c->pinned[2 + 6] + 512) / 1024;
        }
        if (R.mode == F_TRACE && t >= 2) {
            if (R.ty && trace_base + nonhub_cnt <= R.tcap)
                HIP_TRY(launch_trace_y(L_old, L_new, nonhub_lo, nonhub_cnt, R.ty + trace_base, s));
            R.tcount += nonhub_cnt;
        }
        R.changed.push_back(changed);
        R.voted.push_back(voted);
        R.cands.push_back(cand);
        R.ms.push_back(ms);
        R.arcs += arcs;
        R.iterations = t;
        R.changed_last = changed;
        if (learned_round) ++R.learned_rounds;
        quiet = 2 * changed < nonisolated;
        feat_prev = feat != 0;
        // which vertices can change next round (not needed when the next
        // round votes every row anyway: a learned-phase round after a full
        // one without a prediction to feed)
        const bool next_full = learn && full && !(feat_prev && quiet);
        if (!next_full || R.mode != F_LEARNED) {
            const int mark = R.mode == F_TRACE || changed <= push_limit;
            fa.t = t;
            LPA_TRY(timed(c, K_PUSH, 0, 0, [&] { return launch_push(fa, B, mark, s); }));
            all_dirty = !mark;
        } else {
            all_dirty = 1;
        }
        std::swap(L_old, L_new);
        if (t == 1 && R.mode != F_TRACE) {
            if (changed <= thr) {
                R.converged = 1;
                break;
            }
            continue;
        }
        if (R.mode == F_TRACE || phase == PH_PLAIN) {
            if (changed <= thr) {
                R.converged = 1;
                break;
            }
        } else if (phase == PH_LEARN && full) {
            // a full round is a full sweep: its count is the tolerance test
            if (changed <= thr) {
                R.converged = 1;
                break;
            }
        } else if (phase == PH_LEARN) {
            // the skipped rows would have changed with the predicted
            // probabilities: stop predicting once the expected full-round
            // count passes the tolerance test.  Stop too when the predictor
            // kept nearly every candidate: the next round then votes the
            // whole frontier anyway, so it might as well be the check.
            if (changed + expected_skipped <= thr || (learned_round && 5 * voted >= 4 * cand)) {
                phase = PH_CHECK;
                R.check_round = t + 1;
            }
        } else {  // the full check
            if (changed <= thr) {
                R.converged = 1;
                break;
            }
            phase = PH_PLAIN;
        }
    }
    if (labels) HIP_TRY(launch_scatter_labels(labels, c->old_of.as<uint32_t>(), L_old, n, s));
    if (want_insum) {
        if (last_full && R.iterations >= 2) {
            HIP_TRY(hipMemcpyAsync(c->pinned + 16, insums + (size_t)(R.iterations - 1) * kCountWords,
                                   kCountWords * sizeof(u64), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            u64 ins = 0;
            for (int k = 0; k < kCountSlots; ++k) ins += c->pinned[16 + (size_t)k * kCountStride];
            LPA_TRY(modularity_internal(c, g, P, L_old, err_dev, &R.q, R.terms, L_new, ins));
        } else {
            LPA_TRY(modularity_internal(c, g, P, L_old, err_dev, &R.q, R.terms));
        }
    }
    HIP_TRY(hipMemcpyAsync(c->pinned + 1, err_dev, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const uint32_t errbits = reinterpret_cast<uint32_t *>(c->pinned + 1)[0];
    if (errbits) return err_status(errbits);
    return LPA_OK;
}

// ---------------------------------------------------------------- training --

constexpr int kMlpParams = 6 * 32 + 32 + 32 * 32 + 32 + 32 + 1;

uint64_t splitmix(uint64_t &x) {
    uint64_t z = (x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t gcd64(uint64_t a, uint64_t b) {
    while (b) {
        const uint64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

lpa_status ensure_train_bufs(lpa_ctx *c, uint32_t max_batch, uint32_t epochs) {
    const uint32_t nblk = (max_batch + 255) / 256;
    HIP_TRY(c->t_w.ensure(kMlpParams * 4));
    HIP_TRY(c->t_m.ensure(kMlpParams * 4));
    HIP_TRY(c->t_v.ensure(kMlpParams * 4));
    HIP_TRY(c->t_part.ensure((size_t)nblk * (kMlpParams + 1) * 4));
    HIP_TRY(c->t_grad.ensure((kMlpParams + 1) * 4));
    HIP_TRY(c->t_loss.ensure((size_t)std::max<uint32_t>(epochs, 1) * 4));
    return LPA_OK;
}

}  // namespace

namespace {

// ------------------------------------------------------------- batched run --
//
// lpa_run_batch: the packed CSR is binned and relabelled once like a single
// graph (its arcs never leave their graph, so each graph's rows only read
// its own labels); gid maps internal vertices to graphs.  The state reset,
// the persistent kernel that runs every round of every graph and the output
// scatter are captured in one HIP graph, re-captured only when a launch
// parameter changes.

struct BatchLayout {
    u64 *thr, *changed, *last, *hist, *arcs, *clock;
    uint32_t *active, *iters, *n_active, *bar, *btot;
    int32_t *conv;
    size_t bytes;
};

BatchLayout batch_layout(void *base, uint32_t G, uint32_t hist_len) {
    BatchLayout L;
    char *p = static_cast<char *>(base);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *q = p ? p + off : nullptr;
        off += (bytes + 255) & ~(size_t)255;
        return q;
    };
    L.thr = reinterpret_cast<u64 *>(take((size_t)G * 8));
    L.changed = reinterpret_cast<u64 *>(take((size_t)G * 8));
    L.last = reinterpret_cast<u64 *>(take((size_t)G * 8));
    L.hist = reinterpret_cast<u64 *>(take((size_t)G * hist_len * 8));
    L.arcs = reinterpret_cast<u64 *>(take(8));
    L.clock = reinterpret_cast<u64 *>(take(16));
    L.active = reinterpret_cast<uint32_t *>(take((size_t)G * 4));
    L.iters = reinterpret_cast<uint32_t *>(take((size_t)G * 4));
    L.conv = reinterpret_cast<int32_t *>(take((size_t)G * 4));
    L.n_active = reinterpret_cast<uint32_t *>(take(8));
    L.bar = reinterpret_cast<uint32_t *>(take(kBatchBarWords * 4));
    L.btot = reinterpret_cast<uint32_t *>(take((size_t)kBatchBins * kBatchMaxBlocks * 4));
    L.bytes = off;
    return L;
}

constexpr uint32_t kBatchHistMax = 1024;  // rounds whose per-graph counts are kept
constexpr double kBarrierTimeoutS = 10.0;

void clear_batch_stats(lpa_batch_stats *st, uint32_t G) {
    if (!st) return;
    st->graphs = G;
    st->rounds = 0;
    st->converged_graphs = 0;
    st->arcs_processed = 0;
    st->ms_total = 0;
    st->ms_device = 0;
}

lpa_status run_batch_impl(lpa_ctx *c, const lpa_csr *g, const uint64_t *gv, uint32_t G, uint32_t *labels,
                          double tol, uint32_t max_iter, lpa_batch_stats *stats) {
    const auto t_start = std::chrono::steady_clock::now();
    if (!c) return LPA_EINVAL;
    if (c->opt.order != LPA_ORDER_SYNC || c->opt.tie != LPA_TIE_LOWEST) return LPA_EUNSUPPORTED;
    LPA_TRY(check_csr_args(g));
    if (!gv && G) return LPA_EINVAL;
    if (!labels && g->n) return LPA_EINVAL;
    if (!(tol >= 0.0 && tol <= 1.0)) return LPA_EINVAL;
    // the one-lane vote pads short rows with labels 0xFFFFFFFF - j, j < 32
    if (g->n > 0xFFFFFFFFu - kSortNetMax + 1) return LPA_EINVAL;
    if (G == 0) {
        if (g->n) return LPA_EINVAL;
        clear_batch_stats(stats, 0);
        return LPA_OK;
    }
    if (gv[0] != 0 || gv[G] != g->n) return LPA_EINVAL;
    for (uint32_t k = 0; k < G; ++k)
        if (gv[k + 1] < gv[k]) return LPA_EINVAL;
    HIP_TRY(hipSetDevice(c->device));
    const hipStream_t s = c->stream;
    const uint32_t n = g->n;
    clear_batch_stats(stats, G);
    const uint32_t hist_len = std::min<uint32_t>(max_iter, kBatchHistMax);
    std::vector<uint64_t> thr_h(G);
    for (uint32_t k = 0; k < G; ++k) thr_h[k] = (uint64_t)std::floor(tol * (double)(gv[k + 1] - gv[k]));

    std::vector<uint32_t> it_h(G, 0);
    std::vector<int32_t> conv_h(G, 0);
    std::vector<u64> last_h(G, 0), hist_h((size_t)G * hist_len, 0);
    u64 arcs_h = 0;
    double ms_dev = 0;
    if (n == 0) {
        // every graph is empty: one round that changes nothing
        if (max_iter > 0) {
            std::fill(it_h.begin(), it_h.end(), 1u);
            std::fill(conv_h.begin(), conv_h.end(), 1);
        }
    } else {
        HIP_TRY(c->counters.ensure(sizeof(u64)));
        uint32_t *err_dev = reinterpret_cast<uint32_t *>(c->counters.as<u64>());
        HIP_TRY(launch_fill_u64(c->counters.as<u64>(), 0, 1, s));
        LPA_TRY(ensure_pinned(c, 16));
        Plan P;
        // reuse_csr: the internal copy, the vertices' graphs and the graphs'
        // segments kept from the last batch on the same CSR and graph_vptr
        std::vector<uint64_t> bkey = csr_key(c, g);
        bkey.push_back(G);
        bkey.insert(bkey.end(), gv, gv + (size_t)G + 1);
        const bool reuse = c->opt.reuse_csr && !c->prep_key.empty() && c->prep_key == csr_key(c, g) &&
                           c->bprep_key == bkey;
        if (reuse) {
            P = c->prep_plan;
            LPA_TRY(reset_hub_state(c, P));
        } else {
            LPA_TRY(prepare(c, g, P, err_dev, true));
            HIP_TRY(c->gvd.ensure(((size_t)G + 1) * sizeof(uint64_t)));
            HIP_TRY(hipMemcpyAsync(c->gvd.p, gv, ((size_t)G + 1) * sizeof(uint64_t), hipMemcpyHostToDevice, s));
            HIP_TRY(c->gid.ensure((size_t)n * sizeof(uint32_t)));
            HIP_TRY(launch_batch_gid(c->old_of.as<uint32_t>(), n, c->gvd.as<uint64_t>(), G, c->gid.as<uint32_t>(), s));
        }
        HIP_TRY(c->La.ensure((size_t)n * sizeof(uint32_t)));
        HIP_TRY(c->Lb.ensure((size_t)n * sizeof(uint32_t)));
        HIP_TRY(launch_init_labels(c->La.as<uint32_t>(), c->Lb.as<uint32_t>(), c->old_of.as<uint32_t>(), nullptr, n,
                                   s));
        const Bins &B = P.bins;
        const int slots = batch_slots(B);
        const uint64_t units = (uint64_t)B.cnt[BIN_HUB] + B.cnt[BIN_WIDE] + B.cnt[BIN_WAVE] +
                               (B.cnt[BIN_GROUP] + 63) / 64 + (B.cnt[BIN_THREAD] + 63) / 64;
        const uint32_t wpb = (uint32_t)batch_waves_per_block();
        const uint64_t cap_blocks =
            std::min<uint64_t>((uint64_t)batch_blocks_per_cu(slots) * c->num_cu, kBatchMaxBlocks);
        const uint32_t nblocks =
            (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(cap_blocks, (units + wpb - 1) / wpb));
        HIP_TRY(c->bstate.ensure(batch_layout(nullptr, G, hist_len).bytes));
        const BatchLayout L = batch_layout(c->bstate.p, G, hist_len);
        HIP_TRY(hipMemcpyAsync(L.thr, thr_h.data(), (size_t)G * 8, hipMemcpyHostToDevice, s));
        const size_t seg_words = (size_t)kBatchBins * G;
        const size_t pref_words = (size_t)kBatchBins * ((size_t)G + 1);
        HIP_TRY(c->bseg.ensure((2 * seg_words + pref_words) * sizeof(uint32_t)));
        uint32_t *seg_lo = c->bseg.as<uint32_t>(), *seg_cnt = seg_lo + seg_words;
        uint32_t *pref = seg_cnt + seg_words;
        if (!reuse) {
            HIP_TRY(launch_batch_seg(c->gid.as<uint32_t>(), B, G, seg_lo, seg_cnt, s));
            c->bprep_key = bkey;
        }

        BatchArgs b;
        std::memset(&b, 0, sizeof(b));
        b.g = internal_graph(c, g);
        b.L0 = c->La.as<uint32_t>();
        b.L1 = c->Lb.as<uint32_t>();
        b.gid = c->gid.as<uint32_t>();
        b.gv = c->gvd.as<uint64_t>();
        b.orp = g->row_ptr;
        b.sw = c->opt.self_weight;
        for (int k = 0; k < NBINS; ++k) {
            b.lo[k] = B.lo[k];
            b.cnt[k] = B.cnt[k];
        }
        b.G = G;
        b.max_iter = max_iter;
        b.thr = L.thr;
        b.active = L.active;
        b.iters = L.iters;
        b.conv = L.conv;
        b.changed = L.changed;
        b.last = L.last;
        b.hist = L.hist;
        b.hist_len = hist_len;
        b.arcs = L.arcs;
        b.n_active = L.n_active;
        b.bar = L.bar;
        b.err = err_dev;
        const HubState hs = hub_state(c);
        b.slab_off = hs.slab_off;
        b.slab_mask = hs.slab_mask;
        b.touched_off = hs.touched_off;
        b.slab = hs.slab;
        b.touched = hs.touched;
        b.tcount = hs.tcount;
        b.seg_lo = seg_lo;
        b.seg_cnt = seg_cnt;
        b.pref = pref;
        b.btot = L.btot;
        b.dshift = 0;
        while (((uint64_t)nblocks << b.dshift) < G) ++b.dshift;
        b.clock = L.clock;
        int rate_khz = 0;
        HIP_TRY(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, c->device));
        if (rate_khz <= 0) rate_khz = 100000;
        const double limit_ms =
            c->opt.barrier_timeout_us ? 1e-3 * (double)c->opt.barrier_timeout_us : kBarrierTimeoutS * 1e3;
        b.timeout_ticks = (uint64_t)(limit_ms * (double)rate_khz);
        // the captured graph depends on exactly these values
        std::vector<unsigned char> key(sizeof(b) + sizeof(nblocks) + sizeof(labels) + sizeof(n) + sizeof(s) +
                                       sizeof(slots));
        {
            unsigned char *k = key.data();
            std::memcpy(k, &b, sizeof(b));
            k += sizeof(b);
            std::memcpy(k, &nblocks, sizeof(nblocks));
            k += sizeof(nblocks);
            std::memcpy(k, &labels, sizeof(labels));
            k += sizeof(labels);
            std::memcpy(k, &n, sizeof(n));
            k += sizeof(n);
            std::memcpy(k, &s, sizeof(s));
            k += sizeof(s);
            std::memcpy(k, &slots, sizeof(slots));
        }
        if (!c->bexec || key != c->bkey) {
            if (c->bexec) {
                (void)hipGraphExecDestroy(c->bexec);
                c->bexec = nullptr;
            }
            if (!c->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
            const hipStream_t cs = c->cap_stream;
            HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
            hipError_t e = launch_fill_u32(L.active, 1, G, cs);
            if (e == hipSuccess) e = launch_fill_u32(L.iters, 0, G, cs);
            if (e == hipSuccess) e = launch_fill_u32(reinterpret_cast<uint32_t *>(L.conv), 0, G, cs);
            if (e == hipSuccess) e = launch_fill_u64(L.changed, 0, G, cs);
            if (e == hipSuccess) e = launch_fill_u64(L.last, 0, G, cs);
            if (e == hipSuccess && hist_len) e = launch_fill_u64(L.hist, 0, (uint64_t)G * hist_len, cs);
            if (e == hipSuccess) e = launch_fill_u64(L.arcs, 0, 1, cs);
            if (e == hipSuccess) e = launch_fill_u32(L.n_active, 0, 2, cs);
            if (e == hipSuccess) e = launch_fill_u32(L.bar, 0, kBatchBarWords, cs);
            if (e == hipSuccess) e = launch_fill_u64(L.clock, 0, 2, cs);
            if (e == hipSuccess && max_iter) e = launch_batch(b, nblocks, slots, cs);
            if (e == hipSuccess)
                e = launch_batch_out(labels, c->old_of.as<uint32_t>(), c->gid.as<uint32_t>(), b.L0, b.L1, L.iters,
                                     b.gv, n, cs);
            hipGraph_t graph = nullptr;
            const hipError_t e2 = hipStreamEndCapture(cs, &graph);
            if (e == hipSuccess) e = e2;
            if (e == hipSuccess) e = hipGraphInstantiate(&c->bexec, graph, nullptr, nullptr, 0);
            if (graph) (void)hipGraphDestroy(graph);
            if (e != hipSuccess) {
                c->bexec = nullptr;
                return dev_status(e);
            }
            c->bkey = key;
        }
        HIP_TRY(hipGraphLaunch(c->bexec, s));
        uint32_t errbits = 0;
        HIP_TRY(hipMemcpyAsync(&errbits, err_dev, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(it_h.data(), L.iters, (size_t)G * 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(conv_h.data(), L.conv, (size_t)G * 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(last_h.data(), L.last, (size_t)G * 8, hipMemcpyDeviceToHost, s));
        if (stats && stats->changed_hist && hist_len)
            HIP_TRY(hipMemcpyAsync(hist_h.data(), L.hist, hist_h.size() * 8, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(&arcs_h, L.arcs, 8, hipMemcpyDeviceToHost, s));
        u64 clock_h[2] = {0, 0};
        HIP_TRY(hipMemcpyAsync(clock_h, L.clock, 16, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        ms_dev = clock_h[1] > clock_h[0] ? (double)(clock_h[1] - clock_h[0]) / (double)rate_khz : 0.0;
        if (errbits & ERR_TIMEOUT) c->slab_dirty = true;
        if (errbits) return err_status(errbits);
    }
    if (stats) {
        uint32_t rounds = 0, nconv = 0;
        for (uint32_t k = 0; k < G; ++k) {
            rounds = std::max(rounds, it_h[k]);
            nconv += conv_h[k] ? 1u : 0u;
            if (stats->iterations) stats->iterations[k] = it_h[k];
            if (stats->converged) stats->converged[k] = conv_h[k];
            if (stats->changed_last) stats->changed_last[k] = last_h[k];
        }
        if (stats->changed_hist && stats->hist_cap) {
            const uint32_t hc = stats->hist_cap;
            for (uint32_t k = 0; k < G; ++k)
                for (uint32_t t = 0; t < hc; ++t)
                    stats->changed_hist[(size_t)k * hc + t] = t < hist_len ? hist_h[(size_t)k * hist_len + t] : 0;
        }
        stats->rounds = rounds;
        stats->converged_graphs = nconv;
        stats->arcs_processed = arcs_h;
        stats->ms_device = ms_dev;
        stats->ms_total =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    }
    return LPA_OK;
}

// Modularity (as lpa_modularity) of labels on the caller's CSR as stored,
// without the binning and relabelled copy: the kernels of
// lpa_modularity_noalloc with the context's buffers.
lpa_status modularity_direct(lpa_ctx *c, const Graph &G, const uint32_t *labels, double *q_out, uint64_t *terms) {
    const hipStream_t s = c->stream;
    const uint32_t nparts = 1024;
    HIP_TRY(c->K.ensure((size_t)G.n * sizeof(u64)));
    HIP_TRY(c->mod_sums.ensure(8 * sizeof(u64)));
    HIP_TRY(c->partials.ensure(2 * nparts * sizeof(u64)));
    u64 *sums = c->mod_sums.as<u64>();
    LPA_TRY(timed(c, K_MOD, 0, 0, [&] {
        return launch_modularity_any(G, labels, c->K.as<u64>(), sums, reinterpret_cast<uint32_t *>(sums + 2),
                                     c->partials.as<u64>(), nparts, sums + 3, s);
    }));
    LPA_TRY(ensure_pinned(c, 8));
    HIP_TRY(hipMemcpyAsync(c->pinned, sums + 3, 5 * sizeof(u64), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (c->opt.profile) collect_profile(c);
    const uint64_t *res = c->pinned;
    if (res[4]) return err_status((uint32_t)res[4]);
    const unsigned __int128 sk2 = ((unsigned __int128)res[1] << 64) | (unsigned __int128)res[0];
    const u64 two_m = res[2], sigma_in = res[3];
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

// ------------------------------------------------------------------ COPRA --
//
// Rounds of COPRA (lpa_copra.hip) on the caller's CSR.  Per half-round: the
// wavefront and block kernels, one read-back of the changed count and of the
// number of rows whose distinct labels outgrew the block's LDS table; those
// rows (if any) are then voted with tables in device memory sized from their
// degrees, and their changes are read back too.
lpa_status copra_impl(lpa_ctx *c, const lpa_csr *g, uint32_t V, uint32_t *best_out, uint32_t *state_lab,
                      uint32_t *state_coef, uint32_t *state_cnt, double tol, uint32_t max_iter, lpa_stats *stats) {
    const auto t_start = std::chrono::steady_clock::now();
    if (!c) return LPA_EINVAL;
    LPA_TRY(check_csr_args(g));
    if (!best_out && g->n) return LPA_EINVAL;
    if (!(tol >= 0.0 && tol <= 1.0)) return LPA_EINVAL;
    if (V < 1 || V > 64) return LPA_EINVAL;
    if (c->opt.frontier) return LPA_EUNSUPPORTED;
    HIP_TRY(hipSetDevice(c->device));
    const hipStream_t s = c->stream;
    const uint32_t n = g->n;
    clear_stats(stats);
    if (n == 0) return LPA_OK;
    const Graph G{g->row_ptr, g->col, g->w, n, g->m};
    // counters: kCountWords changed words, then the overflow count (word
    // kCountWords), the error word (kCountWords + 1) and the kCopraClasses
    // row-list sizes (u32 from word kCountWords + 2 on)
    HIP_TRY(c->counters.ensure((kCountWords + 8) * sizeof(u64)));
    u64 *cw = c->counters.as<u64>();
    uint32_t *ovf_count = reinterpret_cast<uint32_t *>(cw + kCountWords);
    uint32_t *err = reinterpret_cast<uint32_t *>(cw + kCountWords + 1);
    uint32_t *list_count = reinterpret_cast<uint32_t *>(cw + kCountWords + 2);
    LPA_TRY(ensure_pinned(c, kCountWords + 32));
    HIP_TRY(launch_fill_u64(cw, 0, kCountWords + 8, s));
    HIP_TRY(c->cp_distinct.ensure(n));
    HIP_TRY(c->cp_wsum.ensure((size_t)n * sizeof(u64)));
    HIP_TRY(launch_csr_check(G, err, c->cp_distinct.as<uint8_t>(), c->cp_wsum.as<u64>(), s));
    HIP_TRY(hipMemcpyAsync(c->pinned, err, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (const uint32_t bits = reinterpret_cast<uint32_t *>(c->pinned)[0]) return err_status(bits);

    const uint32_t stride = copra_stride(V);
    for (int b = 0; b < 2; ++b) HIP_TRY(c->cp_rec[b].ensure((size_t)n * stride * sizeof(uint32_t)));
    HIP_TRY(c->cp_rows.ensure((size_t)n * sizeof(uint32_t)));
    HIP_TRY(c->cp_rows1.ensure((size_t)n * sizeof(uint32_t)));
    HIP_TRY(c->cp_rows2.ensure((size_t)n * sizeof(uint32_t)));
    HIP_TRY(c->cp_rows3.ensure((size_t)n * sizeof(uint32_t)));
    // both buffers start alone: rows without arcs are never voted again
    for (int b = 0; b < 2; ++b) HIP_TRY(launch_copra_init(n, stride, c->cp_rec[b].as<uint32_t>(), s));
    uint32_t *const list_w[kCopraClasses] = {c->cp_rows.as<uint32_t>(), c->cp_rows1.as<uint32_t>(),
                                             c->cp_rows2.as<uint32_t>(), c->cp_rows3.as<uint32_t>()};
    HIP_TRY(launch_copra_list(G, V, list_w, list_count, s));
    HIP_TRY(hipMemcpyAsync(c->pinned, list_count, kCopraClasses * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    uint32_t n_list[kCopraClasses];
    std::memcpy(n_list, c->pinned, sizeof(n_list));
    const uint32_t *lists[kCopraClasses] = {list_w[0], list_w[1], list_w[2], list_w[3]};
    const uint32_t n_big = n_list[kCopraClasses - 1];
    HIP_TRY(c->cp_ovf.ensure((size_t)(n_big ? n_big : 1) * sizeof(uint32_t)));

    const uint64_t thr = (uint64_t)std::floor(tol * (double)n);
    const bool semi = c->opt.order == LPA_ORDER_SEMISYNC;
    const uint64_t wb = g->w ? 20 : 16;  // per arc: col (+ weight), count and first slot of the neighbour
    int cur = 0;
    uint32_t it = 0;
    int32_t converged = 0;
    uint64_t changed = 0;
    double ms_rounds = 0;
    if (!c->round_a) HIP_TRY(hipEventCreate(&c->round_a));
    if (!c->round_b) HIP_TRY(hipEventCreate(&c->round_b));
    for (uint32_t t = 1; t <= max_iter; ++t) {
        changed = 0;
        float ms_t = 0.f;
        for (uint32_t h = 0; h <= (semi ? 1u : 0u); ++h) {
            const int nx = cur ^ 1;
            CopraArgs a;
            a.g = G;
            a.V = V;
            a.stride = stride;
            a.in = c->cp_rec[cur].as<uint32_t>();
            a.out = c->cp_rec[nx].as<uint32_t>();
            a.t = t;
            a.half = semi ? h + 1 : 0;
            a.tie = c->opt.tie;
            a.seed = c->opt.seed;
            a.changed = cw;
            a.ovf_rows = c->cp_ovf.as<uint32_t>();
            a.ovf_count = ovf_count;
            a.err = err;
            a.first = t == 1 && h == 0;  // before any vertex voted
            a.distinct = c->cp_distinct.as<uint8_t>();
            HIP_TRY(launch_fill_u64(cw, 0, kCountWords + 1, s));  // changed words and the overflow count
            HIP_TRY(hipEventRecord(c->round_a, s));
            // a half-round votes about half of the arcs; the whole round's
            // bytes are charged to its first launch
            const uint64_t bytes = h ? 0 : wb * g->m + 28ull * n;
            LPA_TRY(timed(c, K_COPRA, bytes, h ? 0 : g->m,
                          [&] { return launch_copra_round(a, lists, n_list, s); }));
            HIP_TRY(hipEventRecord(c->round_b, s));
            // changed words, overflow count, error word
            HIP_TRY(hipMemcpyAsync(c->pinned, cw, (kCountWords + 2) * sizeof(u64), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, c->round_a, c->round_b);
            ms_t += ms;
            const uint32_t n_ovf = reinterpret_cast<uint32_t *>(c->pinned + kCountWords)[0];
            if (n_ovf) {
                // tables in device memory for the rows the LDS could not
                // hold, filled by pieces of at most 2048 / V arcs
                const uint32_t per = 2048u / V;
                HIP_TRY(c->cp_off.ensure(((size_t)n_ovf + 1) * sizeof(u64)));
                HIP_TRY(c->cp_first.ensure((size_t)n_ovf * sizeof(u64)));
                HIP_TRY(launch_copra_sizes(G, V, a.ovf_rows, n_ovf, per, c->cp_off.as<u64>(), c->cp_first.as<u64>(),
                                           s));
                std::vector<u64> off((size_t)n_ovf + 1), first((size_t)n_ovf);
                HIP_TRY(hipMemcpyAsync(off.data(), c->cp_off.p, (size_t)n_ovf * sizeof(u64), hipMemcpyDeviceToHost,
                                       s));
                HIP_TRY(hipMemcpyAsync(first.data(), c->cp_first.p, (size_t)n_ovf * sizeof(u64),
                                       hipMemcpyDeviceToHost, s));
                HIP_TRY(hipStreamSynchronize(s));
                std::vector<u64> sfirst((size_t)n_ovf);
                u64 total = 0, npieces = 0, nslices = 0;
                for (uint32_t i = 0; i < n_ovf; ++i) {
                    const u64 sz = off[i], np = first[i];
                    off[i] = total;
                    first[i] = npieces;
                    sfirst[i] = nslices;
                    total += sz;
                    npieces += np;
                    nslices += (sz + kCopraSliceSlots - 1) / kCopraSliceSlots;
                }
                off[n_ovf] = total;
                HIP_TRY(c->cp_sfirst.ensure((size_t)n_ovf * sizeof(u64)));
                HIP_TRY(hipMemcpyAsync(c->cp_off.p, off.data(), off.size() * sizeof(u64), hipMemcpyHostToDevice, s));
                HIP_TRY(hipMemcpyAsync(c->cp_first.p, first.data(), first.size() * sizeof(u64), hipMemcpyHostToDevice,
                                       s));
                HIP_TRY(hipMemcpyAsync(c->cp_sfirst.p, sfirst.data(), sfirst.size() * sizeof(u64),
                                       hipMemcpyHostToDevice, s));
                const size_t rs_words = (size_t)(5 + 2 * V) * n_ovf;
                HIP_TRY(c->cp_slices.ensure((size_t)nslices * sizeof(CopraPiece)));
                HIP_TRY(c->cp_rowstate.ensure(rs_words * sizeof(u64)));
                HIP_TRY(launch_fill_u64(c->cp_rowstate.as<u64>(), 0, rs_words, s));
                HIP_TRY(c->cp_key.ensure((size_t)total * sizeof(uint32_t)));
                HIP_TRY(c->cp_tal.ensure((size_t)total * sizeof(u64)));
                HIP_TRY(c->cp_pieces.ensure((size_t)npieces * sizeof(CopraPiece)));
                HIP_TRY(c->cp_total.ensure((size_t)n_ovf * sizeof(u64)));
                HIP_TRY(launch_fill_u32(c->cp_key.as<uint32_t>(), 0xFFFFFFFFu, total, s));
                HIP_TRY(launch_fill_u64(c->cp_tal.as<u64>(), 0, total, s));
                HIP_TRY(launch_fill_u64(c->cp_total.as<u64>(), 0, n_ovf, s));
                HIP_TRY(hipEventRecord(c->round_a, s));
                LPA_TRY(timed(c, K_COPRA_GLOBAL, 0, 0, [&] {
                    return launch_copra_global(a, a.ovf_rows, n_ovf, c->cp_first.as<u64>(), per,
                                               c->cp_pieces.as<CopraPiece>(), npieces, c->cp_off.as<u64>(),
                                               c->cp_key.as<uint32_t>(), c->cp_tal.as<u64>(), c->cp_total.as<u64>(),
                                               c->cp_sfirst.as<u64>(), c->cp_slices.as<CopraPiece>(), nslices,
                                               c->cp_rowstate.as<u64>(), s);
                }));
                HIP_TRY(hipEventRecord(c->round_b, s));
                HIP_TRY(hipMemcpyAsync(c->pinned, cw, (kCountWords + 2) * sizeof(u64), hipMemcpyDeviceToHost, s));
                HIP_TRY(hipStreamSynchronize(s));
                (void)hipEventElapsedTime(&ms, c->round_a, c->round_b);
                ms_t += ms;
            }
            for (int k = 0; k < kCountSlots; ++k) changed += c->pinned[(size_t)k * kCountStride];
            cur = nx;
            if (const uint32_t bits = reinterpret_cast<uint32_t *>(c->pinned + kCountWords + 1)[0])
                return err_status(bits);
        }
        ms_rounds += ms_t;
        it = t;
        if (stats) {
            if (stats->changed_per_iter && t <= stats->cap) stats->changed_per_iter[t - 1] = changed;
            if (stats->ms_per_iter && t <= stats->cap) stats->ms_per_iter[t - 1] = ms_t;
        }
        if (changed <= thr) {
            converged = 1;
            break;
        }
    }
    HIP_TRY(launch_copra_output(c->cp_rec[cur].as<uint32_t>(), n, V, stride, best_out, state_lab, state_coef,
                                state_cnt, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (c->opt.profile) collect_profile(c);
    double q = 0;
    uint64_t terms[4] = {0, 0, 0, 0};
    if (c->opt.modularity) LPA_TRY(modularity_direct(c, G, best_out, &q, terms));
    if (stats) {
        stats->iterations = it;
        stats->converged = converged;
        stats->changed_last = changed;
        stats->arcs_processed = g->m * it;
        stats->ms_rounds = ms_rounds;
        stats->modularity = q;
        for (int i = 0; i < 4; ++i) stats->mod_terms[i] = terms[i];
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
    opt->wave_max = 128;
    opt->wide_max = 512;
    opt->merge_max = 512;
    opt->profile = 0;
    opt->modularity = 0;
    opt->frontier = 0;
    opt->barrier_timeout_us = 0;
    opt->order = LPA_ORDER_SYNC;
    opt->tie = LPA_TIE_LOWEST;
    opt->seed = 0;
    opt->reuse_csr = 0;
}

lpa_status lpa_init(lpa_ctx **ctx, int device, void *stream, const lpa_options *opt) {
    if (!ctx) return LPA_EINVAL;
    *ctx = nullptr;
    lpa_options o;
    lpa_default_options(&o);
    if (opt) {
        const lpa_options d = o;
        o = *opt;
        if (!o.thread_max) o.thread_max = d.thread_max;
        if (!o.group_max) o.group_max = d.group_max;
        if (!o.wave_max) o.wave_max = d.wave_max;
        if (!o.wide_max) o.wide_max = d.wide_max;
        if (!o.merge_max) o.merge_max = d.merge_max;
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
    // address of lpa_modularity_noalloc's fixed scratch on this device; a
    // failed lookup is retried (and reported) by that entry point
    (void)noalloc_attach(device);
    for (int k = 0; k < K_COUNT; ++k) {
        std::memset(&c->prof[k], 0, sizeof(lpa_kernel_prof));
        std::snprintf(c->prof[k].name, sizeof(c->prof[k].name), "%s", kKernelNames[k]);
    }
    *ctx = c;
    return LPA_OK;
}

lpa_status lpa_run(lpa_ctx *ctx, const lpa_csr *g, uint32_t *labels_out, double tol, uint32_t max_iter,
                   lpa_stats *stats) {
    if (!ctx || !ctx->opt.frontier) return run_impl(ctx, g, labels_out, tol, max_iter, stats, false);
    const auto t0 = std::chrono::steady_clock::now();
    clear_stats(stats);
    FrontRun R;
    R.mode = F_EXACT;
    LPA_TRY(frontier_impl(ctx, g, labels_out, tol, max_iter, R));
    if (stats) {
        stats->iterations = R.iterations;
        stats->converged = R.converged;
        stats->changed_last = R.changed_last;
        stats->arcs_processed = R.arcs;
        stats->ms_rounds = R.ms_rounds;
        stats->modularity = R.q;
        for (int i = 0; i < 4; ++i) stats->mod_terms[i] = R.terms[i];
        for (uint32_t t = 0; t < R.iterations && t < stats->cap; ++t) {
            if (stats->changed_per_iter) stats->changed_per_iter[t] = R.changed[t];
            if (stats->ms_per_iter) stats->ms_per_iter[t] = R.ms[t];
        }
        stats->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    return LPA_OK;
}

lpa_status lpa_run_learned(lpa_ctx *ctx, const lpa_csr *g, const lpa_mlp *model, uint32_t *labels_out,
                           double tol, uint32_t max_iter, lpa_learned_stats *stats, uint8_t *masks,
                           uint32_t mask_rounds) {
    const auto t0 = std::chrono::steady_clock::now();
    if (!ctx || !model) return LPA_EINVAL;
    if (!(model->tau >= 0.f && model->tau <= 1.f)) return LPA_EINVAL;
    if (stats) {
        stats->iterations = 0;
        stats->converged = 0;
        stats->learned_rounds = 0;
        stats->check_round = 0;
        stats->changed_last = 0;
        stats->arcs_processed = 0;
        stats->ms_total = stats->ms_rounds = 0;
        stats->modularity = 0;
        for (int i = 0; i < 4; ++i) stats->mod_terms[i] = 0;
    }
    FrontRun R;
    R.mode = F_LEARNED;
    R.model = model;
    R.masks = masks;
    R.mask_rounds = masks ? mask_rounds : 0;
    LPA_TRY(frontier_impl(ctx, g, labels_out, tol, max_iter, R));
    if (stats) {
        stats->iterations = R.iterations;
        stats->converged = R.converged;
        stats->learned_rounds = R.learned_rounds;
        stats->check_round = R.check_round <= R.iterations ? R.check_round : 0;
        stats->changed_last = R.changed_last;
        stats->arcs_processed = R.arcs;
        stats->ms_rounds = R.ms_rounds;
        stats->modularity = R.q;
        for (int i = 0; i < 4; ++i) stats->mod_terms[i] = R.terms[i];
        for (uint32_t t = 0; t < R.iterations && t < stats->cap; ++t) {
            if (stats->changed_per_iter) stats->changed_per_iter[t] = R.changed[t];
            if (stats->voted_per_iter) stats->voted_per_iter[t] = R.voted[t];
            if (stats->candidates_per_iter) stats->candidates_per_iter[t] = R.cands[t];
        }
        stats->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    return LPA_OK;
}

lpa_status lpa_trace(lpa_ctx *ctx, const lpa_csr *g, double tol, uint32_t max_iter, float *X, uint8_t *y,
                     uint64_t cap, uint64_t *count) {
    if (!ctx || !count || (cap && (!X || !y))) return LPA_EINVAL;
    *count = 0;
    FrontRun R;
    R.mode = F_TRACE;
    R.tX = X;
    R.ty = y;
    R.tcap = cap;
    LPA_TRY(frontier_impl(ctx, g, nullptr, tol, max_iter, R));
    *count = R.tcount;
    return LPA_OK;
}

lpa_status lpa_mlp_forward(lpa_ctx *ctx, const lpa_mlp *model, const float *X, uint64_t N, float *z) {
    if (!ctx || !model || (N && (!X || !z))) return LPA_EINVAL;
    HIP_TRY(hipSetDevice(ctx->device));
    const MlpDev md = make_mlp_dev(*model);
    HIP_TRY(ctx->f_model.ensure(sizeof(MlpDev)));
    HIP_TRY(hipMemcpyAsync(ctx->f_model.p, &md, sizeof(MlpDev), hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(launch_mlp_forward(ctx->f_model.as<MlpDev>(), X, N, z, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return LPA_OK;
}

lpa_status lpa_mlp_grad(lpa_ctx *ctx, const lpa_mlp *model, const float *X, const uint8_t *y, uint64_t N,
                        float pos_weight, float *grad, float *loss) {
    if (!ctx || !model || !grad || !N || !X || !y || N > 0x80000000ull) return LPA_EINVAL;
    HIP_TRY(hipSetDevice(ctx->device));
    const hipStream_t s = ctx->stream;
    LPA_TRY(ensure_train_bufs(ctx, (uint32_t)N, 1));
    HIP_TRY(hipMemcpyAsync(ctx->t_w.p, model, kMlpParams * 4, hipMemcpyHostToDevice, s));
    HIP_TRY(launch_train_step(X, y, N, 1, 0, 0, (uint32_t)N, ctx->t_w.as<float>(), ctx->t_m.as<float>(),
                              ctx->t_v.as<float>(), ctx->t_part.as<float>(), ctx->t_grad.as<float>(), pos_weight,
                              0.f, 1.f, 1.f, ctx->t_loss.as<float>(), 0, s));
    std::vector<float> h(kMlpParams + 1);
    HIP_TRY(hipMemcpyAsync(h.data(), ctx->t_grad.p, (kMlpParams + 1) * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    std::memcpy(grad, h.data(), kMlpParams * 4);
    if (loss) *loss = h[kMlpParams] / (float)N;
    return LPA_OK;
}

lpa_status lpa_train(lpa_ctx *ctx, const float *X, const uint8_t *y, uint64_t N, const lpa_train_options *opt,
                     lpa_mlp *model, float *loss_per_epoch) {
    if (!ctx || !opt || !model || !N || !X || !y) return LPA_EINVAL;
    if (!opt->batch || (opt->batch & 255) || !(opt->lr > 0.f) || !(opt->pos_weight > 0.f)) return LPA_EINVAL;
    if (N >= 0xFFFFFFFFull) return LPA_EINVAL;
    if (opt->val_n && (!opt->val_X || !opt->val_y)) return LPA_EINVAL;
    if (opt->val_n && !(opt->recall > 0.f && opt->recall <= 1.f)) return LPA_EINVAL;
    HIP_TRY(hipSetDevice(ctx->device));
    const hipStream_t s = ctx->stream;
    const uint32_t batch = (uint32_t)std::min<uint64_t>(opt->batch, ((N + 255) / 256) * 256);
    LPA_TRY(ensure_train_bufs(ctx, batch, opt->epochs));
    HIP_TRY(hipMemcpyAsync(ctx->t_w.p, model, kMlpParams * 4, hipMemcpyHostToDevice, s));
    HIP_TRY(launch_fill_u32(ctx->t_m.as<uint32_t>(), 0, kMlpParams, s));
    HIP_TRY(launch_fill_u32(ctx->t_v.as<uint32_t>(), 0, kMlpParams, s));
    HIP_TRY(launch_fill_u32(ctx->t_loss.as<uint32_t>(), 0, std::max<uint32_t>(opt->epochs, 1), s));
    uint64_t rng = opt->seed;
    uint64_t step = 0;
    for (uint32_t e = 0; e < opt->epochs; ++e) {
        // sample order of this epoch: i -> (mul * i + add) mod N, mul coprime to N
        uint64_t mul = 1, add = 0;
        if (N > 1) {
            do {
                mul = 1 + splitmix(rng) % (N - 1);
            } while (gcd64(mul, N) != 1);
            add = splitmix(rng) % N;
        }
        for (uint64_t start = 0; start < N; start += batch) {
            const uint32_t bn = (uint32_t)std::min<uint64_t>(batch, N - start);
            ++step;
            const float c1 = 1.f - (float)std::pow(0.9, (double)step);
            const float c2 = 1.f - (float)std::pow(0.999, (double)step);
            HIP_TRY(launch_train_step(X, y, N, mul, add, start, bn, ctx->t_w.as<float>(), ctx->t_m.as<float>(),
                                      ctx->t_v.as<float>(), ctx->t_part.as<float>(), ctx->t_grad.as<float>(),
                                      opt->pos_weight, opt->lr, c1, c2, ctx->t_loss.as<float>() + e, 1, s));
        }
    }
    std::vector<float> lossv(std::max<uint32_t>(opt->epochs, 1));
    HIP_TRY(hipMemcpyAsync(model, ctx->t_w.p, kMlpParams * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(lossv.data(), ctx->t_loss.p, lossv.size() * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (loss_per_epoch)
        for (uint32_t e = 0; e < opt->epochs; ++e) loss_per_epoch[e] = lossv[e] / (float)N;
    if (opt->val_n) {
        // tau: the largest threshold keeping `recall` of the positive samples
        HIP_TRY(ctx->t_z.ensure(opt->val_n * 4));
        lpa_mlp m = *model;
        m.tau = 0.f;
        LPA_TRY(lpa_mlp_forward(ctx, &m, opt->val_X, opt->val_n, ctx->t_z.as<float>()));
        std::vector<float> z(opt->val_n);
        std::vector<uint8_t> yy(opt->val_n);
        HIP_TRY(hipMemcpyAsync(z.data(), ctx->t_z.p, opt->val_n * 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(yy.data(), opt->val_y, opt->val_n, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        std::vector<float> zp;
        for (uint64_t i = 0; i < opt->val_n; ++i)
            if (yy[i]) zp.push_back(z[i]);
        if (zp.empty()) {
            model->tau = 0.5f;
        } else {
            std::sort(zp.begin(), zp.end());
            const size_t k = (size_t)std::floor((1.0 - (double)opt->recall) * (double)zp.size());
            const double thr = zp[std::min(k, zp.size() - 1)];
            model->tau = (float)(1.0 / (1.0 + std::exp(-thr)));
        }
    }
    return LPA_OK;
}

lpa_status lpa_run_resume(lpa_ctx *ctx, const lpa_csr *g, uint32_t *labels_inout, double tol, uint32_t max_iter,
                          lpa_stats *stats) {
    return run_impl(ctx, g, labels_inout, tol, max_iter, stats, true);
}

lpa_status lpa_run_batch(lpa_ctx *ctx, const lpa_csr *packed, const uint64_t *graph_vptr, uint32_t G,
                         uint32_t *labels_out, double tol, uint32_t max_iter, lpa_batch_stats *stats) {
    return run_batch_impl(ctx, packed, graph_vptr, G, labels_out, tol, max_iter, stats);
}

lpa_status lpa_autotune(lpa_ctx *c, const lpa_csr *g, const uint64_t *graph_vptr, uint32_t G, uint32_t rounds,
                        lpa_options *chosen, uint32_t *measured) {
    if (!c) return LPA_EINVAL;
    LPA_TRY(check_csr_args(g));
    if (measured) *measured = 0;
    if (rounds == 0) rounds = 2;
    HIP_TRY(hipSetDevice(c->device));
    const hipStream_t s = c->stream;
    // degree signature: fractions of rows and arcs per power-of-two length
    // bucket, in 1/32 steps, plus the magnitudes of n and m
    std::vector<int> key;
    key.push_back(graph_vptr ? 1 : 0);
    key.push_back(g->w ? 1 : 0);
    key.push_back(g->n ? 31 - __builtin_clz(g->n) : -1);
    key.push_back(g->m ? 63 - __builtin_clzll(g->m) : -1);
    if (g->n) {
        HIP_TRY(c->tune_hist.ensure(2 * kDegBuckets * sizeof(u64)));
        HIP_TRY(launch_fill_u64(c->tune_hist.as<u64>(), 0, 2 * kDegBuckets, s));
        HIP_TRY(launch_degree_hist(g->row_ptr, g->n, c->tune_hist.as<u64>(), s));
        std::vector<u64> h(2 * kDegBuckets);
        HIP_TRY(hipMemcpyAsync(h.data(), c->tune_hist.p, h.size() * sizeof(u64), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        for (int b = 0; b < kDegBuckets; ++b) {
            key.push_back((int)std::lround(32.0 * (double)h[b] / (double)g->n));
            key.push_back(g->m ? (int)std::lround(32.0 * (double)h[kDegBuckets + b] / (double)g->m) : 0);
        }
    }
    auto it = c->tune_cache.find(key);
    if (it == c->tune_cache.end()) {
        const lpa_options saved = c->opt;
        lpa_options best = saved;
        double best_ms = 1e300;
        uint32_t tried = 0;
        if (g->n) {
            HIP_TRY(c->tune_labels.ensure((size_t)g->n * sizeof(uint32_t)));
            const uint32_t tms[] = {4, 8}, gms[] = {16, 32}, wms[] = {64, 128}, xms[] = {256, 512};
            for (uint32_t tm : tms)
                for (uint32_t gm : gms)
                    for (uint32_t wm : wms)
                        for (uint32_t xm : xms) {
                            c->opt.thread_max = tm;
                            c->opt.group_max = gm;
                            c->opt.wave_max = wm;
                            c->opt.wide_max = xm;
                            c->opt.profile = 0;
                            c->opt.modularity = 0;
                            c->opt.frontier = 0;
                            double ms = 1e300;
                            for (int rep = 0; rep < 2; ++rep) {
                                double t = 0;
                                lpa_status st;
                                if (graph_vptr) {
                                    lpa_batch_stats bs;
                                    std::memset(&bs, 0, sizeof(bs));
                                    st = run_batch_impl(c, g, graph_vptr, G, c->tune_labels.as<uint32_t>(), 0.0,
                                                        rounds, &bs);
                                    t = bs.ms_device;
                                } else {
                                    lpa_stats rs;
                                    std::memset(&rs, 0, sizeof(rs));
                                    st = run_impl(c, g, c->tune_labels.as<uint32_t>(), 0.0, rounds, &rs, false);
                                    t = rs.ms_rounds;
                                }
                                if (st != LPA_OK) {
                                    c->opt = saved;
                                    return st;
                                }
                                ms = std::min(ms, t);
                            }
                            ++tried;
                            if (ms < best_ms) {
                                best_ms = ms;
                                best = saved;
                                best.thread_max = tm;
                                best.group_max = gm;
                                best.wave_max = wm;
                                best.wide_max = xm;
                            }
                        }
        }
        c->opt = saved;
        it = c->tune_cache.emplace(key, best).first;
        if (measured) *measured = tried;
    }
    c->opt.thread_max = it->second.thread_max;
    c->opt.group_max = it->second.group_max;
    c->opt.wave_max = it->second.wave_max;
    c->opt.wide_max = it->second.wide_max;
    if (chosen) *chosen = c->opt;
    return LPA_OK;
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
    uint32_t *err_dev = reinterpret_cast<uint32_t *>(c->counters.as<u64>());
    HIP_TRY(launch_fill_u64(c->counters.as<u64>(), 0, 1, s));
    HIP_TRY(launch_check_labels(labels, n, err_dev, s));
    Plan P;
    LPA_TRY(prepare(c, g, P, err_dev, false));
    HIP_TRY(c->La.ensure((size_t)n * sizeof(uint32_t)));
    HIP_TRY(launch_init_labels(c->La.as<uint32_t>(), nullptr, c->old_of.as<uint32_t>(), labels, n, s));
    return modularity_internal(c, g, P, c->La.as<uint32_t>(), err_dev, q_out, terms);
}

lpa_status lpa_run_copra(lpa_ctx *c, const lpa_csr *g, uint32_t max_labels, uint32_t *labels_out,
                         uint32_t *state_labels, uint32_t *state_coefs, uint32_t *state_count, double tol,
                         uint32_t max_iter, lpa_stats *stats) {
    return copra_impl(c, g, max_labels, labels_out, state_labels, state_coefs, state_count, tol, max_iter, stats);
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
    DevBuf *bufs[] = {&c->blk_counts, &c->blk_arcs, &c->small,    &c->old_of,    &c->new_of,      &c->rp2,
                      &c->col2,       &c->w2,       &c->rowflag,  &c->La,        &c->Lb,          &c->counters,
                      &c->items,      &c->ritems,   &c->slab_off, &c->slab_mask, &c->touched_off, &c->tcount,
                      &c->best,       &c->own_sum,  &c->hflags,   &c->rowsum,    &c->slab,        &c->touched,
                      &c->K,          &c->mod_sums, &c->partials, &c->cand,      &c->thr,         &c->item_lo,
                      &c->mrows,      &c->slab_pending, &c->hub_tmp, &c->r1_rows, &c->r1_cnt, &c->hub_bnd,
                      &c->hub_src,    &c->gid,  &c->gvd,      &c->bstate, &c->bseg,
                      &c->f_top1, &c->f_top2, &c->f_kw, &c->f_last, &c->f_front, &c->f_stale, &c->f_lists,
                      &c->f_small, &c->f_model, &c->t_w, &c->t_m, &c->t_v, &c->t_part, &c->t_grad,
                      &c->t_loss, &c->t_z, &c->tune_labels, &c->tune_hist,
                      &c->cp_rec[0], &c->cp_rec[1], &c->cp_rows, &c->cp_ovf, &c->cp_off, &c->cp_key, &c->cp_tal,
                      &c->cp_first, &c->cp_pieces, &c->cp_total, &c->cp_rows1, &c->cp_rows2, &c->cp_rows3,
                      &c->cp_distinct, &c->cp_sfirst, &c->cp_slices, &c->cp_rowstate, &c->cp_wsum};
    if (c->bexec) (void)hipGraphExecDestroy(c->bexec);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    for (DevBuf *b : bufs) b->release();
    if (c->pinned) (void)hipHostFree(c->pinned);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    if (c->round_a) (void)hipEventDestroy(c->round_a);
    if (c->round_b) (void)hipEventDestroy(c->round_b);
    if (c->prep_a) (void)hipEventDestroy(c->prep_a);
    if (c->prep_b) (void)hipEventDestroy(c->prep_b);
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
        case LPA_ETIMEDOUT: return "a grid-wide wait of the batched kernel timed out";
        case LPA_ETOOLARGE: return "the input exceeds the fixed scratch of the allocation-free entry point";
    }
    return "unknown status";
}

}  // extern "C"
