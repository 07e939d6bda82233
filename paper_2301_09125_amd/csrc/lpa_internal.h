// lpa_internal.h -- private declarations shared by the runtime (lpa_runtime.hip)
// and the kernel sources of the label-propagation library.
//
// Internal layout.  A run works on a relabelled copy of the caller's CSR:
// the vertices are renumbered bin by bin -- long rows first, then wavefront
// rows, 16-lane rows, one-lane rows and last the vertices without arcs, each
// bin in increasing original id.  Every bin is a contiguous range of internal
// ids, so
// kernels walk ranges instead of index lists, and the labels of the
// high-degree vertices, which most arcs point at, share a few hundred KB at
// the front of the label array where the L2 cache keeps them.  Label VALUES
// stay original vertex ids, so the lowest-label tie-break is unchanged.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

typedef struct lpa_ctx lpa_ctx;

namespace lpa {

// Error bits raised by kernels into a device word.
enum : uint32_t {
    ERR_COL = 1u,     // a col value >= n
    ERR_WOVF = 2u,    // weighted degree + self weight >= 2^32
    ERR_ROWPTR = 4u,  // row_ptr not monotone / not ending at m
    ERR_LABEL = 8u,   // a label value >= n
    ERR_TIMEOUT = 16u,  // a grid barrier of the batch kernel waited too long
    ERR_GRAPH = 32u,  // a batch arc leaves its graph
    ERR_TABLE = 64u,  // a COPRA hashtable had no free slot (a size bound was broken)
};

// Degree bins in internal layout order (see lpa_options in lpa.h).
enum { BIN_HUB = 0, BIN_WIDE = 1, BIN_WAVE = 2, BIN_GROUP = 3, BIN_THREAD = 4, BIN_ZERO = 5, NBINS = 6 };

constexpr int kThreadMaxCap = 8;     // register-array size of the one-lane vote
constexpr int kGroupLanes = 16;
constexpr int kGroupSlots = 64;      // LDS slots per 16-lane group (degree <= 32)
constexpr int kWaveArcsSmall = 128;  // wavefront rows with a small table
constexpr int kWaveSlotsSmall = 256;
constexpr int kWaveArcs = 512;       // arcs per wavefront work item
constexpr int kWaveSlots = 1024;     // LDS slots per wavefront (<= 512 arcs)
// LDS slots of a long-row segment's table.  A segment with more than
// kHubSpill distinct labels would hand its row to the exact slab merge; with
// 1024 slots and at most 512 arcs per segment that cannot happen, and a
// smaller table (more wavefronts per CU) lost more to probing and to rows
// sent to the slab than it won.
constexpr int kHubSlots = 1024;
constexpr uint32_t kHubSpill = 900;
static_assert(kHubSpill + 64 < (uint32_t)kHubSlots, "a capped table must never fill up");
constexpr uint32_t kNone = 0xFFFFFFFFu;
// Long rows relabelled by slices of the caller's id space (lpa_prep.hip).
constexpr uint32_t kSliceShift = 20;     // 2^20 ids (4 MB of the id map) per slice
constexpr uint32_t kSliceMin = 8;        // below 8 slices (32 MB) the direct gather is as fast
constexpr uint32_t kSliceMax = 32;       // beyond, a 512-arc segment holds too few arcs per slice
constexpr uint16_t kSliceNone = 0xFFFF;  // bnd[0] of a segment that is not sorted
constexpr int kDegBuckets = 24;  // row-length histogram of the autotuner

// Long rows: each 512-arc segment reports its kTopK heaviest labels and a
// bound on every label it did not report; rows of at most kMergeWaveSegs
// segments are merged by one wavefront, rows of at most kMergeBlockSegs by
// one block, longer rows always merge through the global slab.
constexpr int kTopK = 4;
constexpr int kMergeWaveSegs = 32;
constexpr int kMergeBlockSegs = 512;
constexpr int kMergeBlockSlots = 2 * kMergeBlockSegs * kTopK;

// The changed count of one round is spread over kCountSlots u64 words
// kCountStride words apart (one cache line each) so that blocks do not
// serialise on a single address; the host adds them up.
constexpr int kCountSlots = 32;
constexpr int kCountStride = 16;
constexpr int kCountWords = kCountSlots * kCountStride;

// Per-row flags of the internal graph.
enum : uint8_t { ROW_DISTINCT = 1 };  // the caller's row lists each neighbour once
// Per-hub flags: HUB_OWN_SEEN and HUB_FALLBACK live for one round,
// HUB_REPEATS and HUB_BIG for the run.
enum : uint32_t { HUB_OWN_SEEN = 1u, HUB_REPEATS = 2u, HUB_FALLBACK = 4u, HUB_BIG = 8u };

struct Graph {
    const uint64_t *rp;
    const uint32_t *col;
    const uint32_t *w;  // nullptr = unit weights
    uint32_t n;
    uint64_t m;
};

// Arguments common to every vote kernel of one round (internal graph).
struct RoundArgs {
    Graph g;
    const uint32_t *L_old;
    uint32_t *L_new;
    const uint8_t *rowflag;       // ROW_DISTINCT per internal row
    uint32_t sw;                  // self weight
    uint32_t check;               // nonzero: verify weighted degrees fit 32 bits
    unsigned long long *changed;  // this round's kCountWords counter words
    uint32_t *err;                // error bits
    const uint32_t *list;         // rows of the launch: list[0..min(cnt, *list_n)) (NULL: lo .. lo+cnt-1)
    const uint32_t *list_n;       // device count of list entries
    uint32_t *top1, *top2;        // vote kernels with FEAT: winning / runner-up tally per row
    uint32_t skip_distinct;       // round 1: rows flagged ROW_DISTINCT were voted by the relabel pass
    // non-NULL: kCountWords counter words that receive the sum over the
    // voted rows of the weight of arcs whose neighbour holds the row's own
    // label (Sigma_in of L_old when every row is voted)
    unsigned long long *insum;
    // Update order and tie-break (see row_mode in lpa_vote_dev.h):
    // half 0: every row votes; 1 / 2: only the rows whose draw for round t
    // puts them in the first / second half vote, the others copy their label
    // from L_old to L_new.  tie 0: strict (lowest label); 1: hashed.  The
    // draws use seed, t and the row's original id orig[row] (NULL when
    // half = tie = 0).
    uint32_t half;
    uint32_t tie;
    uint32_t t;
    unsigned long long seed;
    const uint32_t *orig;
};

// A wavefront work item of a long row: internal row r (= hub index), arcs
// [b0, b1) of the internal CSR, at most kWaveArcs of them.
struct HubItem {
    uint32_t r;
    uint32_t pad;
    uint64_t b0;
    uint64_t b1;
};

// State of the long rows (internal ids 0..H-1; arrays of H entries).
struct HubState {
    const uint64_t *slab_off;     // offset of the row's slab (u64 slots)
    const uint32_t *slab_mask;    // slab size - 1 (power of two >= 2 * degree)
    const uint64_t *touched_off;  // offset of the row's touched-slot list (capacity = degree)
    unsigned long long *slab;     // global hashtable slots, EMPTY between rounds
    uint32_t *touched;            // slot indices claimed this round (kNone = no claim)
    uint32_t *tcount;             // touched-list entries this round (reset by hub_final)
    unsigned long long *best;     // max (weight << 32 | ~label) (reset by hub_final)
    unsigned long long *own_sum;  // weight of neighbours holding the row's own label
    uint32_t *flags;              // HUB_* flags
    unsigned long long *rowsum;   // weighted degree (checked in round 1)
    unsigned long long *cand;     // kTopK (label << 32 | tally) per segment, EMPTY if unused
    uint32_t *thr;                // per segment: tally bound of its unreported labels
    const uint32_t *item_lo;      // H + 1: first segment of each row
    uint32_t *pending;            // nonzero: some row uses the slab this round
    uint32_t *repeats;            // relabel pass: rows flagged HUB_REPEATS (0: round 1 needs no table)
};

// Phase-2 item: touched-list positions [t0, t1) of hub `hub`.
struct ReduceItem {
    uint32_t hub;
    uint32_t t0;
    uint32_t t1;
    uint32_t pad;
};

// Degree thresholds of the bins (see lpa_options).
struct BinCfg {
    uint32_t tmax, gmax, wmax, xmax;
};

// Ranges of internal ids per bin.
struct Bins {
    uint32_t lo[NBINS];
    uint32_t cnt[NBINS];
    uint64_t arcs[NBINS];
};

struct ModArgs {
    Graph g;                   // internal graph
    const uint32_t *labels;    // internal labels (values are original ids < n_orig)
    unsigned long long *K;     // n_orig, summed weighted degree per community
    unsigned long long *sums;  // [0] = 2m, [1] = Sigma_in (incremental: the change of Sigma_in, mod 2^64)
    uint32_t *err;
    // incremental form: the labels of the round before the last one.  Only
    // rows whose label changed in the last round read their arcs' labels
    // (see launch_mod_rows).
    const uint32_t *labels_prev;
};

// Batched run: state of the persistent kernel (lpa_batch.hip).  The bins
// BIN_HUB .. BIN_THREAD vote; rows of graph g in bin k are the segment
// seg_lo[k*G+g] .. + seg_cnt[k*G+g] of internal ids.
constexpr int kBatchBins = 5;
constexpr int kBatchMaxBlocks = 512;  // blocks of one batched launch (one decision slice each)
constexpr int kBatchBarWords = 32 * 17;  // the batched launch's barrier: 16 group counters 128 bytes apart

struct BatchArgs {
    Graph g;                     // internal packed graph
    uint32_t *L0, *L1;           // label buffers; round t reads L0 if t is odd
    const uint32_t *gid;         // internal vertex -> graph
    const uint64_t *gv;          // graph g owns original ids gv[g] .. gv[g+1]-1
    const uint64_t *orp;         // caller's row_ptr (arcs per graph)
    uint32_t sw;
    uint32_t lo[NBINS], cnt[NBINS];
    uint32_t G, max_iter;
    const unsigned long long *thr;  // [G] floor(tol * n_g)
    uint32_t *active;            // [G] 1 while the graph votes
    uint32_t *iters;             // [G] rounds executed
    int32_t *conv;               // [G] tolerance met
    unsigned long long *changed; // [G] changed count of the current round
    unsigned long long *last;    // [G] changed count of the graph's last round
    unsigned long long *hist;    // [G * hist_len] changed counts of rounds 1..hist_len
    uint32_t hist_len;
    unsigned long long *arcs;    // arcs voted, summed over graphs
    unsigned long long *clock;   // [2] wall clock at the kernel's start and end (block 0)
    uint32_t *n_active;          // [2] graphs still voting after round t: word t & 1
    uint32_t *bar;               // [kBatchBarWords]: [0] group arrivals, [1] generation, then the groups' arrival counters
    uint32_t *err;
    const uint64_t *slab_off;    // long rows: per-row global slab ...
    const uint32_t *slab_mask;
    const uint64_t *touched_off;
    unsigned long long *slab;
    uint32_t *touched;
    uint32_t *tcount;
    const uint32_t *seg_lo;      // [kBatchBins * G]
    const uint32_t *seg_cnt;     // [kBatchBins * G]
    uint32_t *pref;              // [kBatchBins * (G+1)] units of voting graphs, prefix sums inside each slice
    uint32_t *btot;              // [kBatchBins * kBatchMaxBlocks] units of voting graphs per slice
    uint32_t dshift;             // block k decides graphs [k << dshift, (k + 1) << dshift)
    uint64_t timeout_ticks;      // wall-clock ticks one barrier may wait
};

// Learned frontier (lpa_learned.hip).  A model in the lane layouts of the
// 32x32x8 bfloat16 MFMA: a1[l] = W1[4*(l/32)+c][l%32] for c = 0..3 (rows 6
// and 7 zero), a2[s][l] = W2[8s+4*(l/32)+c][l%32], four bfloat16 per u64.
struct MlpDev {
    uint64_t a1[64];
    uint64_t a2[4][64];
    float b1[32], b2[32];
    float w3[32];  // rounded to bfloat16
    float b3;
    float zcut;    // keep a candidate iff its logit >= zcut
};

struct FrontArgs {
    Graph g;
    const uint32_t *L_old;
    uint32_t *L_new;
    const uint32_t *top1, *top2;  // tallies of each vertex's last vote
    const uint32_t *kw;           // weighted degree (NULL: unit weights)
    uint32_t *lastchg;            // last round the vertex changed (0: never)
    uint32_t *front;              // == t: the vertex or a neighbour changed in round t-1
    uint8_t *stale;               // skipped since its last vote
    uint8_t *mask;                // round's vote mask by original id, or NULL
    const uint32_t *old_of;
    unsigned long long *cand_count;  // += candidates of the round
    unsigned long long *kept_arcs;   // += arcs of the rows kept for the vote
    unsigned long long *exp_skip;    // += 1024 x predicted change probability of skipped rows
    uint32_t sw, t, max_iter;
    uint32_t all_dirty;  // every vertex counts as having a changed neighbour
    uint32_t keep_all;   // vote every candidate (no prediction)
};

// Round 1 from the unique labels computed by the relabel pass (rows that
// list each neighbour once); see RelabelArgs in lpa_prep.hip.
struct Round1Fuse {
    uint32_t *L1;                 // round-1 label buffer (internal index)
    unsigned long long *changed;  // round-1 counter words
    uint32_t sw;
    // rows of at most wide_max arcs the pass could not vote (a neighbour
    // listed twice or out of order), per bin b: rest_list[lo[b] ..
    // lo[b] + rest_n[b]) (internal rows); round 1 votes just these
    uint32_t *rest_list;
    uint32_t *rest_n;
};

// ---- launchers: lpa_prep.hip ---------------------------------------------
hipError_t launch_fill_u32_iota(uint32_t *a, uint32_t n, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long *p, unsigned long long v, uint64_t count, hipStream_t s);
hipError_t launch_degree_hist(const uint64_t *rp, uint32_t n, unsigned long long *hist, hipStream_t s);
hipError_t launch_hub_plan(const uint64_t *rp2, uint32_t H, uint32_t merge_max, unsigned long long *blk,
                           unsigned long long *out, hipStream_t s);
hipError_t launch_hub_fill(const uint64_t *rp2, uint32_t H, uint32_t merge_max, const unsigned long long *blk,
                           const unsigned long long *out, uint32_t *item_lo, uint64_t *slab_off,
                           uint64_t *touched_off, HubItem *items, ReduceItem *ritems, uint32_t *hflags,
                           uint32_t *slab_mask, uint32_t *mrows, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, uint64_t count, hipStream_t s);
hipError_t launch_check_labels(const uint32_t *labels, uint32_t n, uint32_t *err, hipStream_t s);
uint32_t bin_blocks(uint32_t n);
hipError_t launch_bin_count(const Graph &g, const BinCfg &cfg, uint32_t *blk_counts, unsigned long long *blk_arcs,
                            uint32_t nblk, uint32_t *err, hipStream_t s);
hipError_t launch_bin_scan(uint32_t *blk_counts, unsigned long long *blk_arcs, uint32_t nblk, uint32_t *totals,
                           unsigned long long *arc_totals, hipStream_t s);
hipError_t launch_bin_scatter(const Graph &g, const BinCfg &cfg, const uint32_t *blk_offsets,
                              const unsigned long long *blk_arc_offsets, const uint32_t *totals,
                              const unsigned long long *arc_totals, uint32_t nblk, uint32_t *old_of,
                              uint32_t *new_of, uint64_t *rp2, hipStream_t s);
// Copy the caller's rows into the internal CSR (ids through new_of) and
// flag rows that list each neighbour once.
// Rows [lo, lo + cnt) are bin bin_a below `split` and bin_b from it on.
hipError_t launch_relabel_rows(const Graph &g, const uint32_t *old_of, const uint32_t *new_of, const uint64_t *rp2,
                               uint32_t *col2, uint32_t *w2, uint8_t *rowflag, uint32_t lo, uint32_t cnt,
                               uint32_t split, int bin_a, int bin_b, int per_wave, uint32_t *err,
                               const Round1Fuse *f, hipStream_t s);
// Long rows are relabelled slice by slice of the caller's id space when
// relabel_slices(n) > 0 (n large enough for the id map to outgrow L2): bnd
// then holds count * (S + 1) u16 and isrc count u64 of scratch.
uint32_t relabel_slices(uint32_t n);
hipError_t launch_relabel_hub(const Graph &g, const uint32_t *old_of, const uint32_t *new_of, const uint64_t *rp2,
                              uint32_t *col2, uint32_t *w2, const HubItem *items, uint32_t count,
                              uint32_t *hub_flags, uint32_t *err, const Round1Fuse *f, const HubState *hs,
                              uint32_t H, uint16_t *bnd, uint64_t *isrc, hipStream_t s);
hipError_t launch_init_labels(uint32_t *La, uint32_t *Lb, const uint32_t *old_of, const uint32_t *labels_in,
                              uint32_t n, hipStream_t s);
hipError_t launch_scatter_labels(uint32_t *labels_out, const uint32_t *old_of, const uint32_t *L, uint32_t n_int,
                                 hipStream_t s);

// ---- launchers: lpa_vote.hip ---------------------------------------------
// first = 1: round 1 from the unique initial labels L0(v) = v.  num_cu: the
// device's compute units; grid-stride kernels get whole rounds of the blocks
// that fit on them at once.
hipError_t launch_vote_thread(const RoundArgs &a, uint32_t lo, uint32_t cnt, int first, int feat, int num_cu,
                              hipStream_t s);
hipError_t launch_vote_group(const RoundArgs &a, uint32_t lo, uint32_t cnt, int first, int feat, int num_cu,
                             hipStream_t s);
hipError_t launch_vote_wave(const RoundArgs &a, uint32_t lo, uint32_t cnt, int wide, int first, int feat,
                            int num_cu, hipStream_t s);
hipError_t launch_vote_hub(const RoundArgs &a, const HubItem *items, uint32_t count, const HubState &hs,
                           int first, int fused, int num_cu, hipStream_t s);
// Merge the top-K reports of each listed row; undecided rows get HUB_FALLBACK.
hipError_t launch_hub_merge(const RoundArgs &a, const HubState &hs, const uint32_t *rows, uint32_t count,
                            int per_block, int first, hipStream_t s);
// Slab merge of the segments of HUB_FALLBACK rows.
hipError_t launch_hub_fallback(const RoundArgs &a, const HubItem *items, uint32_t count, const HubState &hs,
                               int num_cu, hipStream_t s);
hipError_t launch_hub_reduce(const RoundArgs &a, const HubState &hs, const ReduceItem *items, uint32_t count,
                             hipStream_t s);
// Winner of the rows decided by best[] (direct, slab) and per-round reset.
hipError_t launch_hub_final(const RoundArgs &a, const HubState &hs, uint32_t count, int first, hipStream_t s);

// ---- launchers: lpa_mod.hip ----------------------------------------------
hipError_t launch_mod_rows(const ModArgs &a, uint32_t lo, uint32_t cnt, int per_wave, hipStream_t s);
hipError_t launch_mod_hub(const ModArgs &a, const HubItem *items, uint32_t count, hipStream_t s);
hipError_t launch_batch_gid(const uint32_t *old_of, uint32_t n, const uint64_t *gv, uint32_t G, uint32_t *gid,
                            hipStream_t s);
hipError_t launch_batch_out(uint32_t *out, const uint32_t *old_of, const uint32_t *gid, const uint32_t *L0,
                            const uint32_t *L1, const uint32_t *iters, const uint64_t *gv, uint32_t n,
                            hipStream_t s);
hipError_t launch_batch_seg(const uint32_t *gid, const Bins &bins, uint32_t G, uint32_t *seg_lo, uint32_t *seg_cnt,
                            hipStream_t s);
hipError_t launch_batch(const BatchArgs &b, uint32_t nblocks, int slots, hipStream_t s);
int batch_slots(const Bins &bins);
int batch_blocks_per_cu(int slots);
int batch_waves_per_block();

hipError_t launch_predict(const FrontArgs &p, const MlpDev *model, uint32_t lo, uint32_t cnt, uint32_t *list,
                          uint32_t *list_count, int num_cu, hipStream_t s);
hipError_t launch_push(const FrontArgs &p, const Bins &B, int mark, hipStream_t s);
hipError_t launch_trace_x(const FrontArgs &p, uint32_t lo, uint32_t cnt, float *X, hipStream_t s);
hipError_t launch_trace_y(const uint32_t *L_old, const uint32_t *L_new, uint32_t lo, uint32_t cnt, uint8_t *y,
                          hipStream_t s);
hipError_t launch_mlp_forward(const MlpDev *model, const float *X, uint64_t N, float *z, hipStream_t s);
int mlp_params();
hipError_t launch_train_step(const float *X, const uint8_t *y, uint64_t N, uint64_t mul, uint64_t add,
                             uint64_t start, uint32_t bn, float *wm, float *m, float *v, float *part, float *grad,
                             float pos_weight, float lr, float c1, float c2, float *loss_acc, int update,
                             hipStream_t s);
hipError_t launch_row_sums(const Graph &g, uint32_t *kw, hipStream_t s);
hipError_t launch_mask_rows(uint8_t *mask, const uint32_t *old_of, uint32_t lo, uint32_t cnt, uint8_t val,
                            hipStream_t s);

// Modularity sums of a CSR as the caller stores it (any row length, row
// bounds and labels checked in the kernel), and the final u128 reduction of
// mod_sumsq_k's partials (lpa_mod.hip).
hipError_t launch_mod_any(const ModArgs &a, hipStream_t s);
hipError_t launch_mod_final(const unsigned long long *partials, uint32_t nparts, const unsigned long long *sums,
                            const uint32_t *err, unsigned long long *out, hipStream_t s);
// The whole modularity of `labels` on a CSR as the caller stores it: clears
// K[0..n) and sums[0..3) (two totals, then the error word that `err` points
// into), then fills out[0..5) = {sum K^2 low, high, 2m, Sigma_in, error bits}.
hipError_t launch_modularity_any(const Graph &g, const uint32_t *labels, unsigned long long *K,
                                 unsigned long long *sums, uint32_t *err, unsigned long long *partials,
                                 uint32_t nparts, unsigned long long *out, hipStream_t s);
// Fixed scratch of lpa_modularity_noalloc: look up its address on `device`
// (current) once; called by lpa_init (lpa_noalloc.hip).
hipError_t noalloc_attach(int device);
// The device and stream a context was made with (lpa_runtime.hip).
int ctx_device(const lpa_ctx *c);
hipStream_t ctx_stream(const lpa_ctx *c);
hipError_t launch_mod_sumsq(const unsigned long long *K, uint32_t n, unsigned long long *partials,
                            uint32_t nparts, hipStream_t s);

}  // namespace lpa
