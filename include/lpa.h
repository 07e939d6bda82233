/*
 * lpa.h -- C ABI of the MI355X (gfx950) RAK label-propagation library.
 *
 * Method: Sahu, "Selecting a suitable Parallel Label-propagation based
 * algorithm for Disjoint Community Detection", arXiv 2301.09125.
 *   - RAK / LPA, weighted (Section 3.2): every vertex starts with a unique
 *     label and, each iteration, adopts the label with the largest total
 *     weight among its neighbours; stop once at most a `tolerance` fraction
 *     of the vertices changed label (Section 3.2, restated in Section 4).
 *   - Modularity (Section 1) as the quality measure.
 *
 * Semantics fixed by this library where the paper leaves them open:
 *   - rounds are synchronous (round t reads only round t-1's labels), so the
 *     result is a deterministic function of the inputs;
 *   - the strict tie-break ("the first" tied label) is the lowest label value;
 *   - the paper's per-vertex self-loop (Section 3.1.2) is `self_weight`, a
 *     weight added to the vertex's own current label (default 1; 0 = vote of
 *     the open neighbourhood).  The CSR itself must not need self-loops;
 *   - a vertex with nothing to vote on keeps its label;
 *   - the run stops after round t when changed_t <= floor(tol * n), n
 *     counting every vertex; `max_iter` caps the rounds.  Hitting the cap is
 *     not an error (`converged` = 0).
 *
 * Conventions for every entry point:
 *   - Graphs are CSR in DEVICE memory, owned by the caller and only read:
 *     row_ptr u64[n+1] (row_ptr[0] = 0, non-decreasing, row_ptr[n] = m),
 *     col u32[m] (values < n), w u32[m] or NULL for unit weights.  The graph
 *     must be symmetric (every arc stored in both directions, equal weights);
 *     symmetry is the caller's contract and is not checked.
 *   - Label buffers are DEVICE memory of n u32, owned by the caller.
 *   - Work is enqueued on the context's HIP stream; every call returns only
 *     once its results are final (it synchronises that stream).
 *   - Errors are negative lpa_status codes; nothing aborts or throws.  After
 *     an error the contents of output buffers are unspecified.
 *   - A context is not thread-safe: use one per host thread / stream.
 */
#ifndef LPA_H
#define LPA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LPA_OK = 0,
    LPA_EINVAL = -1,       /* bad argument or malformed CSR / labels */
    LPA_EOVERFLOW = -2,    /* a vertex's weighted degree + self_weight >= 2^32 */
    LPA_ENOMEM = -3,       /* device or host allocation failed */
    LPA_EDEVICE = -4,      /* a HIP runtime call failed */
    LPA_EUNSUPPORTED = -5, /* option or size this build does not handle */
    LPA_ETIMEDOUT = -6,    /* a grid-wide wait of the batched kernel exceeded
                              its limit (every block left the kernel) */
    LPA_ETOOLARGE = -7     /* the input exceeds the fixed scratch of
                              lpa_modularity_noalloc */
} lpa_status;

typedef struct lpa_ctx lpa_ctx;

/* Graph in device memory (see conventions above). */
typedef struct {
    uint32_t n;                /* vertices, n <= 2^32 - 2 */
    uint64_t m;                /* arcs (each undirected edge counts twice) */
    const uint64_t *row_ptr;   /* device, n + 1 */
    const uint32_t *col;       /* device, m; may be NULL only when m == 0 */
    const uint32_t *w;         /* device, m, or NULL = every weight is 1 */
} lpa_csr;

/* Degree bins: a vertex of degree d is voted by
 *   one lane                                        if 1 <= d <= thread_max,
 *   a 16-lane group with a 64-slot LDS hashtable    if d <= group_max,
 *   one wavefront with a 256-slot LDS hashtable     if d <= wave_max,
 *   one wavefront with a 1024-slot LDS hashtable    if d <= wide_max,
 *   one wavefront per 512-arc segment, the segments' tallies merged
 *   exactly per row                                 otherwise: each segment
 *   reports its 4 heaviest labels and a bound on the rest; a row whose
 *   leader provably wins is decided from the reports, any other row merges
 *   its segments' full tallies in a global hashtable slab.
 * (lpa_run; lpa_run_batch votes the rows of degree <= group_max one per lane,
 * their labels sorted in registers.)
 * Any valid thresholds give the same labels; they only change speed.
 * 0 selects the default. */
typedef struct {
    uint32_t self_weight;  /* weight of the vertex's own label (default 1) */
    uint32_t thread_max;   /* 1..8                    (default 8)   */
    uint32_t group_max;    /* thread_max..32          (default 32)  */
    uint32_t wave_max;     /* group_max..128          (default 128) */
    uint32_t wide_max;     /* wave_max..512           (default 512) */
    uint32_t merge_max;    /* 1..512 (default 512): rows of more segments than
                              this merge their segments' full tallies in a
                              global slab instead of top-K reports */
    uint32_t profile;      /* nonzero: time every kernel launch with HIP events */
    uint32_t modularity;   /* nonzero: lpa_run also reports the modularity of
                              its result in lpa_stats (same definition as
                              lpa_modularity).  After two or more rounds it is
                              built from the last round's own-label weight
                              sums plus the arcs of the vertices that changed
                              in that round, which equals the full definition
                              for the symmetric graphs this library requires */
    uint32_t frontier;     /* 0: lpa_run votes every vertex in every round;
                              1: from round 2 on it votes only the vertices
                              that can change -- those whose closed
                              neighbourhood changed in the previous round
                              (frontier-based propagation, Section 2).  A
                              vertex outside that set sees the tally of its
                              last vote again, so the labels, changed counts
                              and rounds are identical to mode 0. */
    uint32_t barrier_timeout_us; /* lpa_run_batch: the longest a block waits at
                                    a grid-wide barrier of the persistent
                                    kernel before the launch gives up with
                                    LPA_ETIMEDOUT (0 = the default, 10 s) */
    uint32_t order;        /* LPA_ORDER_SYNC (default): round t reads only
                              round t-1's labels.  LPA_ORDER_SEMISYNC: each
                              round is two half-rounds; a vertex's half is the
                              top bit of SplitMix64 output number 2c + 1 from
                              state `seed`, c = t * 2^32 + v, drawn again every
                              round; the first half's vertices vote, then the
                              second half's vertices vote reading the labels
                              the first left, and every vertex keeps its label
                              in the other half.  A deterministic stand-in for
                              the paper's in-place OpenMP updates and COPRA's
                              asynchronous order (Sections 3.2, 3.3); it
                              settles where synchronous rounds swap labels
                              back and forth (nearly bipartite graphs) */
    uint32_t tie;          /* LPA_TIE_LOWEST (default): the strict mode of
                              Section 3.2, "the first" tied label read as the
                              lowest label.  LPA_TIE_HASH: the non-strict mode
                              (a random tied label) made reproducible: label
                              x scores lowbias32(x ^ k), k = the low 32 bits
                              of SplitMix64 output number 2c + 2 (c as above),
                              and the tied label of highest score wins */
    uint64_t seed;         /* draws of order and tie (any value) */
    uint32_t reuse_csr;    /* nonzero: lpa_run and lpa_run_resume keep the
                              binned, relabelled copy of the CSR (steps a1-a2,
                              once per CSR) and reuse it when called again
                              with the same row_ptr, col, w, n, m and bin
                              thresholds; lpa_run_batch likewise, with the
                              same graph_vptr too.  The caller promises the
                              arrays were not written in between.  Any other
                              call that builds a copy (another graph or
                              batch, modularity, frontier runs, the
                              autotuner) replaces it.  Round 1 of lpa_run is
                              then voted by the round kernels instead of the
                              relabel pass. */
} lpa_options;

enum { LPA_ORDER_SYNC = 0, LPA_ORDER_SEMISYNC = 1 };
enum { LPA_TIE_LOWEST = 0, LPA_TIE_HASH = 1 };

/* Run statistics.  The arrays are optional and owned by the caller; when
 * given they receive min(iterations, cap) entries. */
typedef struct {
    uint32_t iterations;        /* rounds executed */
    int32_t converged;          /* 1 if changed_last <= floor(tol * n) */
    uint64_t changed_last;      /* vertices changed in the last round */
    uint64_t arcs_processed;    /* sum over rounds of the arcs voted */
    double ms_total;            /* host wall time of the call */
    double ms_rounds;           /* device time of the vote launches of every
                                   round (HIP events around each round's
                                   launches).  From the unique initial labels,
                                   round 1 of the rows that list each
                                   neighbour once is voted by the pass that
                                   builds the relabelled CSR: that share of
                                   round 1 is in ms_prepare, not here */
    double ms_prepare;          /* device time from the first to the last
                                   launch of the binning and relabel passes
                                   (including round 1's share above and the
                                   device's waits for the host between them) */
    double modularity;          /* with options.modularity: Q of the result */
    uint64_t mod_terms[4];      /* ... and its terms, as lpa_modularity's */
    uint64_t *changed_per_iter; /* host, cap entries, or NULL */
    float *ms_per_iter;         /* host, cap entries, or NULL: device time of
                                   each round's launches, as ms_rounds */
    uint32_t cap;
} lpa_stats;

/* Per-kernel device time collected when options.profile != 0. */
typedef struct {
    char name[32];
    uint64_t launches;
    double ms;          /* summed device time (HIP events around the launch) */
    uint64_t bytes;     /* summed algorithmic bytes of the launches */
    uint64_t arcs;      /* summed arcs the launches voted */
} lpa_kernel_prof;

/* Fill *opt with the defaults listed above. */
void lpa_default_options(lpa_options *opt);

/* Create a context on HIP device `device` that enqueues on `stream`
 * (a hipStream_t; NULL = the device's null stream).  opt may be NULL for the
 * defaults.  Invalid option values give LPA_EINVAL. */
lpa_status lpa_init(lpa_ctx **ctx, int device, void *stream, const lpa_options *opt);

/* RAK from the unique initial labels L0(v) = v (Section 3.2), in the
 * context's update order and tie-break (lpa_options.order, .tie); a context
 * with order or tie set and frontier = 1 gives LPA_EUNSUPPORTED (as do
 * lpa_run_batch, lpa_run_learned and lpa_trace on such a context).
 * labels_out: device u32[n], receives the labels after the last round.
 * tol in [0, 1]; max_iter = 0 returns the initial labels.
 * The run works on a relabelled device copy of the CSR (vertices grouped by
 * degree bin, high-degree vertices first) that the context allocates: about
 * 4 bytes per arc (8 with weights) plus 25 bytes per vertex, and between
 * 2^23 and 2^25 vertices about 0.15 bytes per arc of the rows of more than
 * wide_max arcs (where each slice of the vertex ids starts in them: those
 * rows are relabelled slice by slice).
 * Errors: LPA_EINVAL (null pointer, tol outside [0,1] or NaN, n too large,
 * malformed row_ptr, col value >= n), LPA_EOVERFLOW, LPA_ENOMEM,
 * LPA_EDEVICE. */
lpa_status lpa_run(lpa_ctx *ctx, const lpa_csr *g, uint32_t *labels_out, double tol,
                   uint32_t max_iter, lpa_stats *stats);

/* Same as lpa_run but starts from the labels already in labels_inout
 * (device u32[n], every value < n), e.g. to resume an interrupted run.
 * Running k rounds and resuming for the rest equals one uninterrupted run. */
lpa_status lpa_run_resume(lpa_ctx *ctx, const lpa_csr *g, uint32_t *labels_inout, double tol,
                          uint32_t max_iter, lpa_stats *stats);

/* Weighted Newman-Girvan modularity (Section 1) of `labels` (device u32[n],
 * values < n) on the CSR as stored:
 *   Q = Sigma_in / 2m - sum_c K_c^2 / (2m)^2,
 * 2m = sum of arc weights, Sigma_in = weight of arcs whose ends share a
 * label, K_c = summed weighted degree of community c; Q = 0 when 2m = 0.
 * The sums are exact integers; only that last expression is FP64.
 * q_out: host double.  terms: host u64[4] or NULL, receives
 * {2m, Sigma_in, low 64 bits of sum K_c^2, high 64 bits}. */
lpa_status lpa_modularity(lpa_ctx *ctx, const lpa_csr *g, const uint32_t *labels,
                          double *q_out, uint64_t *terms);

/* COPRA (Section 3.3): label propagation in which every vertex holds up to
 * max_labels (1..64) pairs (label, belonging coefficient), coefficients
 * summing to 1.  From every vertex alone with belonging 1, each round a
 * vertex collects its neighbours' pairs, each coefficient multiplied by the
 * connecting edge weight (its own pairs are not collected); it keeps the
 * labels whose collected weight is positive and at least 1/max_labels of
 * the total, or, if none is, its best label alone; and it normalises what
 * it kept.  The best label is the heaviest collected one, ties broken as
 * options.tie says (lowest label, or the hashed priority of non-strict
 * RAK); a vertex without arcs is its own community.  Rounds follow
 * options.order (synchronous, or the semi-synchronous halves of RAK, the
 * deterministic stand-in for the paper's asynchronous COPRA) and stop after
 * round t iff at most floor(tol * n) best labels changed in it, or after
 * max_iter rounds (the paper settles on tol = 0.01 for COPRA).
 * Coefficients are exact fixed point: integers in units of 2^-16 (65536 =
 * 1); a kept label gets floor(tally * 65536 / kept_sum) and the best label
 * also what the floors leave out of 65536.  options.self_weight does not
 * apply; options.frontier must be 0 (LPA_EUNSUPPORTED otherwise).
 * labels_out: device u32[n], the best label of every vertex (the disjoint
 * result).  state_labels / state_coefs: device u32[n * max_labels] or NULL:
 * vertex v's kept pairs in slots v * max_labels + i, i < state_count[v],
 * labels increasing (slots past state_count[v] are left as they were);
 * state_count: device u32[n] or NULL.  The CSR is read as stored (no
 * relabelled copy); the context holds two state records per vertex of
 * 2 + 2 * max_labels u32 words rounded up to a power of two up to 128 bytes
 * (64 bytes each for max_labels 4), and tables in device memory for rows
 * whose distinct labels outgrow the on-chip table (at most
 * 24 * deg * max_labels bytes for such a row).  stats: as lpa_run (changed
 * counts are best-label changes; arcs_processed = m per round; with
 * options.modularity the modularity of labels_out).  Errors: as lpa_run,
 * LPA_EINVAL also for max_labels outside 1..64. */
lpa_status lpa_run_copra(lpa_ctx *ctx, const lpa_csr *g, uint32_t max_labels, uint32_t *labels_out,
                         uint32_t *state_labels, uint32_t *state_coefs, uint32_t *state_count, double tol,
                         uint32_t max_iter, lpa_stats *stats);

/* lpa_modularity for callers that cannot allocate (code between HIP graph
 * captures, tight serving loops, harnesses that forbid hipMalloc): the same
 * result and terms as lpa_modularity, computed without any device, pinned
 * or host allocation.  Its scratch is one fixed device array of
 * LPA_NOALLOC_MAX_N + 2064 u64 words (about 32 MiB) per GPU, held until the
 * process ends, whose address lpa_init looks up.  The CSR is read as stored
 * (no relabelled copy); ctx supplies only the device and the stream.
 * Every call on a GPU shares that GPU's scratch: calls that overlap on one
 * GPU (other streams, other threads, other contexts) race and must be
 * serialised by the caller.  Returns when q_out and terms are final.
 * Errors: LPA_ETOOLARGE when n > LPA_NOALLOC_MAX_N; LPA_EINVAL for a null
 * pointer, a malformed row_ptr, a col value or a label >= n; LPA_EDEVICE. */
#define LPA_NOALLOC_MAX_N (1u << 22)
lpa_status lpa_modularity_noalloc(lpa_ctx *ctx, const lpa_csr *g, const uint32_t *labels,
                                  double *q_out, uint64_t *terms);

/* Batched-run statistics.  The per-graph arrays are optional host arrays
 * owned by the caller (NULL = not wanted). */
typedef struct {
    uint32_t graphs;            /* G */
    uint32_t rounds;            /* rounds of the launch = max_g iterations[g] */
    uint32_t converged_graphs;  /* graphs whose tolerance test passed */
    uint64_t arcs_processed;    /* sum over graphs of arcs x rounds voted */
    double ms_total;            /* host wall time of the call */
    double ms_device;           /* duration of the persistent kernel (device
                                   wall clock read at its start and end) */
    uint32_t *iterations;       /* [G] rounds executed per graph */
    int32_t *converged;         /* [G] 1 if changed_last[g] <= floor(tol * n_g) */
    uint64_t *changed_last;     /* [G] changed count of the graph's last round */
    uint64_t *changed_hist;     /* [G * hist_cap]: row g holds the changed count
                                   of rounds 1..min(iterations[g], hist_cap),
                                   zeros after */
    uint32_t hist_cap;
} lpa_batch_stats;

/* RAK (Section 3.2) on G independent graphs packed in one CSR: graph g owns
 * vertices graph_vptr[g] .. graph_vptr[g+1]-1, and its arcs must stay among
 * them.  Every graph runs exactly as lpa_run would run it alone: labels
 * start as its local vertex ids, its tolerance test is
 * changed_g <= floor(tol * n_g) and it stops voting on its own once that test
 * passes or after max_iter rounds, while the others go on.  All rounds of
 * all graphs run in one persistent kernel launch (blocks kept co-resident,
 * grid-wide barriers between rounds); that launch and its set-up are
 * captured once in a HIP graph per context and layout, then replayed.
 * graph_vptr: host u64[G+1], graph_vptr[0] = 0, non-decreasing,
 *   graph_vptr[G] = packed->n (empty graphs are allowed).
 * labels_out: device u32[n]; vertex v of graph g receives its final label
 *   as a local id (global label - graph_vptr[g]).
 * Errors: those of lpa_run, LPA_EINVAL also for a malformed graph_vptr,
 * an arc leaving its graph or packed->n above 2^32 - 32, and LPA_ETIMEDOUT. */
lpa_status lpa_run_batch(lpa_ctx *ctx, const lpa_csr *packed, const uint64_t *graph_vptr, uint32_t G,
                         uint32_t *labels_out, double tol, uint32_t max_iter, lpa_batch_stats *stats);

/* ---- Learned frontier -------------------------------------------------
 *
 * Not part of the paper: a small network predicts, for every vertex that
 * may change in a round (see lpa_options.frontier), whether it will; only the
 * predicted changers are voted, the others keep their label for that round.
 * Features of vertex v before round t, from the state after round t-1
 * (top1 / top2 = winning and runner-up tally of v's most recent vote, both
 * including the self weight; k = weighted degree; sw = self weight):
 *   f1 = log2(1 + deg v)         f2 = (top1 - top2) / (k + sw)
 *   f3 = 1 if v changed in t-1   f4 = top1 / (k + sw)
 *   f5 = 1 if v or a neighbour changed in t-1 (1 when not tracked)
 *   f6 = t / max_iter
 * Network: h1 = relu(x W1 + b1); h2 = relu(bf16(h1) W2 + b2);
 * z = h2 . w3 + b3, with x, W1, W2 and w3 rounded to bfloat16 and FP32
 * accumulation; v is voted iff sigmoid(z) >= tau. */
typedef struct {
    float w1[6][32];
    float b1[32];
    float w2[32][32];
    float b2[32];
    float w3[32];
    float b3;
    float tau;  /* decision threshold in [0, 1]; 0 votes every candidate */
} lpa_mlp;

typedef struct {
    uint32_t iterations;        /* rounds executed */
    int32_t converged;          /* 1 if the run ended by a passed full check */
    uint32_t learned_rounds;    /* rounds in which the network chose */
    uint32_t check_round;       /* first round that voted every candidate
                                   after the learned rounds (0: none) */
    uint64_t changed_last;
    uint64_t arcs_processed;    /* arcs of the rows actually voted */
    double ms_total;
    double ms_rounds;
    double modularity;          /* with options.modularity: Q of the result */
    uint64_t mod_terms[4];      /* ... and its terms, as lpa_modularity's */
    uint64_t *changed_per_iter;    /* host, cap entries, or NULL */
    uint64_t *voted_per_iter;      /* rows voted per round, or NULL */
    uint64_t *candidates_per_iter; /* rows that could change per round, or NULL */
    uint32_t cap;
} lpa_learned_stats;

/* RAK with the learned frontier.  Round 1 votes every vertex.  The network
 * is consulted for a round only when the round before recorded top-two
 * tallies and changed fewer than half of the non-isolated vertices (tallies
 * are recorded after a round that changed fewer than half); other rounds
 * vote every vertex and end the run when they pass the tolerance test.  A
 * consulted round votes the candidates the network keeps (and every vertex
 * skipped in the round before); once its changed count plus the predicted
 * changes of the rows it skipped is at most floor(tol * n), or the network
 * kept at least 4/5 of the candidates, the next round votes every candidate
 * (a full check, equivalent to voting every vertex).  If the check passes the
 * run has converged; otherwise rounds go on voting every candidate (plain
 * RAK) until the tolerance test passes or max_iter rounds have run.  Rows
 * longer than wide_max arcs are voted in every round.
 * model: host.  masks: device u8[mask_rounds * n] or NULL; row t-1 receives
 * 1 for every vertex voted in round t (by original id), for replaying the
 * run.  The result approximates lpa_run's; with tau = 0 it is identical.
 * Errors: those of lpa_run, LPA_EINVAL for tau outside [0, 1]. */
lpa_status lpa_run_learned(lpa_ctx *ctx, const lpa_csr *g, const lpa_mlp *model, uint32_t *labels_out,
                           double tol, uint32_t max_iter, lpa_learned_stats *stats, uint8_t *masks,
                           uint32_t mask_rounds);

/* Training samples from a plain run (every vertex voted every round, exact
 * f5): for every round t >= 2 and every row of at most wide_max arcs with
 * at least one arc, the features before round t (6 floats, unrounded) and
 * y = 1 if the row changed in round t.  X: device float[cap * 6], y: device
 * u8[cap]; *count receives the number of samples (also when above cap, in
 * which case only cap were written).  The run stops as lpa_run does. */
lpa_status lpa_trace(lpa_ctx *ctx, const lpa_csr *g, double tol, uint32_t max_iter, float *X, uint8_t *y,
                     uint64_t cap, uint64_t *count);

typedef struct {
    uint32_t epochs;       /* passes over the samples */
    uint32_t batch;        /* samples per Adam step, a multiple of 256 */
    float lr;              /* Adam step size (beta1 0.9, beta2 0.999, eps 1e-8) */
    float pos_weight;      /* weight of the positive class in the loss */
    uint64_t seed;         /* sample order of each epoch */
    const float *val_X;    /* device validation samples, or NULL */
    const uint8_t *val_y;
    uint64_t val_n;
    float recall;          /* with validation samples: tau is set to the
                              largest value that keeps at least this
                              fraction of the positive validation samples */
} lpa_train_options;

/* Train model (host, in: initial weights, out: trained weights) on device
 * samples X (float[N * 6]) and y (u8[N]) with the weighted binary
 * cross-entropy of the logit, mean over each batch.  loss_per_epoch: host
 * float[epochs] (mean training loss of each epoch) or NULL. */
lpa_status lpa_train(lpa_ctx *ctx, const float *X, const uint8_t *y, uint64_t N, const lpa_train_options *opt,
                     lpa_mlp *model, float *loss_per_epoch);

/* Logits of N samples (device X float[N * 6] -> device z float[N]) with the
 * inference arithmetic used by lpa_run_learned. */
lpa_status lpa_mlp_forward(lpa_ctx *ctx, const lpa_mlp *model, const float *X, uint64_t N, float *z);

/* Loss and gradient (host float[1313], in the lpa_mlp field order w1, b1,
 * w2, b2, w3, b3) of the training loss over all N samples, as lpa_train
 * computes them for one batch (N <= 2^31). */
lpa_status lpa_mlp_grad(lpa_ctx *ctx, const lpa_mlp *model, const float *X, const uint8_t *y, uint64_t N,
                        float pos_weight, float *grad, float *loss);

/* Autotuner of the degree bins: times `rounds` rounds (0 = 2) of lpa_run --
 * or of lpa_run_batch when graph_vptr is given -- under every combination of
 * thread_max {4, 8}, group_max {16, 32}, wave_max {64, 128} and wide_max
 * {256, 512}, and makes the fastest the context's thresholds.  The choice is
 * cached in the context under the graph's degree signature (share of rows
 * and of arcs per power-of-two row length, in 1/32 steps, with the orders of
 * magnitude of n and m); a graph with a cached signature is not timed again.
 * chosen: host, receives the context's options afterwards (may be NULL);
 * measured: host, the number of candidates timed (0 on a cache hit; may be
 * NULL).  Labels never depend on the thresholds, only the speed does. */
lpa_status lpa_autotune(lpa_ctx *ctx, const lpa_csr *g, const uint64_t *graph_vptr, uint32_t G, uint32_t rounds,
                        lpa_options *chosen, uint32_t *measured);

/* Copy up to `cap` per-kernel profile records into out (host); *count gets
 * the number of records available.  lpa_profile_reset clears them. */
lpa_status lpa_profile_get(lpa_ctx *ctx, lpa_kernel_prof *out, uint32_t cap, uint32_t *count);
lpa_status lpa_profile_reset(lpa_ctx *ctx);

/* Release every device and host resource of the context (NULL is a no-op). */
void lpa_destroy(lpa_ctx *ctx);

/* Static description of a status code. */
const char *lpa_strerror(lpa_status s);

#ifdef __cplusplus
}
#endif

#endif /* LPA_H */
