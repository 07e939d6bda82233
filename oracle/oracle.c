/*
 * oracle.c -- plain, deliberately slow CPU reference for the RAK label
 * propagation method and the modularity measure.  Built without OpenMP
 * (liboracle.so) it is sequential; built with it (liboracle_omp.so) the
 * vertices of a round are shared among threads with the same arithmetic.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this code.  It shares nothing with
 * the GPU library: no headers, no helpers, no tables.
 *
 * What is computed (Sahu, "Selecting a suitable Parallel Label-propagation
 * based algorithm for Disjoint Community Detection", arXiv 2301.09125):
 *
 *  - RAK / LPA, weighted form (Section 3.2; Section 2 for the method): every
 *    vertex starts with a unique label; in each iteration every vertex takes
 *    the label whose incident edge weight is largest.  Readings taken where
 *    the paper leaves the detail open:
 *      * synchronous rounds: round t reads only the labels of round t-1;
 *      * "strict" tie-break (pick the first of the tied labels) made
 *        order-free as: the lowest label value among the tied ones;
 *      * the paper adds a self-loop to every vertex (Section 3.1.2); the CSR
 *        holds none and a self_weight is added to the vertex's own label
 *        (self_weight = 1 mirrors the paper, 0 gives the open neighbourhood);
 *      * a vertex with nothing to vote on keeps its label;
 *      * convergence (Section 3.2 and Section 4): the tolerance is the largest
 *        fraction of vertices allowed to change; stop after round t when
 *        changed_t <= floor(tol * n), n counting every vertex;
 *      * an iteration cap max_iter; hitting it is reported, not an error.
 *  - Modularity (Newman-Girvan, Section 1): with 2m = sum of all arc weights,
 *    Sigma_in = weight of arcs whose endpoints share a label and
 *    K_c = sum of weighted degrees in community c,
 *    Q = Sigma_in / 2m - sum_c K_c^2 / (2m)^2, evaluated on the CSR as given.
 *    All sums are exact integers; only the final expression is FP64.
 *
 * The vote is the textbook definition: gather (label, weight) pairs of the
 * closed neighbourhood, sort them by label, add up equal labels, keep the
 * heaviest (lowest label on ties).
 *
 * Two further forms (orc_rak_ext):
 *  - non-strict tie-break (Section 3.2: a random one of the tied labels),
 *    made reproducible: every label gets the priority lowbias32(label ^ k),
 *    k drawn per (seed, round t, vertex v) from SplitMix64, and the tied
 *    label of highest priority wins.  lowbias32 is a bijection of 32-bit
 *    words, so distinct labels never share a priority;
 *  - semi-synchronous rounds, a deterministic stand-in for the paper's
 *    in-place OpenMP updates and COPRA's asynchronous order (Sections 3.2,
 *    3.3): each round is two half-rounds; half h votes the vertices of half
 *    h (the top bit of a SplitMix64 draw per vertex and round, or a given
 *    split kept for every round) reading the labels left by the half before,
 *    the other vertices keep theirs.  A vertex votes once per round, so
 *    changed_t still counts the vertices whose label differs from round t-1.
 *    The split is drawn again every round: two neighbours that are each
 *    other's heaviest neighbour swap labels while they share a half, and a
 *    fixed split would keep such pairs swapping forever.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct { uint32_t label; uint32_t weight; } pair_lw;

static int by_label(const void *a, const void *b) {
    uint32_t x = ((const pair_lw *)a)->label, y = ((const pair_lw *)b)->label;
    return (x > y) - (x < y);
}

/* Validation shared by every entry: returns 0 or -1 (bad CSR) / -2 (a
 * vertex's weighted degree plus self weight does not fit 32 bits). */
static int check_csr(uint32_t n, const uint64_t *rp, const uint32_t *col, const uint32_t *w,
                     uint32_t self_weight) {
    if (!rp) return -1;
    if (rp[0] != 0) return -1;
    for (uint32_t v = 0; v < n; ++v) {
        if (rp[v + 1] < rp[v]) return -1;
        uint64_t tot = self_weight;
        for (uint64_t e = rp[v]; e < rp[v + 1]; ++e) {
            if (col[e] >= n) return -1;
            tot += w ? w[e] : 1u;
        }
        if (tot > 0xFFFFFFFFull) return -2;
    }
    return 0;
}

/* SplitMix64 (G. Steele, D. Lea, C. Flood, "Fast splittable pseudorandom
 * number generators", OOPSLA 2014): output number c + 1 (c >= 0) of the
 * generator started from state `seed`, i.e. the mix of seed + (c+1)*gamma. */
uint64_t orc_splitmix64_at(uint64_t seed, uint64_t c) {
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * (c + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* lowbias32 (C. Wellons, "Prospecting for Hash Functions", 2018): a
 * bijection of 32-bit words. */
uint32_t orc_lowbias32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

/* The draws of vertex v in round t >= 1 are SplitMix64 outputs number
 * 2c + 1 and 2c + 2 for c = t * 2^32 + v: the first decides the half of a
 * semi-synchronous round (its top bit), the second gives the tie key. */
int orc_half_of(uint64_t seed, uint32_t t, uint32_t v) {
    return (int)(orc_splitmix64_at(seed, ((((uint64_t)t << 32) | v) << 1)) >> 63);
}

/* Tie key k of vertex v in round t >= 1 (non-strict votes). */
uint32_t orc_tie_key(uint64_t seed, uint32_t t, uint32_t v) {
    return (uint32_t)orc_splitmix64_at(seed, ((((uint64_t)t << 32) | v) << 1) | 1u);
}

/* How a vote breaks ties: strict (the lowest tied label) or hashed (the
 * tied label of highest priority lowbias32(label ^ k)). */
typedef struct { int hashed; uint32_t k; } tie_rule;

/* The label vertex v takes from L_old.  buf must hold deg(v)+1 pairs.
 * When top1/top2 are given they receive the winning tally and the largest
 * tally of any other label (0 when there is none; both 0 for an empty
 * vote). */
static uint32_t vote_tie(uint32_t v, const uint64_t *rp, const uint32_t *col, const uint32_t *w,
                         uint32_t self_weight, const uint32_t *L_old, pair_lw *buf, uint64_t *top1,
                         uint64_t *top2, tie_rule tie) {
    uint64_t k = 0;
    if (self_weight > 0) {
        buf[k].label = L_old[v];
        buf[k].weight = self_weight;
        ++k;
    }
    for (uint64_t e = rp[v]; e < rp[v + 1]; ++e) {
        buf[k].label = L_old[col[e]];
        buf[k].weight = w ? w[e] : 1u;
        ++k;
    }
    if (top1) *top1 = 0;
    if (top2) *top2 = 0;
    if (k == 0) return L_old[v];
    qsort(buf, (size_t)k, sizeof(pair_lw), by_label);
    uint32_t best_label = 0;
    uint64_t best_weight = 0, second_weight = 0;
    int have = 0;
    uint64_t i = 0;
    while (i < k) {
        uint32_t lab = buf[i].label;
        uint64_t sum = 0;
        while (i < k && buf[i].label == lab) sum += buf[i++].weight;
        /* labels arrive in increasing order, so under the strict rule a
         * strictly larger sum is needed to displace the current best: ties
         * keep the lower label.  The hashed rule lets a tied label with a
         * higher priority take over. */
        int wins = !have || sum > best_weight;
        if (have && sum == best_weight && tie.hashed &&
            orc_lowbias32(lab ^ tie.k) > orc_lowbias32(best_label ^ tie.k))
            wins = 1;
        if (wins) {
            if (have) second_weight = best_weight;
            best_label = lab;
            best_weight = sum;
            have = 1;
        } else if (sum > second_weight) {
            second_weight = sum;
        }
    }
    if (top1) *top1 = best_weight;
    if (top2) *top2 = second_weight;
    return best_label;
}

static uint32_t vote(uint32_t v, const uint64_t *rp, const uint32_t *col, const uint32_t *w,
                     uint32_t self_weight, const uint32_t *L_old, pair_lw *buf, uint64_t *top1,
                     uint64_t *top2) {
    tie_rule strict = {0, 0};
    return vote_tie(v, rp, col, w, self_weight, L_old, buf, top1, top2, strict);
}

static uint64_t max_degree(uint32_t n, const uint64_t *rp) {
    uint64_t d = 0;
    for (uint32_t v = 0; v < n; ++v)
        if (rp[v + 1] - rp[v] > d) d = rp[v + 1] - rp[v];
    return d;
}

/* One synchronous round over the vertices with active[v] != 0 (all if
 * active == NULL); inactive vertices copy their label.  Returns the number
 * of vertices whose label changed, or a negative code.
 *
 * Built with OpenMP (liboracle_omp.so) the vertices are shared among the
 * threads, each with a vote buffer of its own -- the paper's OpenMP RAK gives
 * every thread a separately allocated hashtable (Section 3.2).  A round only
 * reads L_old and each vertex writes only its own L_new entry, so the result
 * does not depend on the number of threads. */
static int64_t round_tie(uint32_t n, const uint64_t *rp, const uint32_t *col, const uint32_t *w,
                         uint32_t self_weight, const uint32_t *L_old, uint32_t *L_new, const uint8_t *active,
                         int hashed, uint64_t seed, uint32_t t) {
    const size_t cap = (size_t)(max_degree(n, rp) + 1);
    int64_t changed = 0;
    int failed = 0;
#pragma omp parallel reduction(+ : changed) reduction(| : failed)
    {
        pair_lw *buf = (pair_lw *)malloc(cap * sizeof(pair_lw));
        if (!buf) {
            failed = 1;
        } else {
#pragma omp for schedule(dynamic, 1024)
            for (int64_t i = 0; i < (int64_t)n; ++i) {
                uint32_t v = (uint32_t)i;
                tie_rule tie = {hashed, hashed ? orc_tie_key(seed, t, v) : 0u};
                uint32_t lab = (active && !active[v])
                                   ? L_old[v]
                                   : vote_tie(v, rp, col, w, self_weight, L_old, buf, NULL, NULL, tie);
                L_new[v] = lab;
                changed += (lab != L_old[v]);
            }
            free(buf);
        }
    }
    return failed ? -3 : changed;
}

int64_t orc_rak_round(uint32_t n, const uint64_t *rp, const uint32_t *col, const uint32_t *w,
                      uint32_t self_weight, const uint32_t *L_old, uint32_t *L_new,
                      const uint8_t *active) {
    return round_tie(n, rp, col, w, self_weight, L_old, L_new, active, 0, 0, 0);
}

/* Threads a round of orc_rak_round may use (1 without OpenMP). */
int orc_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* One synchronous round over every vertex that also reports, per vertex,
 * the winning tally (top1) and the largest tally of any other label (top2),
 * both including the self weight on the vertex's own label.  Returns the
 * number of changed vertices or a negative code. */
int64_t orc_rak_round_top2(uint32_t n, const uint64_t *rp, const uint32_t *col, const uint32_t *w,
                           uint32_t self_weight, const uint32_t *L_old, uint32_t *L_new, uint64_t *top1,
                           uint64_t *top2) {
    if (!top1 || !top2) return -1;
    int rc = check_csr(n, rp, col, w, self_weight);
    if (rc) return rc;
    pair_lw *buf = (pair_lw *)malloc((size_t)(max_degree(n, rp) + 1) * sizeof(pair_lw));
    if (!buf) return -3;
    int64_t changed = 0;
    for (uint32_t v = 0; v < n; ++v) {
        uint32_t lab = vote(v, rp, col, w, self_weight, L_old, buf, &top1[v], &top2[v]);
        L_new[v] = lab;
        changed += (lab != L_old[v]);
    }
    free(buf);
    return changed;
}

/* Full RAK run.
 *   init_labels: NULL for the unique initial labels L0(v) = v, else the
 *                labels to resume from (copied, not modified);
 *   labels_out:  n labels after the last executed round;
 *   changed_per_iter: max_iter entries (may be NULL);
 *   iterations:  rounds executed; converged: 1 if the tolerance test passed.
 * Returns 0, -1 (invalid input), -2 (weight overflow), -3 (out of memory). */
int orc_rak(uint32_t n, const uint64_t *rp, const uint32_t *col, const uint32_t *w,
            uint32_t self_weight, double tol, uint32_t max_iter, const uint32_t *init_labels,
            uint32_t *labels_out, uint64_t *changed_per_iter, uint32_t *iterations,
            int32_t *converged) {
    if (!(tol >= 0.0 && tol <= 1.0) || !labels_out || !iterations || !converged) return -1;
    if (n > 0xFFFFFFFEu) return -1;
    int rc = check_csr(n, rp, col, w, self_weight);
    if (rc) return rc;
    if (init_labels)
        for (uint32_t v = 0; v < n; ++v)
            if (init_labels[v] >= n) return -1;
    const uint64_t thr = (uint64_t)floor(tol * (double)n);
    uint32_t *a = (uint32_t *)malloc((size_t)(n ? n : 1) * sizeof(uint32_t));
    uint32_t *b = (uint32_t *)malloc((size_t)(n ? n : 1) * sizeof(uint32_t));
    if (!a || !b) { free(a); free(b); return -3; }
    for (uint32_t v = 0; v < n; ++v) a[v] = init_labels ? init_labels[v] : v;
    *iterations = 0;
    *converged = 0;
    for (uint32_t t = 1; t <= max_iter; ++t) {
        int64_t ch = orc_rak_round(n, rp, col, w, self_weight, a, b, NULL);
        if (ch < 0) { free(a); free(b); return (int)ch; }
        uint32_t *s = a; a = b; b = s;
        if (changed_per_iter) changed_per_iter[t - 1] = (uint64_t)ch;
        *iterations = t;
        if ((uint64_t)ch <= thr) { *converged = 1; break; }
    }
    memcpy(labels_out, a, (size_t)n * sizeof(uint32_t));
    free(a);
    free(b);
    return 0;
}

/* RAK with a choice of update order and tie-break (see the header).
 *   order: 0 synchronous rounds, 1 semi-synchronous rounds;
 *   hashed: 0 strict (lowest tied label), 1 hashed priorities (non-strict);
 *   seed: draws of both; halves: NULL, or n entries in {0, 1}: a split used
 *   in every round instead of the drawn ones.
 * Other arguments and the return value as orc_rak. */
int orc_rak_ext(uint32_t n, const uint64_t *rp, const uint32_t *col, const uint32_t *w,
                uint32_t self_weight, double tol, uint32_t max_iter, const uint32_t *init_labels,
                int order, int hashed, uint64_t seed, const uint8_t *halves, uint32_t *labels_out,
                uint64_t *changed_per_iter, uint32_t *iterations, int32_t *converged) {
    if (!(tol >= 0.0 && tol <= 1.0) || !labels_out || !iterations || !converged) return -1;
    if (n > 0xFFFFFFFEu || order < 0 || order > 1) return -1;
    int rc = check_csr(n, rp, col, w, self_weight);
    if (rc) return rc;
    if (init_labels)
        for (uint32_t v = 0; v < n; ++v)
            if (init_labels[v] >= n) return -1;
    const uint64_t thr = (uint64_t)floor(tol * (double)n);
    uint32_t *a = (uint32_t *)malloc((size_t)(n ? n : 1) * sizeof(uint32_t));
    uint32_t *b = (uint32_t *)malloc((size_t)(n ? n : 1) * sizeof(uint32_t));
    uint8_t *m0 = (uint8_t *)malloc((size_t)(n ? n : 1));
    uint8_t *m1 = (uint8_t *)malloc((size_t)(n ? n : 1));
    if (!a || !b || !m0 || !m1) { free(a); free(b); free(m0); free(m1); return -3; }
    for (uint32_t v = 0; v < n; ++v) a[v] = init_labels ? init_labels[v] : v;
    *iterations = 0;
    *converged = 0;
    for (uint32_t t = 1; t <= max_iter; ++t) {
        int64_t ch;
        if (order == 1)
            for (uint32_t v = 0; v < n; ++v) {
                int h = halves ? (halves[v] != 0) : orc_half_of(seed, t, v);
                m0[v] = (uint8_t)(h == 0);
                m1[v] = (uint8_t)(h == 1);
            }
        if (order == 0) {
            ch = round_tie(n, rp, col, w, self_weight, a, b, NULL, hashed, seed, t);
            if (ch >= 0) { uint32_t *s = a; a = b; b = s; }
        } else {
            ch = round_tie(n, rp, col, w, self_weight, a, b, m0, hashed, seed, t);
            if (ch >= 0) {
                uint32_t *s = a; a = b; b = s;
                int64_t ch1 = round_tie(n, rp, col, w, self_weight, a, b, m1, hashed, seed, t);
                if (ch1 < 0) ch = ch1;
                else { s = a; a = b; b = s; ch += ch1; }
            }
        }
        if (ch < 0) { free(a); free(b); free(m0); free(m1); return (int)ch; }
        if (changed_per_iter) changed_per_iter[t - 1] = (uint64_t)ch;
        *iterations = t;
        if ((uint64_t)ch <= thr) { *converged = 1; break; }
    }
    memcpy(labels_out, a, (size_t)n * sizeof(uint32_t));
    free(a); free(b); free(m0); free(m1);
    return 0;
}

/* Rounds restricted to given vertex sets: round t votes only the vertices
 * with masks[(t-1)*n + v] != 0 and copies the others.  Used to replay a run
 * that skipped vertices.  changed_per_iter gets rounds entries. */
int orc_rak_masked(uint32_t n, const uint64_t *rp, const uint32_t *col, const uint32_t *w,
                   uint32_t self_weight, uint32_t rounds, const uint8_t *masks,
                   const uint32_t *init_labels, uint32_t *labels_out, uint64_t *changed_per_iter) {
    if (!labels_out || (rounds && !masks)) return -1;
    int rc = check_csr(n, rp, col, w, self_weight);
    if (rc) return rc;
    uint32_t *a = (uint32_t *)malloc((size_t)(n ? n : 1) * sizeof(uint32_t));
    uint32_t *b = (uint32_t *)malloc((size_t)(n ? n : 1) * sizeof(uint32_t));
    if (!a || !b) { free(a); free(b); return -3; }
    for (uint32_t v = 0; v < n; ++v) a[v] = init_labels ? init_labels[v] : v;
    for (uint32_t t = 0; t < rounds; ++t) {
        int64_t ch = orc_rak_round(n, rp, col, w, self_weight, a, b, masks + (size_t)t * n);
        if (ch < 0) { free(a); free(b); return (int)ch; }
        uint32_t *s = a; a = b; b = s;
        if (changed_per_iter) changed_per_iter[t] = (uint64_t)ch;
    }
    memcpy(labels_out, a, (size_t)n * sizeof(uint32_t));
    free(a);
    free(b);
    return 0;
}

/* Weighted Newman-Girvan modularity of `labels` on the CSR as stored.
 * Outputs the exact integer sums too: two_m = sum of arc weights,
 * sigma_in = weight of same-label arcs, sum_k2 = sum_c K_c^2 as two 64-bit
 * halves (lo, hi).  Q = 0 when two_m = 0.  Returns 0 or -1. */
int orc_modularity(uint32_t n, const uint64_t *rp, const uint32_t *col, const uint32_t *w,
                   const uint32_t *labels, double *q_out, uint64_t *two_m_out,
                   uint64_t *sigma_in_out, uint64_t *sum_k2_out) {
    if (!q_out || !labels) return -1;
    int rc = check_csr(n, rp, col, w, 0);
    if (rc) return rc;
    for (uint32_t v = 0; v < n; ++v)
        if (labels[v] >= n) return -1;
    uint64_t *K = (uint64_t *)calloc((size_t)(n ? n : 1), sizeof(uint64_t));
    if (!K) return -3;
    uint64_t two_m = 0, sigma_in = 0;
    for (uint32_t v = 0; v < n; ++v) {
        uint64_t k_v = 0;
        for (uint64_t e = rp[v]; e < rp[v + 1]; ++e) {
            uint64_t we = w ? w[e] : 1u;
            k_v += we;
            if (labels[col[e]] == labels[v]) sigma_in += we;
        }
        two_m += k_v;
        K[labels[v]] += k_v;
    }
    unsigned __int128 sk2 = 0;
    for (uint32_t c = 0; c < n; ++c) sk2 += (unsigned __int128)K[c] * K[c];
    free(K);
    double q = 0.0;
    if (two_m > 0) {
        double W = (double)two_m;
        q = (double)sigma_in / W - (double)sk2 / (W * W);
    }
    *q_out = q;
    if (two_m_out) *two_m_out = two_m;
    if (sigma_in_out) *sigma_in_out = sigma_in;
    if (sum_k2_out) {
        sum_k2_out[0] = (uint64_t)sk2;
        sum_k2_out[1] = (uint64_t)(sk2 >> 64);
    }
    return 0;
}

/* ------------------------------------------------------------------ COPRA --
 *
 * COPRA (Section 3.3): every vertex holds a set of (label, belonging
 * coefficient) pairs whose coefficients sum to 1; it starts as its own
 * community with belonging 1.  In each iteration a vertex collects the
 * labels of its neighbourhood (not its own), each neighbour's coefficients
 * scaled by the connecting edge weight; it keeps the labels whose share of
 * the collected weight reaches the threshold 1/max_labels; if none does, it
 * keeps only the best label; a vertex with nothing to collect joins its own
 * community; the kept labels are normalised to sum to 1.  Convergence is
 * counted as in RAK, on the vertices whose best label changed, and the
 * result is each vertex's best label.
 *
 * Readings taken here (the paper leaves them open):
 *   - synchronous rounds, as for RAK here, or, standing in for the paper's
 *     asynchronous COPRA, semi-synchronous rounds (two half-rounds over the
 *     halves orc_half_of draws, a vertex of the other half keeping its
 *     state), as orc_rak_ext;
 *   - coefficients are fixed point, integer multiples of 2^-16 (COPRA_ONE =
 *     2^16 stands for 1), so every sum is an exact integer: the collected
 *     tally of label c at v is sum over arcs (v,u,w) of w * b_u(c), and the
 *     total is weighted_degree(v) * 2^16;
 *   - a label is kept iff tally > 0 and tally * max_labels >= total
 *     (Gregory's original rule drops coefficients below 1/max_labels; a
 *     vertex whose arcs all weigh 0 collects nothing to share and keeps its
 *     best label alone);
 *   - the best label is the one of largest tally; ties go to the lowest
 *     label (strict, as RAK) or, for "a random best label" (the paper's
 *     wording), to the tied label of highest priority lowbias32(label ^ k),
 *     k = orc_tie_key(seed, t, v), as the non-strict RAK; if nothing reaches
 *     the threshold the best label is kept alone with coefficient 1;
 *   - normalisation: b(c) = floor(tally(c) * 2^16 / sum of kept tallies),
 *     and what the floors leave out of 2^16 goes to the best label, so the
 *     coefficients sum to exactly 2^16.
 * With max_labels = 1 a label is kept only when it is the only one, so the
 * vertex takes its best label: RAK with self weight 0. */

#define COPRA_ONE 65536u

typedef struct { uint32_t label; uint64_t tally; } pair_lt;

static int by_label_lt(const void *a, const void *b) {
    uint32_t x = ((const pair_lt *)a)->label, y = ((const pair_lt *)b)->label;
    return (x > y) - (x < y);
}

/* One round for vertex v: reads the state (lab, coef, cnt) of the previous
 * round (V slots per vertex), writes v's new state and returns its best
 * label.  buf holds deg(v) * V pairs. */
static uint32_t copra_vertex(uint32_t v, const uint64_t *rp, const uint32_t *col, const uint32_t *w, uint32_t V,
                             const uint32_t *lab, const uint32_t *coef, const uint32_t *cnt, pair_lt *buf,
                             uint32_t *nlab, uint32_t *ncoef, uint32_t *ncnt, tie_rule tie) {
    uint64_t k = 0, total = 0;
    for (uint64_t e = rp[v]; e < rp[v + 1]; ++e) {
        uint32_t u = col[e];
        uint64_t we = w ? w[e] : 1u;
        total += we * COPRA_ONE;
        for (uint32_t i = 0; i < cnt[u]; ++i) {
            buf[k].label = lab[(size_t)u * V + i];
            buf[k].tally = we * coef[(size_t)u * V + i];
            ++k;
        }
    }
    uint32_t *ol = nlab + (size_t)v * V, *oc = ncoef + (size_t)v * V;
    if (k == 0) {  /* nothing collected: its own community */
        ol[0] = v;
        oc[0] = COPRA_ONE;
        *ncnt = 1;
        return v;
    }
    qsort(buf, (size_t)k, sizeof(pair_lt), by_label_lt);
    /* sum runs of equal labels in place: buf[0..d) = distinct labels */
    uint64_t d = 0;
    for (uint64_t i = 0; i < k;) {
        uint32_t l = buf[i].label;
        uint64_t s = 0;
        while (i < k && buf[i].label == l) s += buf[i++].tally;
        buf[d].label = l;
        buf[d].tally = s;
        ++d;
    }
    uint64_t bi = 0;  /* labels ascend: a strictly larger tally is needed to win */
    for (uint64_t i = 1; i < d; ++i)
        if (buf[i].tally > buf[bi].tally ||
            (tie.hashed && buf[i].tally == buf[bi].tally &&
             orc_lowbias32(buf[i].label ^ tie.k) > orc_lowbias32(buf[bi].label ^ tie.k)))
            bi = i;
    uint64_t kept_sum = 0;
    uint32_t kept = 0;
    for (uint64_t i = 0; i < d; ++i)
        if (buf[i].tally > 0 && buf[i].tally * V >= total) {
            kept_sum += buf[i].tally;
            ++kept;
        }
    if (kept == 0) {
        ol[0] = buf[bi].label;
        oc[0] = COPRA_ONE;
        *ncnt = 1;
        return buf[bi].label;
    }
    uint32_t j = 0, given = 0, best_slot = 0;
    for (uint64_t i = 0; i < d; ++i)
        if (buf[i].tally > 0 && buf[i].tally * V >= total) {
            uint32_t c = (uint32_t)(buf[i].tally * COPRA_ONE / kept_sum);
            if (i == bi) best_slot = j;
            ol[j] = buf[i].label;
            oc[j] = c;
            given += c;
            ++j;
        }
    oc[best_slot] += COPRA_ONE - given;
    *ncnt = kept;
    return buf[bi].label;
}

/* COPRA run (see above).  max_labels in 1..64; order (0 synchronous, 1
 * semi-synchronous), hashed, seed: as orc_rak_ext.
 *   best_out:  n best labels after the last executed round;
 *   state_lab, state_coef (n * max_labels) and state_cnt (n): the final
 *              state, or NULL;
 *   changed_per_iter: max_iter entries (may be NULL): vertices whose best
 *              label changed in each round.
 * Returns 0, -1 (invalid input), -2 (weight overflow), -3 (out of memory). */
int orc_copra(uint32_t n, const uint64_t *rp, const uint32_t *col, const uint32_t *w, uint32_t max_labels,
              int order, int hashed, uint64_t seed, double tol, uint32_t max_iter, uint32_t *best_out,
              uint32_t *state_lab,
              uint32_t *state_coef, uint32_t *state_cnt, uint64_t *changed_per_iter, uint32_t *iterations,
              int32_t *converged) {
    if (!(tol >= 0.0 && tol <= 1.0) || !best_out || !iterations || !converged) return -1;
    if (n > 0xFFFFFFFEu || max_labels < 1 || max_labels > 64 || order < 0 || order > 1) return -1;
    int rc = check_csr(n, rp, col, w, 0);
    if (rc) return rc;
    const uint32_t V = max_labels;
    const size_t nv = (size_t)(n ? n : 1);
    const uint64_t thr = (uint64_t)floor(tol * (double)n);
    uint32_t *lab[2], *coef[2], *cnt[2], *best[2];
    int fail = 0;
    for (int s = 0; s < 2; ++s) {
        lab[s] = (uint32_t *)malloc(nv * V * sizeof(uint32_t));
        coef[s] = (uint32_t *)malloc(nv * V * sizeof(uint32_t));
        cnt[s] = (uint32_t *)malloc(nv * sizeof(uint32_t));
        best[s] = (uint32_t *)malloc(nv * sizeof(uint32_t));
        fail |= !lab[s] || !coef[s] || !cnt[s] || !best[s];
    }
    pair_lt *buf = (pair_lt *)malloc((size_t)(max_degree(n, rp) * V + 1) * sizeof(pair_lt));
    if (fail || !buf) {
        for (int s = 0; s < 2; ++s) { free(lab[s]); free(coef[s]); free(cnt[s]); free(best[s]); }
        free(buf);
        return -3;
    }
    for (uint32_t v = 0; v < n; ++v) {  /* every vertex its own community */
        lab[0][(size_t)v * V] = v;
        coef[0][(size_t)v * V] = COPRA_ONE;
        cnt[0][v] = 1;
        best[0][v] = v;
    }
    int cur = 0;
    *iterations = 0;
    *converged = 0;
    for (uint32_t t = 1; t <= max_iter; ++t) {
        uint64_t ch = 0;
        for (int h = 0; h <= order; ++h) {  /* one pass, or the two halves */
            const int nx = cur ^ 1;
            for (uint32_t v = 0; v < n; ++v) {
                if (order && orc_half_of(seed, t, v) != h) {  /* the other half keeps its state */
                    memcpy(lab[nx] + (size_t)v * V, lab[cur] + (size_t)v * V, V * sizeof(uint32_t));
                    memcpy(coef[nx] + (size_t)v * V, coef[cur] + (size_t)v * V, V * sizeof(uint32_t));
                    cnt[nx][v] = cnt[cur][v];
                    best[nx][v] = best[cur][v];
                    continue;
                }
                tie_rule tie = {hashed, hashed ? orc_tie_key(seed, t, v) : 0u};
                best[nx][v] = copra_vertex(v, rp, col, w, V, lab[cur], coef[cur], cnt[cur], buf, lab[nx], coef[nx],
                                           &cnt[nx][v], tie);
                ch += best[nx][v] != best[cur][v];
            }
            cur = nx;
        }
        if (changed_per_iter) changed_per_iter[t - 1] = ch;
        *iterations = t;
        if (ch <= thr) { *converged = 1; break; }
    }
    memcpy(best_out, best[cur], (size_t)n * sizeof(uint32_t));
    if (state_lab && state_coef && state_cnt) {
        memcpy(state_lab, lab[cur], (size_t)n * V * sizeof(uint32_t));
        memcpy(state_coef, coef[cur], (size_t)n * V * sizeof(uint32_t));
        memcpy(state_cnt, cnt[cur], (size_t)n * sizeof(uint32_t));
    }
    for (int s = 0; s < 2; ++s) { free(lab[s]); free(coef[s]); free(cnt[s]); free(best[s]); }
    free(buf);
    return 0;
}
