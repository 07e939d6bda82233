/*
 * graphgen.c -- seeded synthetic graph generators that feed both the CPU
 * oracle and the GPU library.  This module holds no label-propagation
 * arithmetic: it only draws random graphs and packs them as symmetric CSR.
 *
 * Output format (all generators): n vertices, m arcs, row_ptr u64[n+1],
 * col u32[m] sorted ascending inside each row, no self-loops, no duplicate
 * arcs, every undirected edge stored in both directions, optional u32
 * weights w[m] that are identical on both arcs of an edge.
 *
 * Randomness is counter based (the splitmix64 output function of Steele,
 * Lea and Flood, "Fast splittable pseudorandom number generators", 2014,
 * applied to key + (counter+1)*golden_gamma), so every draw is a pure
 * function of (seed, stream, counter).  Results therefore do not depend on
 * the number of OpenMP threads.
 *
 * Graph classes follow the shapes of the paper's dataset (Table 1): skewed
 * web/social graphs (R-MAT), near-planar road networks (damaged lattice with
 * diagonal shortcuts) and planted-partition graphs (SBM).  The paper adds a
 * self-loop to every vertex (Section 3.1.2); here the CSR holds none and the
 * library models that loop with its self_weight option instead.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define GG_VERSION 1u

typedef struct {
    uint32_t n;
    uint64_t m;
    uint64_t *row_ptr;
    uint32_t *col;
    uint32_t *w; /* NULL when the class is unweighted */
} gg_csr;

uint32_t gg_version(void) { return GG_VERSION; }

/* ------------------------------------------------------------------ RNG -- */

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static inline uint64_t gg_key(uint64_t seed, uint64_t stream) {
    return mix64(mix64(seed + 0x9E3779B97F4A7C15ull) ^ (stream * 0xD1B54A32D192ED03ull));
}
static inline uint64_t gg_draw(uint64_t key, uint64_t ctr) {
    return mix64(key + (ctr + 1) * 0x9E3779B97F4A7C15ull);
}
/* uniform double in [0,1) with 53 random bits */
static inline double u01(uint64_t h) { return (double)(h >> 11) * (1.0 / 9007199254740992.0); }

uint64_t gg_hash(uint64_t seed, uint64_t stream, uint64_t ctr) {
    return gg_draw(gg_key(seed, stream), ctr);
}

/* ------------------------------------------------- edge list -> CSR ----- */

/* An edge source produces undirected pairs (u,v) by index; it is called
 * twice (count pass, fill pass) and must be deterministic. */
typedef struct edge_src edge_src;
typedef int (*edge_fn)(const edge_src *s, uint64_t i, uint32_t *u, uint32_t *v);
struct edge_src {
    edge_fn fn;
    uint64_t count;
    uint32_t n;
    /* generator parameters */
    uint64_t key, key2, key3;
    uint32_t scale, rows, cols;
    double a, b, c, p, p2;
    const uint32_t *perm;
    const uint32_t *eu, *ev; /* explicit edge list */
};

static int cmp_u32(const void *x, const void *y) {
    uint32_t a = *(const uint32_t *)x, b = *(const uint32_t *)y;
    return (a > b) - (a < b);
}

/* Sort a row in place and drop duplicates; returns the new length. */
static uint64_t sort_unique(uint32_t *r, uint64_t len) {
    if (len < 2) return len;
    qsort(r, (size_t)len, sizeof(uint32_t), cmp_u32);
    uint64_t k = 1;
    for (uint64_t i = 1; i < len; ++i)
        if (r[i] != r[k - 1]) r[k++] = r[i];
    return k;
}

static int build_csr(const edge_src *s, gg_csr *out) {
    const uint32_t n = s->n;
    uint64_t *deg = (uint64_t *)calloc((size_t)n + 1, sizeof(uint64_t));
    if (!deg) return -3;
    /* pass 1: degrees with both directions, self-loops dropped */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)s->count; ++i) {
        uint32_t u, v;
        if (!s->fn(s, (uint64_t)i, &u, &v) || u == v) continue;
#pragma omp atomic
        deg[u]++;
#pragma omp atomic
        deg[v]++;
    }
    uint64_t *off = (uint64_t *)malloc(((size_t)n + 1) * sizeof(uint64_t));
    if (!off) { free(deg); return -3; }
    off[0] = 0;
    for (uint32_t v = 0; v < n; ++v) off[v + 1] = off[v] + deg[v];
    uint64_t tot = off[n];
    uint32_t *tmp = (uint32_t *)malloc((size_t)(tot ? tot : 1) * sizeof(uint32_t));
    if (!tmp) { free(deg); free(off); return -3; }
    memcpy(deg, off, (size_t)n * sizeof(uint64_t)); /* deg becomes cursor */
    /* pass 2: scatter (order inside a row is fixed by the sort below) */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)s->count; ++i) {
        uint32_t u, v;
        if (!s->fn(s, (uint64_t)i, &u, &v) || u == v) continue;
        uint64_t pu, pv;
#pragma omp atomic capture
        pu = deg[u]++;
#pragma omp atomic capture
        pv = deg[v]++;
        tmp[pu] = v;
        tmp[pv] = u;
    }
    /* pass 3: sort + dedup each row */
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t v = 0; v < (int64_t)n; ++v)
        deg[v] = sort_unique(tmp + off[v], off[v + 1] - off[v]);
    uint64_t *rp = (uint64_t *)malloc(((size_t)n + 1) * sizeof(uint64_t));
    if (!rp) { free(deg); free(off); free(tmp); return -3; }
    rp[0] = 0;
    for (uint32_t v = 0; v < n; ++v) rp[v + 1] = rp[v] + deg[v];
    uint64_t m = rp[n];
    uint32_t *col = (uint32_t *)malloc((size_t)(m ? m : 1) * sizeof(uint32_t));
    if (!col) { free(deg); free(off); free(tmp); free(rp); return -3; }
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t v = 0; v < (int64_t)n; ++v)
        memcpy(col + rp[v], tmp + off[v], (size_t)deg[v] * sizeof(uint32_t));
    free(tmp);
    free(off);
    free(deg);
    out->n = n;
    out->m = m;
    out->row_ptr = rp;
    out->col = col;
    out->w = NULL;
    return 0;
}

void gg_free(gg_csr *g) {
    if (!g) return;
    free(g->row_ptr);
    free(g->col);
    free(g->w);
    g->row_ptr = NULL;
    g->col = NULL;
    g->w = NULL;
}

/* Weight of the undirected edge {u,v}: uniform integer in [lo,hi], a pure
 * function of the unordered pair so both arcs agree. */
static int assign_weights(gg_csr *g, uint64_t seed, uint32_t lo, uint32_t hi) {
    g->w = (uint32_t *)malloc((size_t)(g->m ? g->m : 1) * sizeof(uint32_t));
    if (!g->w) return -3;
    uint64_t key = gg_key(seed, 0x77u);
    uint64_t span = (uint64_t)hi - lo + 1;
    uint64_t n = g->n;
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t v = 0; v < (int64_t)g->n; ++v) {
        for (uint64_t e = g->row_ptr[v]; e < g->row_ptr[v + 1]; ++e) {
            uint64_t u = g->col[e];
            uint64_t a = (uint64_t)v < u ? (uint64_t)v : u, b = (uint64_t)v < u ? u : (uint64_t)v;
            uint64_t h = gg_draw(key, a * n + b);
            g->w[e] = lo + (uint32_t)((h >> 32) % span);
        }
    }
    return 0;
}

/* -------------------------------------------------------------- R-MAT -- */

/* Sample i: `scale` quadrant choices with probabilities (a,b,c,1-a-b-c),
 * two choices per 64-bit draw (32 bits each), most significant bit first.
 * Then both endpoints go through the seeded permutation. */
static int rmat_edge(const edge_src *s, uint64_t i, uint32_t *u, uint32_t *v) {
    uint32_t src = 0, dst = 0;
    const double ab = s->a + s->b, abc = s->a + s->b + s->c;
    for (uint32_t l = 0; l < s->scale; l += 2) {
        uint64_t h = gg_draw(s->key, i * 32 + (l >> 1));
        for (uint32_t k = 0; k < 2 && l + k < s->scale; ++k) {
            double r = (double)(uint32_t)(k ? h : (h >> 32)) * (1.0 / 4294967296.0);
            uint32_t bs, bd;
            if (r < s->a) { bs = 0; bd = 0; }
            else if (r < ab) { bs = 0; bd = 1; }
            else if (r < abc) { bs = 1; bd = 0; }
            else { bs = 1; bd = 1; }
            src = (src << 1) | bs;
            dst = (dst << 1) | bd;
        }
    }
    if (s->perm) { src = s->perm[src]; dst = s->perm[dst]; }
    *u = src;
    *v = dst;
    return 1;
}

/* Seeded Fisher-Yates permutation of [0,n). */
static uint32_t *make_perm(uint32_t n, uint64_t seed) {
    uint32_t *p = (uint32_t *)malloc((size_t)(n ? n : 1) * sizeof(uint32_t));
    if (!p) return NULL;
    for (uint32_t i = 0; i < n; ++i) p[i] = i;
    uint64_t key = gg_key(seed, 0x5045524dull);
    for (uint32_t i = n; i > 1; --i) {
        uint64_t j = gg_draw(key, i) % i;
        uint32_t t = p[i - 1];
        p[i - 1] = p[j];
        p[j] = t;
    }
    return p;
}

int gg_rmat(uint32_t scale, uint32_t edge_factor, double a, double b, double c,
            uint64_t seed, int permute, gg_csr *out) {
    if (!out || scale < 1 || scale > 31 || a < 0 || b < 0 || c < 0 || a + b + c > 1.0) return -1;
    edge_src s;
    memset(&s, 0, sizeof s);
    s.fn = rmat_edge;
    s.n = 1u << scale;
    s.count = (uint64_t)edge_factor << scale;
    s.scale = scale;
    s.a = a; s.b = b; s.c = c;
    s.key = gg_key(seed, 0x524d4154ull);
    uint32_t *perm = NULL;
    if (permute) {
        perm = make_perm(s.n, seed);
        if (!perm) return -3;
        s.perm = perm;
    }
    int rc = build_csr(&s, out);
    free(perm);
    return rc;
}

/* --------------------------------------------------------------- road -- */

/* Edge index space: 2*v (right neighbour), 2*v+1 (down neighbour),
 * 2*n + v (diagonal shortcut of v).  Lattice edges are deleted with
 * probability p; each vertex not on the last row adds a diagonal to the
 * next row with probability p2, direction by a fair coin, reflected at the
 * left/right border. */
static int road_edge(const edge_src *s, uint64_t i, uint32_t *u, uint32_t *v) {
    const uint64_t n = (uint64_t)s->rows * s->cols;
    if (i < 2 * n) {
        uint64_t x = i >> 1;
        uint32_t r = (uint32_t)(x / s->cols), c = (uint32_t)(x % s->cols);
        if (i & 1) { if (r + 1 >= s->rows) return 0; }
        else { if (c + 1 >= s->cols) return 0; }
        if (u01(gg_draw(s->key, i)) < s->p) return 0;
        *u = (uint32_t)x;
        *v = (i & 1) ? (uint32_t)(x + s->cols) : (uint32_t)(x + 1);
        return 1;
    }
    uint64_t x = i - 2 * n;
    uint32_t r = (uint32_t)(x / s->cols), c = (uint32_t)(x % s->cols);
    if (r + 1 >= s->rows) return 0;
    uint64_t h = gg_draw(s->key2, x);
    if (u01(h) >= s->p2) return 0;
    int64_t cc = (int64_t)c + ((gg_draw(s->key3, x) & 1) ? 1 : -1);
    if (cc < 0) cc = c + 1;
    if (cc >= (int64_t)s->cols) cc = (int64_t)c - 1;
    if (cc < 0 || cc >= (int64_t)s->cols) return 0; /* single column */
    *u = (uint32_t)x;
    *v = (uint32_t)((uint64_t)(r + 1) * s->cols + (uint64_t)cc);
    return 1;
}

int gg_road(uint32_t rows, uint32_t cols, double p_delete, double p_diag,
            uint32_t wmin, uint32_t wmax, uint64_t seed, gg_csr *out) {
    if (!out || rows == 0 || cols == 0 || (uint64_t)rows * cols > 0xFFFFFFFEull || wmin > wmax) return -1;
    edge_src s;
    memset(&s, 0, sizeof s);
    s.fn = road_edge;
    s.rows = rows;
    s.cols = cols;
    s.n = rows * cols;
    s.count = 3ull * s.n;
    s.p = p_delete;
    s.p2 = p_diag;
    s.key = gg_key(seed, 0x4c415454ull);
    s.key2 = gg_key(seed, 0x44494147ull);
    s.key3 = gg_key(seed, 0x5349474eull);
    int rc = build_csr(&s, out);
    if (rc) return rc;
    if (wmax > 0) {
        rc = assign_weights(out, seed, wmin, wmax);
        if (rc) { gg_free(out); return rc; }
    }
    return 0;
}

/* ---------------------------------------------------------------- SBM -- */

/* Planted partition: k contiguous blocks of near-equal size (the first n%k
 * blocks get one extra vertex); each pair i<j is an edge independently with
 * probability p_in (same block) or p_out.  Pairs are sampled exactly with
 * geometric skipping (Batagelj and Brandes, Phys. Rev. E 71, 2005) so the
 * cost is O(n + edges).  Row i draws from stream (i, segment) so rows are
 * independent; the edge list is materialised once and then packed. */
typedef struct { uint32_t *u, *v; uint64_t len, cap; } evec;

static int evec_push(evec *e, uint32_t a, uint32_t b) {
    if (e->len == e->cap) {
        uint64_t nc = e->cap ? e->cap * 2 : 1024;
        uint32_t *nu = (uint32_t *)realloc(e->u, nc * sizeof(uint32_t));
        if (!nu) return -3;
        e->u = nu;
        uint32_t *nv = (uint32_t *)realloc(e->v, nc * sizeof(uint32_t));
        if (!nv) return -3;
        e->v = nv;
        e->cap = nc;
    }
    e->u[e->len] = a;
    e->v[e->len] = b;
    e->len++;
    return 0;
}

static inline uint32_t block_of(uint64_t i, uint32_t n, uint32_t k) {
    uint32_t q = n / k, r = n % k;
    uint64_t big = (uint64_t)r * (q + 1);
    if (i < big) return (uint32_t)(i / (q + 1));
    return r + (uint32_t)((i - big) / q);
}
static inline uint64_t block_end(uint32_t b, uint32_t n, uint32_t k) {
    uint32_t q = n / k, r = n % k;
    return (uint64_t)(b + 1) * q + (b + 1 < r ? b + 1 : r);
}

/* Append to e the sampled pairs (i,j), j in [lo,hi), each with prob p. */
static int sample_range(evec *e, uint32_t i, uint64_t lo, uint64_t hi, double p, uint64_t key) {
    if (p <= 0.0 || lo >= hi) return 0;
    uint64_t ctr = 0;
    if (p >= 1.0) {
        for (uint64_t j = lo; j < hi; ++j)
            if (evec_push(e, i, (uint32_t)j)) return -3;
        return 0;
    }
    const double lq = log1p(-p);
    uint64_t j = lo;
    for (;;) {
        double r = u01(gg_draw(key, ctr++));
        double skip = floor(log1p(-r) / lq); /* r in [0,1): log1p(-r) finite */
        if (skip >= (double)(hi - j)) break;
        j += (uint64_t)skip;
        if (evec_push(e, i, (uint32_t)j)) return -3;
        ++j;
        if (j >= hi) break;
    }
    return 0;
}

static int list_edge(const edge_src *s, uint64_t i, uint32_t *u, uint32_t *v) {
    *u = s->eu[i];
    *v = s->ev[i];
    return 1;
}

static int sbm_edges(uint32_t n, uint32_t k, double p_in, double p_out, uint64_t seed, evec *all) {
    int nt = 1;
#ifdef _OPENMP
    nt = omp_get_max_threads();
#endif
    evec *parts = (evec *)calloc((size_t)nt, sizeof(evec));
    if (!parts) return -3;
    int err = 0;
#pragma omp parallel num_threads(nt)
    {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
#pragma omp for schedule(static)
        for (int64_t i = 0; i < (int64_t)n; ++i) {
            uint32_t b = block_of((uint64_t)i, n, k);
            uint64_t be = block_end(b, n, k);
            int rc = sample_range(&parts[t], (uint32_t)i, (uint64_t)i + 1, be, p_in,
                                  gg_key(seed, 2 * (uint64_t)i));
            rc |= sample_range(&parts[t], (uint32_t)i, be, n, p_out, gg_key(seed, 2 * (uint64_t)i + 1));
            if (rc) {
#pragma omp atomic write
                err = rc;
            }
        }
    }
    /* threads own contiguous row ranges (static schedule), so concatenating
     * in thread order gives the row-major order independent of timing */
    uint64_t tot = 0;
    for (int t = 0; t < nt; ++t) tot += parts[t].len;
    all->u = (uint32_t *)malloc((size_t)(tot ? tot : 1) * sizeof(uint32_t));
    all->v = (uint32_t *)malloc((size_t)(tot ? tot : 1) * sizeof(uint32_t));
    all->len = all->cap = tot;
    if (!all->u || !all->v) err = -3;
    uint64_t o = 0;
    for (int t = 0; t < nt; ++t) {
        if (!err) {
            memcpy(all->u + o, parts[t].u, parts[t].len * sizeof(uint32_t));
            memcpy(all->v + o, parts[t].v, parts[t].len * sizeof(uint32_t));
        }
        o += parts[t].len;
        free(parts[t].u);
        free(parts[t].v);
    }
    free(parts);
    return err;
}

int gg_sbm(uint32_t n, uint32_t k, double p_in, double p_out, uint64_t seed, gg_csr *out) {
    if (!out || n == 0 || k == 0 || k > n || n > 0xFFFFFFFEu) return -1;
    evec e;
    memset(&e, 0, sizeof e);
    int rc = sbm_edges(n, k, p_in, p_out, seed, &e);
    if (rc) { free(e.u); free(e.v); return rc; }
    edge_src s;
    memset(&s, 0, sizeof s);
    s.fn = list_edge;
    s.n = n;
    s.count = e.len;
    s.eu = e.u;
    s.ev = e.v;
    rc = build_csr(&s, out);
    free(e.u);
    free(e.v);
    return rc;
}

/* Arbitrary undirected edge list -> symmetric deduplicated CSR, self-loops
 * dropped.  Used by tests to build small hand-made graphs. */
int gg_from_edges(uint32_t n, uint64_t ne, const uint32_t *eu, const uint32_t *ev, gg_csr *out) {
    if (!out || (ne && (!eu || !ev))) return -1;
    for (uint64_t i = 0; i < ne; ++i)
        if (eu[i] >= n || ev[i] >= n) return -1;
    edge_src s;
    memset(&s, 0, sizeof s);
    s.fn = list_edge;
    s.n = n;
    s.count = ne;
    s.eu = eu;
    s.ev = ev;
    return build_csr(&s, out);
}

/* Attach pair-hashed weights in [lo,hi] to an existing CSR (tests). */
int gg_weights(gg_csr *g, uint64_t seed, uint32_t lo, uint32_t hi) {
    if (!g || lo > hi) return -1;
    free(g->w);
    g->w = NULL;
    return assign_weights(g, seed, lo, hi);
}

/* ------------------------------------------------------- SBM batches -- */

/* A batch of G planted-partition graphs packed into one CSR (vertex ranges
 * gv[g]..gv[g+1], arcs stay inside their graph).  Graph g: n_g =
 * round(exp(U[ln n_min, ln n_max])), k_g uniform in [8, min(64, n_g/25)]
 * (at least 1), near-equal contiguous blocks of mean size s = n_g/k_g,
 * p_in = deg_in/(s-1) clamped to 0.5 and p_out = deg_out/(n_g - s), so the
 * expected intra- and inter-block degrees are deg_in and deg_out.  The
 * per-graph seed is derived from (seed, g).  blocks_out (optional, filled
 * when not NULL after the call) receives every vertex's planted block. */
int gg_sbm_batch(uint32_t G, uint32_t n_min, uint32_t n_max, double deg_in, double deg_out, uint64_t seed,
                 gg_csr *out, uint64_t *gv, uint32_t *kk) {
    if (!out || !gv || G == 0 || n_min < 50 || n_max < n_min) return -1;
    uint64_t key = gg_key(seed, 0x42415443ull);
    uint32_t *ng = (uint32_t *)malloc((size_t)G * sizeof(uint32_t));
    uint32_t *kg = (uint32_t *)malloc((size_t)G * sizeof(uint32_t));
    gg_csr *parts = (gg_csr *)calloc((size_t)G, sizeof(gg_csr));
    if (!ng || !kg || !parts) { free(ng); free(kg); free(parts); return -3; }
    const double l0 = log((double)n_min), l1 = log((double)n_max);
    uint64_t total_n = 0;
    for (uint32_t g = 0; g < G; ++g) {
        double r = u01(gg_draw(key, 2ull * g));
        uint32_t n = (uint32_t)llround(exp(l0 + (l1 - l0) * r));
        if (n < n_min) n = n_min;
        if (n > n_max) n = n_max;
        uint32_t kmax = n / 25;
        if (kmax > 64) kmax = 64;
        uint32_t kmin = 8 < kmax ? 8 : (kmax ? kmax : 1);
        if (kmax < kmin) kmax = kmin;
        uint32_t k = kmin + (uint32_t)(gg_draw(key, 2ull * g + 1) % (uint64_t)(kmax - kmin + 1));
        ng[g] = n;
        kg[g] = k;
        total_n += n;
    }
    if (total_n > 0xFFFFFFFEull) { free(ng); free(kg); free(parts); return -1; }
    int err = 0;
    /* each graph draws from its own streams; gg_sbm parallelises inside */
    for (uint32_t g = 0; g < G && !err; ++g) {
        const double n = ng[g], s = n / kg[g];
        double p_in = deg_in / (s - 1.0);
        if (p_in > 0.5) p_in = 0.5;
        double p_out = (n - s) > 0 ? deg_out / (n - s) : 0.0;
        if (p_out > 1.0) p_out = 1.0;
        int rc = gg_sbm(ng[g], kg[g], p_in, p_out, gg_draw(key, 0x100000000ull + g), &parts[g]);
        if (rc) err = rc;
    }
    if (!err) {
        uint64_t m = 0;
        gv[0] = 0;
        for (uint32_t g = 0; g < G; ++g) {
            gv[g + 1] = gv[g] + ng[g];
            m += parts[g].m;
        }
        uint64_t *rp = (uint64_t *)malloc(((size_t)total_n + 1) * sizeof(uint64_t));
        uint32_t *col = (uint32_t *)malloc((size_t)(m ? m : 1) * sizeof(uint32_t));
        if (!rp || !col) {
            free(rp);
            free(col);
            err = -3;
        } else {
            uint64_t ao = 0;
            for (uint32_t g = 0; g < G; ++g) {
                const uint64_t vo = gv[g];
                for (uint32_t v = 0; v < ng[g]; ++v) rp[vo + v] = ao + parts[g].row_ptr[v];
                for (uint64_t e = 0; e < parts[g].m; ++e) col[ao + e] = (uint32_t)(vo + parts[g].col[e]);
                ao += parts[g].m;
            }
            rp[total_n] = ao;
            out->n = (uint32_t)total_n;
            out->m = m;
            out->row_ptr = rp;
            out->col = col;
            out->w = NULL;
        }
    }
    if (kk && !err)
        for (uint32_t g = 0; g < G; ++g) kk[g] = kg[g];
    for (uint32_t g = 0; g < G; ++g) gg_free(&parts[g]);
    free(parts);
    free(ng);
    free(kg);
    return err;
}
