"""The host C code (the oracle, oracle/oracle.c, and the graph generator,
graphgen/graphgen.c) built with gcc's AddressSanitizer and
UndefinedBehaviorSanitizer into one standalone driver, which generates small
graphs of every class and runs every oracle entry point on them (both update
orders and tie rules, the masked and top-2 rounds, modularity, COPRA at 1, 4
and 64 labels) plus their error paths.  Any out-of-bounds access, leak or
undefined operation ends the driver with a nonzero status.  CPU only: no GPU
code is involved."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r"""
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct { uint32_t n; uint64_t m; uint64_t *row_ptr; uint32_t *col; uint32_t *w; } gg_csr;
int gg_rmat(uint32_t, uint32_t, double, double, double, uint64_t, int, gg_csr *);
int gg_road(uint32_t, uint32_t, double, double, uint32_t, uint32_t, uint64_t, gg_csr *);
int gg_sbm(uint32_t, uint32_t, double, double, uint64_t, gg_csr *);
int gg_from_edges(uint32_t, uint64_t, const uint32_t *, const uint32_t *, gg_csr *);
int gg_weights(gg_csr *, uint64_t, uint32_t, uint32_t);
int gg_sbm_batch(uint32_t, uint32_t, uint32_t, double, double, uint64_t, gg_csr *, uint64_t *, uint32_t *);
void gg_free(gg_csr *);

int orc_rak(uint32_t, const uint64_t *, const uint32_t *, const uint32_t *, uint32_t, double, uint32_t,
            const uint32_t *, uint32_t *, uint64_t *, uint32_t *, int32_t *);
int orc_rak_ext(uint32_t, const uint64_t *, const uint32_t *, const uint32_t *, uint32_t, double, uint32_t,
                const uint32_t *, int, int, uint64_t, const uint8_t *, uint32_t *, uint64_t *, uint32_t *,
                int32_t *);
int64_t orc_rak_round_top2(uint32_t, const uint64_t *, const uint32_t *, const uint32_t *, uint32_t,
                           const uint32_t *, uint32_t *, uint64_t *, uint64_t *);
int orc_rak_masked(uint32_t, const uint64_t *, const uint32_t *, const uint32_t *, uint32_t, uint32_t,
                   const uint8_t *, const uint32_t *, uint32_t *, uint64_t *);
int orc_modularity(uint32_t, const uint64_t *, const uint32_t *, const uint32_t *, const uint32_t *, double *,
                   uint64_t *, uint64_t *, uint64_t *);
int orc_copra(uint32_t, const uint64_t *, const uint32_t *, const uint32_t *, uint32_t, int, int, uint64_t,
              double, uint32_t, uint32_t *, uint32_t *, uint32_t *, uint32_t *, uint64_t *, uint32_t *, int32_t *);

#define CHECK(x) do { if (!(x)) { fprintf(stderr, "check failed line %d: %s\n", __LINE__, #x); exit(2); } } while (0)

static void run_all(const gg_csr *g, uint32_t sw) {
    const uint32_t n = g->n;
    uint32_t *lab = malloc((n ? n : 1) * sizeof(uint32_t)), *lab2 = malloc((n ? n : 1) * sizeof(uint32_t));
    uint64_t ch[20], sigma[4];
    uint32_t it;
    int32_t conv;
    double q;
    CHECK(orc_rak(n, g->row_ptr, g->col, g->w, sw, 0.05, 20, NULL, lab, ch, &it, &conv) == 0);
    CHECK(orc_modularity(n, g->row_ptr, g->col, g->w, lab, &q, &sigma[0], &sigma[1], &sigma[2]) == 0);
    for (int order = 0; order < 2; ++order)
        for (int hashed = 0; hashed < 2; ++hashed)
            CHECK(orc_rak_ext(n, g->row_ptr, g->col, g->w, sw, 0.0, 6, lab, order, hashed, 7u + order,
                              NULL, lab2, ch, &it, &conv) == 0);
    uint64_t *t1 = malloc((n ? n : 1) * sizeof(uint64_t)), *t2 = malloc((n ? n : 1) * sizeof(uint64_t));
    CHECK(orc_rak_round_top2(n, g->row_ptr, g->col, g->w, sw, lab, lab2, t1, t2) >= 0);
    uint8_t *masks = malloc(2 * (size_t)(n ? n : 1));
    for (uint32_t v = 0; v < 2 * n; ++v) masks[v] = (uint8_t)((v * 2654435761u) >> 31);
    CHECK(orc_rak_masked(n, g->row_ptr, g->col, g->w, sw, 2, masks, NULL, lab2, ch) == 0);
    if (sw == 0) {
        const uint32_t Vs[3] = {1, 4, 64};
        for (int k = 0; k < 3; ++k) {
            const uint32_t V = Vs[k];
            uint32_t *sl = malloc((size_t)(n ? n : 1) * V * sizeof(uint32_t));
            uint32_t *sc = malloc((size_t)(n ? n : 1) * V * sizeof(uint32_t));
            uint32_t *sn = malloc((n ? n : 1) * sizeof(uint32_t));
            CHECK(orc_copra(n, g->row_ptr, g->col, g->w, V, k & 1, k == 2, 3u, 0.01, 8, lab2, sl, sc, sn, ch,
                            &it, &conv) == 0);
            free(sl); free(sc); free(sn);
        }
    }
    free(lab); free(lab2); free(t1); free(t2); free(masks);
}

static void error_paths(const gg_csr *g) {
    const uint32_t n = g->n;
    uint32_t *lab = malloc(n * sizeof(uint32_t));
    uint32_t it;
    int32_t conv;
    uint32_t *bad = malloc(g->m * sizeof(uint32_t));
    memcpy(bad, g->col, g->m * sizeof(uint32_t));
    bad[g->m / 2] = n;  /* a column id out of range */
    CHECK(orc_rak(n, g->row_ptr, bad, g->w, 0, 0.05, 5, NULL, lab, NULL, &it, &conv) == -1);
    CHECK(orc_rak(n, g->row_ptr, g->col, g->w, 0, 1.5, 5, NULL, lab, NULL, &it, &conv) == -1);
    CHECK(orc_rak(n, g->row_ptr, g->col, g->w, 0xFFFFFFFFu, 0.05, 5, NULL, lab, NULL, &it, &conv) == -2);
    uint32_t *init = malloc(n * sizeof(uint32_t));
    for (uint32_t v = 0; v < n; ++v) init[v] = v;
    init[n - 1] = n;  /* an initial label out of range */
    CHECK(orc_rak(n, g->row_ptr, g->col, g->w, 0, 0.05, 5, init, lab, NULL, &it, &conv) == -1);
    double q;
    CHECK(orc_modularity(n, g->row_ptr, g->col, g->w, init, &q, NULL, NULL, NULL) == -1);
    CHECK(orc_copra(n, g->row_ptr, g->col, g->w, 65, 0, 0, 1, 0.01, 5, lab, NULL, NULL, NULL, NULL, &it,
                    &conv) == -1);
    free(lab); free(bad); free(init);
}

int main(void) {
    gg_csr g;
    CHECK(gg_rmat(9, 8, 0.57, 0.19, 0.19, 3, 1, &g) == 0);
    run_all(&g, 0);
    run_all(&g, 2);
    error_paths(&g);
    CHECK(gg_weights(&g, 5, 0, 4) == 0);  /* zero weights included */
    run_all(&g, 1);
    gg_free(&g);
    CHECK(gg_road(16, 16, 0.3, 0.05, 1, 8, 4, &g) == 0);
    run_all(&g, 0);
    gg_free(&g);
    CHECK(gg_sbm(400, 8, 0.1, 0.005, 2, &g) == 0);
    run_all(&g, 0);
    gg_free(&g);
    uint32_t eu[300], ev[300];
    for (uint32_t i = 0; i < 300; ++i) { eu[i] = 0; ev[i] = i + 1; }  /* a star */
    CHECK(gg_from_edges(301, 300, eu, ev, &g) == 0);
    run_all(&g, 0);
    gg_free(&g);
    CHECK(gg_from_edges(5, 0, eu, ev, &g) == 0);  /* no edges at all */
    run_all(&g, 0);
    gg_free(&g);
    uint64_t gv[9];
    uint32_t kk[8];
    CHECK(gg_sbm_batch(8, 50, 400, 8.0, 1.0, 6, &g, gv, kk) == 0);
    run_all(&g, 0);
    gg_free(&g);
    printf("ok\n");
    return 0;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no gcc")
def test_host_c_under_asan_ubsan(tmp_path):
    src = tmp_path / "driver.c"
    exe = tmp_path / "driver"
    src.write_text(DRIVER)
    cmd = ["gcc", "-std=gnu11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", str(src), os.path.join(ROOT, "oracle", "oracle.c"),
           os.path.join(ROOT, "graphgen", "graphgen.c"), "-lm", "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600, env=env)
    if "LeakSanitizer has encountered a fatal error" in out.stderr:  # no ptrace here: leaks unchecked
        env["ASAN_OPTIONS"] = "detect_leaks=0"
        out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600, env=env)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout[-2000:] + out.stderr[-4000:]
