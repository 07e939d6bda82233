"""Pins of the CPU oracle against facts the method fixes (not against itself).

RAK/LPA, weighted, synchronous, lowest-label tie-break (arXiv 2301.09125,
Section 3.2), self-loop weight of Section 3.1.2, tolerance rule of Sections 3.2
and 4; modularity of Section 1; NMI named in Section 2.
"""
import itertools
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------ brute force --

def dense(g):
    """Adjacency indicator E and weight matrix A of a CSR (tiny graphs)."""
    n = g.n
    E = np.zeros((n, n), dtype=bool)
    A = np.zeros((n, n), dtype=np.int64)
    for v in range(n):
        for e in range(int(g.row_ptr[v]), int(g.row_ptr[v + 1])):
            u = int(g.col[e])
            E[v, u] = True
            A[v, u] += 1 if g.w is None else int(g.w[e])
    return E, A


def brute_round(E, A, L, sw):
    """Definition-level vote: for every vertex try every label value 0..n-1,
    tally the weight of closed-neighbourhood members holding it, keep the
    heaviest label present (lowest on ties), or the old label if none."""
    n = len(L)
    new = []
    for v in range(n):
        best, best_w = None, -1
        for lab in range(n):
            present = sw > 0 and L[v] == lab
            tally = sw if (sw > 0 and L[v] == lab) else 0
            for u in range(n):
                if E[v, u] and L[u] == lab:
                    present = True
                    tally += A[v, u]
            if present and tally > best_w:
                best, best_w = lab, tally
        new.append(L[v] if best is None else best)
    return new


def brute_run(E, A, sw, tol, max_iter):
    n = E.shape[0]
    L = list(range(n))
    thr = math.floor(tol * n)
    changed = []
    for _ in range(max_iter):
        N = brute_round(E, A, L, sw)
        ch = sum(1 for a, b in zip(L, N) if a != b)
        changed.append(ch)
        L = N
        if ch <= thr:
            return L, changed, True
    return L, changed, False


def brute_modularity(E, A, L):
    """(1/2m) sum_ij (A_ij - k_i k_j / 2m) delta(c_i, c_j) as an exact fraction."""
    n = len(L)
    two_m = int(A.sum())
    if two_m == 0:
        return Fraction(0)
    k = A.sum(axis=1)
    s = Fraction(0)
    for i in range(n):
        for j in range(n):
            if L[i] == L[j]:
                s += Fraction(int(A[i, j])) - Fraction(int(k[i]) * int(k[j]), two_m)
    return s / two_m


def all_graphs(n):
    pairs = list(itertools.combinations(range(n), 2))
    for mask in range(1 << len(pairs)):
        yield [p for i, p in enumerate(pairs) if mask >> i & 1]


# --------------------------------------------------------------- golden ----

def test_golden_weighted6(gg, orc):
    fx = json.load(open(os.path.join(GOLDEN, "weighted6.json")))
    n = fx["n"]
    g = gg.from_edges(n, [(a, b) for a, b, _ in fx["edges"]])
    wmap = {}
    for a, b, w in fx["edges"]:
        wmap[(a, b)] = wmap[(b, a)] = w
    src = np.repeat(np.arange(n), np.diff(g.row_ptr).astype(np.int64))
    g.w = np.array([wmap[(int(s), int(d))] for s, d in zip(src, g.col)], dtype=np.uint32)
    sw = fx["self_weight"]
    L = np.arange(n, dtype=np.uint32)
    for expect in fx["rounds"]:
        L, _ = orc.rak_round(g, L, self_weight=sw)
        assert L.tolist() == expect
    for run in fx["runs"]:
        r = orc.rak(g, tol=run["tol"], max_iter=run["max_iter"], self_weight=sw)
        assert r.labels.tolist() == run["labels"]
        assert r.changed == run["changed"]
        assert r.converged == run["converged"]
        assert r.iterations == len(run["changed"])
    m = fx["modularity"]
    res = orc.modularity(g, np.array(m["labels"], dtype=np.uint32))
    assert (res.two_m, res.sigma_in, res.sum_k2) == (m["two_m"], m["sigma_in"], m["sum_k2"])
    assert res.q == pytest.approx(m["q_num"] / m["q_den"], abs=1e-15)


def test_golden_cliques(gg, orc):
    fx = json.load(open(os.path.join(GOLDEN, "cliques.json")))
    for c in fx["cases"]:
        k, s = c["k"], c["s"]
        edges = [(b * s + i, b * s + j) for b in range(k) for i in range(s) for j in range(i + 1, s)]
        g = gg.from_edges(k * s, edges)
        lab = np.repeat(np.arange(k, dtype=np.uint32) * s, s)
        assert orc.modularity(g, lab).q == pytest.approx(c["q_num"] / c["q_den"], abs=1e-14)
        r = orc.rak(g, tol=0.0, max_iter=10, self_weight=1)
        assert r.changed == c["changed_sw1"]
        assert r.converged
        assert np.array_equal(r.labels, lab)


# ----------------------------------------------------------- closed forms --

def test_clique_open_neighbourhood(gg, orc):
    # self_weight 0, K_s with s >= 3: round 1 every vertex moves (vertex 0 to
    # 1, the rest to 0), round 2 only vertex 0 moves back to 0, then stable.
    for s in (3, 4, 7):
        g = gg.from_edges(s, itertools.combinations(range(s), 2))
        r = orc.rak(g, tol=0.0, max_iter=10, self_weight=0)
        assert r.changed == [s, 1, 0]
        assert r.labels.tolist() == [0] * s


def test_k2_oscillates_and_k1_is_fixed(gg, orc):
    g = gg.from_edges(3, [(0, 1)])  # K2 plus an isolated vertex
    r = orc.rak(g, tol=0.0, max_iter=7, self_weight=0)
    assert r.changed == [2] * 7
    assert not r.converged and r.iterations == 7
    assert r.labels.tolist() == [1, 0, 2]  # odd number of swaps; vertex 2 keeps its label


def test_path_closed_form(gg, orc):
    # P_n, unit weights, self_weight 1: L_t(i) = max(0, i - t), changed_t = n - t
    for n in (2, 5, 17, 64):
        g = gg.from_edges(n, [(i, i + 1) for i in range(n - 1)])
        L = np.arange(n, dtype=np.uint32)
        for t in range(1, n + 2):
            L, ch = orc.rak_round(g, L, self_weight=1)
            assert L.tolist() == [max(0, i - t) for i in range(n)]
            assert ch == max(0, n - t)
        r = orc.rak(g, tol=0.0, max_iter=n + 5, self_weight=1)
        assert r.converged and r.iterations == n
        assert r.changed == [n - t for t in range(1, n + 1)]


def test_star(gg, orc):
    s = 9
    g = gg.from_edges(s + 1, [(0, i) for i in range(1, s + 1)])
    r = orc.rak(g, tol=0.0, max_iter=6, self_weight=0)
    assert r.changed == [s + 1] * 6 and not r.converged
    r = orc.rak(g, tol=0.0, max_iter=6, self_weight=1)
    assert r.changed == [s, 0] and r.converged
    assert r.labels.tolist() == [0] * (s + 1)


def test_isolated_and_empty(gg, orc):
    g = gg.from_edges(5, [])
    for sw in (0, 1):
        r = orc.rak(g, tol=0.0, max_iter=3, self_weight=sw)
        assert r.labels.tolist() == list(range(5))
        assert r.changed == [0] and r.converged
    g0 = gg.from_edges(0, [])
    r = orc.rak(g0, tol=0.0, max_iter=3)
    assert r.labels.size == 0 and r.changed == [0]
    r = orc.rak(gg.sbm(200, 4, 0.3, 0.01, 5), tol=0.05, max_iter=0)
    assert r.iterations == 0 and r.labels.tolist() == list(range(200))


def test_tolerance_is_floor_of_fraction(gg, orc):
    # path P_10: changed_t = 10 - t.  tol=0.25 -> thr = 2 -> stop at t=8.
    g = gg.from_edges(10, [(i, i + 1) for i in range(9)])
    assert orc.rak(g, tol=0.25, max_iter=20).iterations == 8
    assert orc.rak(g, tol=0.29, max_iter=20).iterations == 8   # floor(2.9) = 2
    assert orc.rak(g, tol=0.3, max_iter=20).iterations == 7    # thr = 3
    assert orc.rak(g, tol=1.0, max_iter=20).iterations == 1


def test_weights_pick_heaviest_label(gg, orc):
    # vertex 0 has neighbours 1 (w 5) and 2,3 (w 2 each, both labelled 9 after
    # we relabel): heaviest single label is 9 (4) only if 1's weight < 4.
    g = gg.from_edges(4, [(0, 1), (0, 2), (0, 3)])
    wm = {(0, 1): 5, (0, 2): 2, (0, 3): 2}
    src = np.repeat(np.arange(4), np.diff(g.row_ptr).astype(np.int64))
    g.w = np.array([wm[(min(a, b), max(a, b))] for a, b in zip(src, g.col)], dtype=np.uint32)
    L = np.array([0, 1, 3, 3], dtype=np.uint32)
    new, _ = orc.rak_round(g, L, self_weight=0)
    assert new[0] == 1  # 5 > 4
    g.w[g.w == 5] = 4
    new, _ = orc.rak_round(g, L, self_weight=0)
    assert new[0] == 1  # 4 vs 4: tie -> lowest label 1
    g.w[g.w == 4] = 3
    new, _ = orc.rak_round(g, L, self_weight=0)
    assert new[0] == 3  # 3 < 4


# ------------------------------------------------------------ brute force --

@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_exhaustive_small_graphs(gg, orc, n):
    for edges in all_graphs(n):
        g = gg.from_edges(n, edges)
        E, A = dense(g)
        for sw in (0, 1):
            L, ch, conv = brute_run(E, A, sw, 0.0, 8)
            r = orc.rak(g, tol=0.0, max_iter=8, self_weight=sw)
            assert r.labels.tolist() == L, (edges, sw)
            assert r.changed == ch and r.converged == conv


def test_sampled_six_vertex_graphs(gg, orc):
    rng = np.random.default_rng(6)
    pairs = list(itertools.combinations(range(6), 2))
    for mask in rng.choice(1 << 15, size=600, replace=False):
        edges = [p for i, p in enumerate(pairs) if int(mask) >> i & 1]
        g = gg.from_edges(6, edges)
        E, A = dense(g)
        for sw in (0, 1):
            L, ch, conv = brute_run(E, A, sw, 0.0, 8)
            r = orc.rak(g, tol=0.0, max_iter=8, self_weight=sw)
            assert r.labels.tolist() == L and r.changed == ch and r.converged == conv


def test_random_weighted_small_graphs(gg, orc):
    rng = np.random.default_rng(7)
    for trial in range(150):
        n = int(rng.integers(2, 13))
        p = rng.uniform(0.1, 0.9)
        edges = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < p]
        lo = int(rng.integers(0, 2))  # zero weights allowed: such labels stay candidates
        g = gg.from_edges(n, edges, weights=(trial, lo, int(rng.integers(lo, 9))))
        E, A = dense(g)
        sw = int(rng.choice([0, 1, 3]))
        tol = float(rng.choice([0.0, 0.1, 0.3]))
        L, ch, conv = brute_run(E, A, sw, tol, 10)
        r = orc.rak(g, tol=tol, max_iter=10, self_weight=sw)
        assert r.labels.tolist() == L and r.changed == ch and r.converged == conv
        lab = np.array(L, dtype=np.uint32)
        assert Fraction(orc.modularity(g, lab).q).limit_denominator(10**12) == pytest.approx(
            brute_modularity(E, A, L), abs=1e-12)


# ------------------------------------------------------------ invariants --

def closed_neighbourhood_ok(g, old, new):
    for v in range(g.n):
        nb = [int(old[v])] + [int(old[u]) for u in g.col[g.row_ptr[v]:g.row_ptr[v + 1]]]
        if int(new[v]) not in nb:
            return False
    return True


def test_closed_neighbourhood_every_round(gg, orc):
    for g in (gg.rmat(9, seed=3), gg.road(20, 30, seed=9), gg.sbm(300, 6, 0.2, 0.01, 4)):
        for sw in (0, 1):
            L = np.arange(g.n, dtype=np.uint32)
            for _ in range(6):
                N, _ = orc.rak_round(g, L, self_weight=sw)
                assert closed_neighbourhood_ok(g, L, N)
                L = N


def fixed_point_ok(g, L, sw):
    """Every vertex already holds its own vote winner (checked by tallying
    with numpy, independent of the oracle's sorted-pair vote)."""
    deg = np.diff(g.row_ptr).astype(np.int64)
    src = np.repeat(np.arange(g.n), deg)
    w = np.ones(g.m, dtype=np.int64) if g.w is None else g.w.astype(np.int64)
    key_lab = L[g.col].astype(np.int64)
    if sw > 0:
        src = np.concatenate([src, np.arange(g.n)])
        key_lab = np.concatenate([key_lab, L.astype(np.int64)])
        w = np.concatenate([w, np.full(g.n, sw, np.int64)])
    pair = src * g.n + key_lab
    up, inv = np.unique(pair, return_inverse=True)
    tally = np.bincount(inv, weights=w).astype(np.int64)
    pv, pl = up // g.n, up % g.n
    order = np.lexsort((pl, -tally, pv))  # per vertex: heaviest first, then lowest label
    first = np.ones(len(order), dtype=bool)
    first[1:] = pv[order][1:] != pv[order][:-1]
    win = np.array(L, dtype=np.int64)
    win[pv[order][first]] = pl[order][first]
    return np.array_equal(win, L.astype(np.int64))


def test_fixed_point_at_tol_zero(gg, orc):
    graphs = [gg.sbm(400, 8, 0.3, 0.005, 11), gg.rmat(10, seed=5), gg.road(16, 16, seed=2),
              gg.with_weights(gg.sbm(300, 5, 0.2, 0.01, 12), 3, 1, 6)]
    seen = 0
    for g in graphs:
        for sw in (0, 1):
            r = orc.rak(g, tol=0.0, max_iter=60, self_weight=sw)
            if r.converged:
                seen += 1
                assert fixed_point_ok(g, r.labels, sw)
            else:
                assert r.iterations == 60 and r.changed[-1] > 0
    assert seen >= 3


def test_fixed_point_check_catches_non_fixed_labels(gg, orc):
    g = gg.sbm(200, 4, 0.3, 0.01, 13)
    assert not fixed_point_ok(g, np.arange(g.n, dtype=np.uint32), 1)


def test_resume_equals_uninterrupted(gg, orc):
    g = gg.rmat(11, seed=8)
    full = orc.rak(g, tol=0.0, max_iter=6)
    part = orc.rak(g, tol=0.0, max_iter=3)
    rest = orc.rak(g, tol=0.0, max_iter=3, init_labels=part.labels)
    assert np.array_equal(rest.labels, full.labels)
    assert part.changed + rest.changed == full.changed


def test_masked_replay_all_ones_equals_plain(gg, orc):
    g = gg.road(30, 30, seed=5)
    masks = np.ones((5, g.n), dtype=np.uint8)
    out, ch = orc.rak_masked(g, masks)
    r = orc.rak(g, tol=0.0, max_iter=5)
    assert np.array_equal(out, r.labels) and ch == r.changed
    masks[2, ::2] = 0  # skipped vertices copy their label
    out2, _ = orc.rak_masked(g, masks[:3])
    L = np.arange(g.n, dtype=np.uint32)
    for t in range(3):
        N, _ = orc.rak_round(g, L)
        N[masks[t] == 0] = L[masks[t] == 0]
        L = N
    assert np.array_equal(out2, L)


# ------------------------------------------------------------ modularity --

def test_modularity_closed_forms(gg, orc):
    g = gg.sbm(500, 5, 0.2, 0.02, 21)
    assert orc.modularity(g, np.zeros(g.n, np.uint32)).q == pytest.approx(0.0, abs=1e-15)
    k = np.diff(g.row_ptr).astype(np.float64)
    single = orc.modularity(g, np.arange(g.n, dtype=np.uint32)).q
    assert single == pytest.approx(-np.sum(k * k) / g.m ** 2, rel=1e-12)
    assert orc.modularity(gg.from_edges(4, []), np.arange(4, dtype=np.uint32)).q == 0.0


def test_modularity_range_and_bruteforce(gg, orc):
    rng = np.random.default_rng(3)
    for _ in range(40):
        n = int(rng.integers(2, 14))
        edges = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < 0.4]
        g = gg.from_edges(n, edges, weights=(int(rng.integers(1 << 30)), 1, 5))
        lab = rng.integers(0, n, size=n).astype(np.uint32)
        E, A = dense(g)
        q = orc.modularity(g, lab).q
        assert -0.5 - 1e-12 <= q <= 1.0
        assert q == pytest.approx(float(brute_modularity(E, A, lab.tolist())), abs=1e-12)
    # bipartite K_{3,3} split by side is the -0.5 extreme
    g = gg.from_edges(6, [(i, j) for i in range(3) for j in range(3, 6)])
    assert orc.modularity(g, np.array([0, 0, 0, 3, 3, 3], np.uint32)).q == pytest.approx(-0.5)


# -------------------------------------------------------------------- NMI --

def test_nmi_against_sklearn(orc):
    from sklearn.metrics import normalized_mutual_info_score as skl
    rng = np.random.default_rng(9)
    for _ in range(30):
        n = int(rng.integers(1, 300))
        a = rng.integers(0, int(rng.integers(1, 12)), size=n)
        b = rng.integers(0, int(rng.integers(1, 12)), size=n)
        assert orc.nmi(a, b) == pytest.approx(skl(a, b, average_method="arithmetic"), abs=1e-12)


def test_nmi_identities(orc):
    rng = np.random.default_rng(10)
    a = rng.integers(0, 7, size=500)
    perm = rng.permutation(7)
    assert orc.nmi(a, a) == pytest.approx(1.0)
    assert orc.nmi(a, perm[a] + 100) == pytest.approx(1.0)
    assert orc.nmi(np.zeros(10), np.zeros(10)) == 1.0
    # independent partitions: the 2x2 product partition has I = 0
    x = np.array([0, 0, 1, 1] * 25)
    y = np.array([0, 1, 0, 1] * 25)
    assert orc.nmi(x, y) == pytest.approx(0.0, abs=1e-12)


# ------------------------------------------------------------ error paths --

def test_oracle_rejects_bad_input(gg, orc):
    bad_col = gg.from_csr_arrays(2, [0, 1, 2], [1, 5])
    with pytest.raises(orc.OracleError):
        orc.rak(bad_col)
    bad_rp = gg.from_csr_arrays(2, [0, 2, 1], [1, 0])
    with pytest.raises(orc.OracleError):
        orc.rak(bad_rp)
    heavy = gg.from_csr_arrays(2, [0, 1, 2], [1, 0], [0xFFFFFFFF, 0xFFFFFFFF])
    with pytest.raises(orc.OracleError) as ei:
        orc.rak(heavy, self_weight=1)
    assert ei.value.code == -2
    ok = orc.rak(heavy, self_weight=0, max_iter=1)
    assert ok.labels.tolist() == [1, 0]
    with pytest.raises(orc.OracleError):
        orc.rak(gg.from_edges(3, [(0, 1)]), tol=1.5)


# ------------------------------------------------ OpenMP build of the oracle --

@pytest.mark.parametrize("make", [
    lambda gg: gg.rmat(14, seed=14),
    lambda gg: gg.with_weights(gg.rmat(13, seed=5), 9, 1, 6),
    lambda gg: gg.road(256, 256, 0.3, 0.01, 1, 8, seed=7),
    lambda gg: gg.sbm(2000, 20, 0.1, 0.005, seed=3),
])
def test_parallel_oracle_equals_sequential(make):
    """The OpenMP build of the same source (the paper's OpenMP RAK, Section
    3.2: a round's vertices shared among threads, a vote buffer per thread)
    gives the sequential labels and changed counts bit for bit: synchronous
    rounds only read the previous round's labels."""
    import graphgen as gg
    import oracle
    g = make(gg)
    for sw in (0, 1):
        seq = oracle.rak(g, tol=0.0, max_iter=12, self_weight=sw)
        par = oracle.rak(g, tol=0.0, max_iter=12, self_weight=sw, parallel=True)
        assert np.array_equal(seq.labels, par.labels)
        assert seq.changed == par.changed and seq.iterations == par.iterations
        lab, ch = oracle.rak_round(g, seq.labels, self_weight=sw, parallel=True)
        lab2, ch2 = oracle.rak_round(g, seq.labels, self_weight=sw)
        assert ch == ch2 and np.array_equal(lab, lab2)
    assert oracle.threads(True) >= 1 and oracle.threads(False) == 1


# ------------------------- non-strict (hashed) ties and semi-synchronous rounds --

def brute_round_ext(E, A, L, sw, active=None, prio=None):
    """Definition-level vote over every label value 0..n-1 (dense), for the
    vertices with active[v] (all when None); the heaviest label present wins,
    ties going to the highest prio(v, label) (None: the lowest label)."""
    n = len(L)
    new = list(L)
    for v in range(n):
        if active is not None and not active[v]:
            continue
        best, best_key = None, None
        for lab in range(n):
            present = sw > 0 and L[v] == lab
            tally = sw if present else 0
            for u in range(n):
                if E[v, u] and L[u] == lab:
                    present = True
                    tally += A[v, u]
            if not present:
                continue
            key = (tally, -lab if prio is None else prio(v, lab))
            if best_key is None or key > best_key:
                best, best_key = lab, key
        new[v] = L[v] if best is None else best
    return new


def brute_run_ext(E, A, sw, tol, max_iter, halves_t=None, prio_t=None):
    """Rounds of brute_round_ext; halves_t(t) gives round t's split (None:
    synchronous rounds), prio_t(t, v, label) the tie priorities."""
    n = E.shape[0]
    L = list(range(n))
    thr = math.floor(tol * n)
    changed = []
    for t in range(1, max_iter + 1):
        prio = None if prio_t is None else (lambda v, lab, t=t: prio_t(t, v, lab))
        if halves_t is None:
            N = brute_round_ext(E, A, L, sw, None, prio)
        else:
            halves = halves_t(t)
            M = brute_round_ext(E, A, L, sw, [h == 0 for h in halves], prio)
            N = brute_round_ext(E, A, M, sw, [h == 1 for h in halves], prio)
        ch = sum(1 for a, b in zip(L, N) if a != b)
        changed.append(ch)
        L = N
        if ch <= thr:
            return L, changed, True
    return L, changed, False


def test_splitmix64_known_answers(orc):
    # the first outputs of SplitMix64 started from state 0, as published with
    # the generator's reference code
    assert [orc.splitmix64_at(0, c) for c in range(3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                                          0x06C45D188009454F]


def test_lowbias32_inverts_with_published_inverse(orc):
    # the inverse published with lowbias32 recovers every input: a bijection,
    # so two labels never share a tie priority
    M = 0xFFFFFFFF

    def inv(x):
        x ^= x >> 16
        x = x * 0x43021123 & M
        x ^= (x >> 15) ^ (x >> 30)
        x = x * 0x1D69E2A5 & M
        x ^= x >> 16
        return x

    xs = [0, 1, 2, M, 0x80000000] + [int(x) for x in np.random.default_rng(1).integers(0, 1 << 32, 3000)]
    assert all(inv(orc.lowbias32(x)) == x for x in xs)
    assert len({orc.lowbias32(x) for x in range(1 << 12)}) == 1 << 12


def hashed_prio(orc, seed):
    return lambda t, v, lab: orc.lowbias32(lab ^ orc.tie_key(seed, t, v))


@pytest.mark.parametrize("n", [3, 4, 5])
def test_hashed_tie_brute_force_small_graphs(gg, orc, n):
    """Every graph on n <= 5 vertices: the oracle's non-strict votes equal the
    dense voter that breaks ties by the highest priority."""
    rng = np.random.default_rng(n)
    for edges in all_graphs(n):
        g = gg.from_edges(n, edges)
        E, A = dense(g)
        for sw in (0, 1):
            seed = int(rng.integers(0, 1 << 63))
            L, ch, conv = brute_run_ext(E, A, sw, 0.0, 6, None, hashed_prio(orc, seed))
            r = orc.rak_ext(g, tol=0.0, max_iter=6, self_weight=sw, tie="hash", seed=seed)
            assert r.labels.tolist() == L and r.changed == ch and r.converged == conv, (edges, sw)


def test_hashed_tie_picks_uniformly(gg, orc):
    """Non-strict mode picks a random one of the tied labels (Section 3.2):
    the centre of a star K_{1,5} with self weight 0 sees five labels of
    tally 1; over 3000 seeds each wins about a fifth of the time (chi-square,
    4 degrees of freedom, 0.1 % level 18.5), and the strict mode always takes
    the lowest."""
    g = gg.from_edges(6, [(0, i) for i in range(1, 6)])
    wins = np.zeros(6, int)
    for seed in range(3000):
        lab, _ = orc.rak_ext(g, tol=1.0, max_iter=1, self_weight=0, tie="hash", seed=seed).labels, 0
        wins[int(lab[0])] += 1
    assert wins[0] == 0 and wins.sum() == 3000
    exp = 3000 / 5
    chi2 = float(((wins[1:] - exp) ** 2 / exp).sum())
    assert chi2 < 18.5, wins
    assert orc.rak_ext(g, tol=1.0, max_iter=1, self_weight=0).labels[0] == 1


def test_hashed_equals_strict_without_ties(gg, orc):
    """With self weight 0 and distinct powers of two as edge weights no two
    labels ever tie, so the non-strict and strict modes agree."""
    rng = np.random.default_rng(3)
    for trial in range(40):
        n = int(rng.integers(4, 12))
        pairs = [p for p in itertools.combinations(range(n), 2) if rng.random() < 0.4][:30]
        if not pairs:
            continue
        g = gg.from_edges(n, pairs)
        wmap = {}
        for i, (a, b) in enumerate(pairs):
            wmap[(a, b)] = wmap[(b, a)] = 1 << i
        src = np.repeat(np.arange(n), np.diff(g.row_ptr).astype(np.int64))
        g.w = np.array([wmap[(int(s), int(d))] for s, d in zip(src, g.col)], dtype=np.uint32)
        a = orc.rak_ext(g, tol=0.0, max_iter=8, self_weight=0, tie="hash", seed=trial)
        b = orc.rak(g, tol=0.0, max_iter=8, self_weight=0)
        assert np.array_equal(a.labels, b.labels) and a.changed == b.changed


@pytest.mark.parametrize("n", [3, 4, 5])
def test_semisync_brute_force_small_graphs(gg, orc, n):
    """Every graph on n <= 5 vertices, under a random split kept for every
    round and under the splits drawn per round: the oracle's semi-synchronous
    rounds equal two dense half-rounds per round, the second reading the
    labels the first left."""
    rng = np.random.default_rng(10 + n)
    for edges in all_graphs(n):
        g = gg.from_edges(n, edges)
        E, A = dense(g)
        for sw in (0, 1):
            halves = rng.integers(0, 2, n).astype(np.uint8)
            L, ch, conv = brute_run_ext(E, A, sw, 0.0, 6, lambda t: halves.tolist())
            r = orc.rak_ext(g, tol=0.0, max_iter=6, self_weight=sw, order="semisync", halves=halves)
            assert r.labels.tolist() == L and r.changed == ch and r.converged == conv, (edges, sw, halves)
            seed = int(rng.integers(0, 1 << 63))  # halves drawn every round, and hashed ties
            L, ch, conv = brute_run_ext(E, A, sw, 0.0, 6, lambda t: [orc.half_of(seed, t, v) for v in range(n)],
                                        hashed_prio(orc, seed))
            r = orc.rak_ext(g, tol=0.0, max_iter=6, self_weight=sw, order="semisync", tie="hash", seed=seed)
            assert r.labels.tolist() == L and r.changed == ch, (edges, sw, seed)


def test_semisync_closed_forms(gg, orc):
    # K2, self weight 0: in different halves the first mover takes the other's
    # label and the pair agrees; in the same half they swap forever
    g = gg.from_edges(2, [(0, 1)])
    r = orc.rak_ext(g, tol=0.0, max_iter=6, self_weight=0, order="semisync", halves=np.array([0, 1], np.uint8))
    assert r.labels.tolist() == [1, 1] and r.changed == [1, 0] and r.converged
    r = orc.rak_ext(g, tol=0.0, max_iter=6, self_weight=0, order="semisync", halves=np.array([1, 1], np.uint8))
    assert r.changed == [2] * 6 and not r.converged
    # path P_n, self weight 1, even vertices in the first half: even i >= 2
    # takes i-1, odd vertices keep theirs except an odd last vertex, which
    # ties and takes its neighbour's new label; stable from round 2
    for n in range(2, 12):
        g = gg.from_edges(n, [(i, i + 1) for i in range(n - 1)])
        halves = np.array([i % 2 for i in range(n)], np.uint8)
        want = [i - 1 if (i % 2 == 0 and i >= 2) else i for i in range(n)]
        if (n - 1) % 2 == 1:
            want[n - 1] = want[n - 2]
        r = orc.rak_ext(g, tol=0.0, max_iter=10, self_weight=1, order="semisync", halves=halves)
        ch1 = sum(1 for i in range(n) if want[i] != i)
        assert r.labels.tolist() == want and r.changed == [ch1, 0], n


def test_semisync_with_one_half_is_synchronous(gg, orc):
    """If every vertex is in the first half the second half-round is empty
    and a semi-synchronous round is a synchronous one."""
    for g in (gg.rmat(11, seed=2), gg.with_weights(gg.road(40, 40, 0.3, 0.01, 1, 8, seed=3), 1, 1, 8)):
        for tie in ("lowest", "hash"):
            a = orc.rak_ext(g, tol=0.0, max_iter=10, order="semisync", tie=tie, seed=9,
                            halves=np.zeros(g.n, np.uint8))
            b = orc.rak_ext(g, tol=0.0, max_iter=10, tie=tie, seed=9)
            assert np.array_equal(a.labels, b.labels) and a.changed == b.changed


def test_semisync_converges_on_road_lattice(gg, orc):
    """The motivation for the semi-synchronous order: on a road-like lattice
    synchronous rounds keep swapping labels (nearly every vertex changes in
    every round), while two half-rounds per round settle; the drawn halves
    split the vertices about evenly, independently from round to round.  A
    split kept fixed leaves the pairs of mutually heaviest neighbours that
    share a half swapping forever."""
    g = gg.road(128, 128, 0.3, 0.01, 1, 8, seed=11)
    s = orc.rak_ext(g, tol=0.05, max_iter=20)
    h = orc.rak_ext(g, tol=0.05, max_iter=20, order="semisync", seed=11)
    assert not s.converged and min(s.changed) > 0.5 * g.n
    assert h.converged and h.iterations <= 8
    assert orc.modularity(g, h.labels).q > 0.6
    h1 = np.array([orc.half_of(11, 1, v) for v in range(g.n)])
    h2 = np.array([orc.half_of(11, 2, v) for v in range(g.n)])
    assert abs(int(h1.sum()) - g.n / 2) < 4 * math.sqrt(g.n)
    assert abs(int((h1 == h2).sum()) - g.n / 2) < 4 * math.sqrt(g.n)
    fixed = orc.rak_ext(g, tol=0.05, max_iter=20, order="semisync", halves=h1.astype(np.uint8))
    assert not fixed.converged


def test_parallel_oracle_ext_equals_sequential(gg, orc):
    g = gg.with_weights(gg.rmat(13, seed=8), 2, 1, 4)
    for order in ("sync", "semisync"):
        for tie in ("lowest", "hash"):
            a = orc.rak_ext(g, tol=0.0, max_iter=8, order=order, tie=tie, seed=77)
            b = orc.rak_ext(g, tol=0.0, max_iter=8, order=order, tie=tie, seed=77, parallel=True)
            assert np.array_equal(a.labels, b.labels) and a.changed == b.changed


# ------------------------------------------------------------------ COPRA --

ONE = 1 << 16  # the oracle's fixed-point belonging coefficient 1


def brute_copra(E, A, V, tol, max_iter, order="sync", prio_t=None, halves_t=None):
    """COPRA (Section 3.3) by its definition on a dense state matrix B[v][c]
    (coefficients in units of 2^-16): collect sum_u A[v,u] B[u][c] for every
    label value c, keep c iff tally * V >= total, keep only the best label
    when nothing passes, normalise with floors and give the remainder to the
    best label; a vertex with no arcs is its own community.  Returns the
    best labels, the changed counts and the final state as sorted pairs."""
    n = E.shape[0]
    B = [[ONE if c == v else 0 for c in range(n)] for v in range(n)]
    best = list(range(n))
    thr = math.floor(tol * n)
    changed = []

    def vote(v, Bs, t):
        total = int(A[v].sum()) * ONE
        tally = [sum(int(A[v, u]) * Bs[u][c] for u in range(n)) for c in range(n)]
        present = [c for c in range(n) if any(E[v, u] and Bs[u][c] for u in range(n))]
        if not present:
            return [ONE if c == v else 0 for c in range(n)], v
        key = (lambda c: (tally[c], -c)) if prio_t is None else (lambda c: (tally[c], prio_t(t, v, c)))
        b = max(present, key=key)
        kept = [c for c in present if tally[c] > 0 and tally[c] * V >= total]
        row = [0] * n
        if not kept:
            row[b] = ONE
            return row, b
        s = sum(tally[c] for c in kept)
        for c in kept:
            row[c] = tally[c] * ONE // s
        row[b] += ONE - sum(row)
        return row, b

    for t in range(1, max_iter + 1):
        nb = list(best)
        passes = [None] if order == "sync" else [0, 1]
        for h in passes:
            NB = [list(r) for r in B]
            for v in range(n):
                if h is not None and halves_t(t)[v] != h:
                    continue
                NB[v], nb[v] = vote(v, B, t)
            B = NB
        ch = sum(1 for a, b in zip(best, nb) if a != b)
        changed.append(ch)
        best = nb
        if ch <= thr:
            break
    state = [sorted((c, x) for c, x in enumerate(B[v]) if x) for v in range(n)]
    return best, changed, state


@pytest.mark.parametrize("n", [3, 4, 5])
def test_copra_brute_force_small_graphs(gg, orc, n):
    """Every graph on n <= 5 vertices, unit and random weights, max_labels 1
    to 3, synchronous and semi-synchronous, strict and hashed ties: the
    oracle's best labels, changed counts and final states equal the dense
    definition."""
    rng = np.random.default_rng(20 + n)
    for edges in all_graphs(n):
        if not edges:
            continue
        g = gg.from_edges(n, edges)
        if rng.random() < 0.5:
            wmap = {}
            for a, b in edges:
                wmap[(a, b)] = wmap[(b, a)] = int(rng.integers(1, 5))
            src = np.repeat(np.arange(n), np.diff(g.row_ptr).astype(np.int64))
            g.w = np.array([wmap[(int(s), int(d))] for s, d in zip(src, g.col)], dtype=np.uint32)
        E, A = dense(g)
        V = int(rng.integers(1, 4))
        order = "semisync" if rng.random() < 0.5 else "sync"
        tie = "hash" if rng.random() < 0.5 else "lowest"
        seed = int(rng.integers(0, 1 << 63))
        best, ch, state = brute_copra(E, A, V, 0.0, 5, order, hashed_prio(orc, seed) if tie == "hash" else None,
                                      lambda t: [orc.half_of(seed, t, v) for v in range(n)])
        r = orc.copra(g, max_labels=V, tol=0.0, max_iter=5, order=order, tie=tie, seed=seed)
        assert r.labels.tolist() == best and r.changed == ch, (edges, V, order, tie)
        assert r.state == state, (edges, V, order, tie)


def test_copra_one_label_is_rak_without_self_loop(gg, orc):
    """With max_labels 1 a label is kept only when it is the only one, so a
    vertex takes its best label: COPRA is RAK with self weight 0 (labels and
    changed counts), in every order and tie rule."""
    for g in (gg.rmat(12, seed=3), gg.with_weights(gg.road(48, 48, 0.3, 0.01, 1, 8, seed=4), 2, 1, 8),
              gg.with_weights(gg.sbm(800, 8, 0.1, 0.01, seed=5), 7, 1, 3)):
        for order in ("sync", "semisync"):
            for tie in ("lowest", "hash"):
                c = orc.copra(g, max_labels=1, tol=0.0, max_iter=8, order=order, tie=tie, seed=11)
                r = orc.rak_ext(g, tol=0.0, max_iter=8, self_weight=0, order=order, tie=tie, seed=11)
                assert np.array_equal(c.labels, r.labels) and c.changed == r.changed, (g.name, order, tie)
                assert all(len(s) == 1 and s[0][1] == ONE for s in c.state)


def test_copra_state_invariants(gg, orc):
    """Every vertex holds 1..max_labels labels whose coefficients sum to 1,
    its best label among them with the largest coefficient."""
    g = gg.with_weights(gg.rmat(11, seed=6), 3, 1, 6)
    for V in (2, 4, 8):
        r = orc.copra(g, max_labels=V, tol=0.0, max_iter=6, tie="hash", seed=V)
        for v, st in enumerate(r.state):
            assert 1 <= len(st) <= V
            assert sum(x for _, x in st) == ONE
            d = dict(st)
            assert int(r.labels[v]) in d and d[int(r.labels[v])] == max(d.values())


def test_copra_closed_forms(gg, orc):
    # star K_{1,s}, max_labels >= s, one round: the centre keeps every leaf's
    # label with floor(1/s) and the remainder on label 1 (lowest of the tied
    # best); each leaf keeps the centre's label alone
    for s in (3, 4, 5):
        g = gg.from_edges(s + 1, [(0, i) for i in range(1, s + 1)])
        r = orc.copra(g, max_labels=s, tol=0.0, max_iter=1)
        q = ONE // s
        assert r.state[0] == [(1, q + ONE - s * q)] + [(i, q) for i in range(2, s + 1)]
        assert all(r.state[i] == [(0, ONE)] for i in range(1, s + 1))
        assert r.labels.tolist() == [1] + [0] * s and r.changed == [s + 1]
        # below the threshold: max_labels < s keeps only the best label
        r = orc.copra(g, max_labels=s - 1, tol=0.0, max_iter=1)
        assert r.state[0] == [(1, ONE)]
    # clique K_s, max_labels >= s-1: round 1 every vertex keeps the s-1 other
    # labels with equal shares, the remainder on the lowest other label
    for s in (3, 4, 6):
        g = gg.from_edges(s, itertools.combinations(range(s), 2))
        r = orc.copra(g, max_labels=s - 1, tol=0.0, max_iter=1)
        q = ONE // (s - 1)
        for v in range(s):
            others = [u for u in range(s) if u != v]
            want = [(u, q + (ONE - (s - 1) * q if u == others[0] else 0)) for u in others]
            assert r.state[v] == want
    # isolated vertices stay their own community
    g = gg.from_edges(4, [(0, 1)])
    r = orc.copra(g, max_labels=2, tol=0.0, max_iter=3)
    assert r.state[2] == [(2, ONE)] and r.state[3] == [(3, ONE)]
    # arcs of weight 0 bring labels but no weight: the best (lowest) label alone
    g = gg.from_edges(3, [(0, 1), (0, 2)])
    g.w = np.zeros(g.m, np.uint32)
    r = orc.copra(g, max_labels=4, tol=0.0, max_iter=1)
    assert r.state[0] == [(1, ONE)] and r.state[1] == [(0, ONE)] and r.state[2] == [(0, ONE)]
