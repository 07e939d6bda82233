"""GPU parity of COPRA (arXiv 2301.09125, Section 3.3) against the oracle's
orc_copra: best labels, per-round changed counts, round counts and the final
state (kept labels, fixed-point belonging coefficients, counts) bit for bit,
in both update orders and with both tie rules.

The graphs reach every path: rows of deg * max_labels <= 32 (16 lanes
each) and <= 512 (one wavefront each), longer rows (one block with an LDS
table, or in round 1 without one when each neighbour is listed once, and
with one when a row repeats neighbours), and rows whose distinct labels
outgrow that table (a broom's centre: tables in device memory).
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ORDER = {"sync": 0, "semisync": 1}
TIE = {"lowest": 0, "hash": 1}
MODES = [(o, t) for o in ORDER for t in TIE]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lpa():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import paper_2301_09125_amd as P
    return P


def dev(lpa, g):
    return lpa.DeviceGraph.from_csr(g, "cuda")


def star(gg, arms):
    g = gg.from_edges(arms + 1, [(0, i) for i in range(1, arms + 1)])
    g.name = f"star{arms}"
    return g


def assert_copra(orc, lpa, g, V, order, tie, seed, tol=0.01, max_iter=20, **opts):
    ref = orc.copra(g, max_labels=V, tol=tol, max_iter=max_iter, order=order, tie=tie, seed=seed)
    with lpa.Context(0, order=ORDER[order], tie=TIE[tie], seed=seed, **opts) as c:
        best, st, (sl, sc, sn) = c.run_copra(dev(lpa, g), max_labels=V, tol=tol, max_iter=max_iter, state=True)
    tag = (getattr(g, "name", ""), V, order, tie, seed)
    assert st.changed == ref.changed, (tag, st.changed, ref.changed)
    assert st.iterations == ref.iterations and st.converged == ref.converged, tag
    got = lpa.labels_to_numpy(best)
    mism = np.flatnonzero(got != ref.labels)
    assert mism.size == 0, f"{tag}: {mism.size} best labels differ, first {mism[:8]}"
    cnt = sn.cpu().numpy().view(np.uint32)
    lab = sl.cpu().numpy().view(np.uint32)
    coef = sc.cpu().numpy().view(np.uint32)
    ref_cnt = np.array([len(s) for s in ref.state], dtype=np.uint32)
    assert np.array_equal(cnt, ref_cnt), tag
    for v in range(g.n):
        k = int(cnt[v])
        if list(zip(lab[v, :k].tolist(), coef[v, :k].tolist())) != ref.state[v]:
            raise AssertionError(f"{tag}: state of vertex {v} differs: "
                                 f"{list(zip(lab[v, :k].tolist(), coef[v, :k].tolist()))} vs {ref.state[v]}")
    assert st.arcs_processed == g.m * st.iterations
    return ref, st


def corpus(gg):
    return [gg.rmat(10, seed=3), gg.with_weights(gg.rmat(12, seed=4), 6, 1, 5), gg.sbm(2000, 20, 0.1, 0.005, seed=2),
            gg.road(64, 64, 0.3, 0.01, 1, 8, seed=5), star(gg, 1200)]


@pytest.mark.parametrize("order,tie", MODES)
def test_copra_corpus(gg, orc, lpa, order, tie):
    for g in corpus(gg):
        for V in (1, 2, 3, 4, 7, 16):  # records of 4, 8, 8, 16, 16 and 64 words
            say("[copra]", order, tie, getattr(g, "name", ""), g.n, g.m, "V", V)
            assert_copra(orc, lpa, g, V, order, tie, 7 + V, tol=0.0, max_iter=8)


def test_copra_max_labels_64_and_tolerances(gg, orc, lpa):
    g = gg.with_weights(gg.rmat(11, seed=8), 3, 1, 4)
    for tol in (0.0, 0.01, 0.05):
        assert_copra(orc, lpa, g, 64, "sync", "lowest", 1, tol=tol)
        assert_copra(orc, lpa, g, 64, "semisync", "hash", 2, tol=tol)


def broom(gg, arms):
    # a centre with `arms` leaves, each leaf with a pendant of its own: after
    # round 1 every leaf holds the centre's label and its pendant's, so in
    # round 2 the centre collects arms + 1 distinct labels
    g = gg.from_edges(2 * arms + 1, [(0, i) for i in range(1, arms + 1)] + [(i, arms + i) for i in range(1, arms + 1)])
    g.name = f"broom{arms}"
    return g


def test_copra_rows_beyond_the_lds_table(gg, orc, lpa):
    # the broom's centre in round 2 (5001 distinct labels) is more than the
    # block's LDS table takes: voted with a table in device memory; a
    # 5000-arc star decides its centre in round 1 without a table; the
    # R-MAT graph has rows of every kind
    for g in (broom(gg, 5000), star(gg, 5000), gg.rmat(15, seed=15)):
        for order, tie in MODES:
            say("[copra] big rows", getattr(g, "name", ""), order, tie)
            assert_copra(orc, lpa, g, 4, order, tie, 3, tol=0.0, max_iter=6)


def test_copra_long_row_with_repeated_neighbours(gg, orc, lpa):
    # a 600-arc row that lists each of its 300 neighbours twice: round 1
    # must sum the repeats (the table path, not the one-arc-per-label one)
    rp = np.concatenate([[0, 600], 600 + np.arange(1, 301)]).astype(np.uint64)
    col = np.concatenate([np.repeat(np.arange(1, 301), 2), np.zeros(300)]).astype(np.uint32)
    g = gg.from_csr_arrays(301, rp, col, name="repeats600")
    for order, tie in MODES:
        for V in (1, 4):
            assert_copra(orc, lpa, g, V, order, tie, 5, tol=0.0, max_iter=4)
    gw = gg.from_csr_arrays(301, rp, col, w=np.arange(1, 901, dtype=np.uint32) % 7, name="repeats600_w")
    assert_copra(orc, lpa, gw, 4, "sync", "lowest", 0, tol=0.0, max_iter=4)


def test_copra_one_label_is_rak_without_self_weight(gg, orc, lpa):
    # max_labels = 1 keeps only the best label: RAK with self weight 0
    g = gg.with_weights(gg.rmat(13, seed=6), 2, 1, 7)
    with lpa.Context(0) as c:
        best, st = c.run_copra(dev(lpa, g), max_labels=1, tol=0.05, max_iter=20)
    ref = orc.rak(g, tol=0.05, max_iter=20, self_weight=0)
    assert np.array_equal(lpa.labels_to_numpy(best), ref.labels)
    assert st.changed == ref.changed


def test_copra_reports_modularity_and_repeats(gg, orc, lpa):
    g = gg.sbm(2000, 20, 0.1, 0.005, seed=9)
    with lpa.Context(0, modularity=1) as c:
        b1, st1 = c.run_copra(dev(lpa, g), max_labels=4, tol=0.01, max_iter=20)
        b2, st2 = c.run_copra(dev(lpa, g), max_labels=4, tol=0.01, max_iter=20)
    l1 = lpa.labels_to_numpy(b1)
    assert np.array_equal(l1, lpa.labels_to_numpy(b2)) and st1.changed == st2.changed
    m = orc.modularity(g, l1)
    assert st1.mod_terms == {"two_m": m.two_m, "sigma_in": m.sigma_in, "sum_k2": m.sum_k2}
    assert abs(st1.modularity - m.q) <= 1e-9


def test_copra_degenerate_and_errors(gg, orc, lpa):
    import torch
    with lpa.Context(0) as c:
        # isolated vertices and max_iter 0
        g = gg.from_edges(5, [(0, 1)])
        best, st = c.run_copra(dev(lpa, g), max_labels=4, tol=0.0, max_iter=0)
        assert st.iterations == 0 and np.array_equal(lpa.labels_to_numpy(best), np.arange(5))
        ref, _ = assert_copra(orc, lpa, g, 4, "sync", "lowest", 0, tol=0.0, max_iter=5)
        for V in (0, 65):
            with pytest.raises(lpa.LpaError) as ei:
                c.run_copra(dev(lpa, g), max_labels=V)
            assert ei.value.code == lpa.LPA_EINVAL
        # a col value >= n is found before any round reads the state
        d = dev(lpa, gg.rmat(8, seed=2))
        col = d.col.clone()
        col[3] = d.n
        with pytest.raises(lpa.LpaError) as ei:
            c.run_copra(lpa.DeviceGraph(d.n, d.row_ptr, col), max_labels=4)
        assert ei.value.code == lpa.LPA_EINVAL
        # empty graph
        e = lpa.DeviceGraph(0, torch.zeros(1, dtype=torch.int64, device="cuda"),
                            torch.zeros(0, dtype=torch.int32, device="cuda"))
        _, st = c.run_copra(e, max_labels=4)
        assert st.iterations == 0
    with pytest.raises(lpa.LpaError) as ei:
        with lpa.Context(0, frontier=1) as c:
            c.run_copra(dev(lpa, g), max_labels=4)
    assert ei.value.code == lpa.LPA_EUNSUPPORTED
