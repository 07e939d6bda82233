"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Bar: bit-exact labels, identical per-round changed counts, iteration counts
and convergence flags; modularity with identical integer terms (Q within
1e-9, expected equal).  RAK of arXiv 2301.09125 Section 3.2, modularity of
Section 1.
"""
import itertools
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    return torch


@pytest.fixture(scope="module")
def lpa(torch_mod):
    import paper_2301_09125_amd as P
    return P


@pytest.fixture(scope="module")
def ctx(lpa):
    c = lpa.Context(0)
    yield c
    c.close()


def dev(lpa, g, weights=True):
    return lpa.DeviceGraph.from_csr(g, "cuda", weights=weights)


def gpu_run(lpa, ctx, g, tol, max_iter, sw, **opts):
    dg = dev(lpa, g)
    c = ctx if (sw == 1 and not opts) else lpa.Context(0, self_weight=sw, **opts)
    lab, st = c.run(dg, tol=tol, max_iter=max_iter)
    return lpa.labels_to_numpy(lab), st


def assert_same(orc, lpa, ctx, g, tol=0.05, max_iter=20, sw=1, **opts):
    ref = orc.rak(g, tol=tol, max_iter=max_iter, self_weight=sw)
    lab, st = gpu_run(lpa, ctx, g, tol, max_iter, sw, **opts)
    assert st.iterations == ref.iterations, (g.name, st.changed, ref.changed)
    assert st.changed == ref.changed, (g.name, st.changed, ref.changed)
    assert st.converged == ref.converged
    mism = np.flatnonzero(lab != ref.labels)
    assert mism.size == 0, f"{g.name}: {mism.size} labels differ, first {mism[:8]}"
    if not opts.get("frontier"):  # every round votes every arc
        assert st.arcs_processed == g.m * st.iterations, (g.name, st.arcs_processed, g.m, st.iterations)
    return ref, lab, st


# ------------------------------------------------------------ small corpus --

def test_golden_fixture_on_gpu(gg, orc, lpa, ctx):
    import json
    fx = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "weighted6.json")))
    n = fx["n"]
    g = gg.from_edges(n, [(a, b) for a, b, _ in fx["edges"]])
    wmap = {}
    for a, b, w in fx["edges"]:
        wmap[(a, b)] = wmap[(b, a)] = w
    src = np.repeat(np.arange(n), np.diff(g.row_ptr).astype(np.int64))
    g.w = np.array([wmap[(int(s), int(d))] for s, d in zip(src, g.col)], dtype=np.uint32)
    for run in fx["runs"]:
        lab, st = gpu_run(lpa, ctx, g, run["tol"], run["max_iter"], fx["self_weight"])
        assert lab.tolist() == run["labels"]
        assert st.changed == run["changed"] and st.converged == run["converged"]
    m = fx["modularity"]
    q, terms = ctx.modularity(dev(lpa, g), _t(np.array(m["labels"], np.uint32)))
    assert (terms["two_m"], terms["sigma_in"], terms["sum_k2"]) == (m["two_m"], m["sigma_in"], m["sum_k2"])
    assert abs(q - m["q_num"] / m["q_den"]) < 1e-12


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).cuda()


def test_small_graph_corpus(gg, orc, lpa, ctx):
    rng = np.random.default_rng(100)
    graphs = []
    for n in (1, 2, 3, 5, 9):
        graphs.append(gg.from_edges(n, itertools.combinations(range(n), 2)))
    graphs.append(gg.from_edges(17, [(i, i + 1) for i in range(16)]))
    graphs.append(gg.from_edges(10, [(0, i) for i in range(1, 10)]))
    graphs.append(gg.from_edges(6, []))
    for t in range(40):
        n = int(rng.integers(2, 40))
        p = rng.uniform(0.05, 0.8)
        edges = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < p]
        lo = int(rng.integers(0, 2))
        graphs.append(gg.from_edges(n, edges, weights=(t, lo, int(rng.integers(lo, 9)))))
    say("corpus", len(graphs))
    for g in graphs:
        for sw in (0, 1, 3):
            for tol in (0.0, 0.05):
                assert_same(orc, lpa, ctx, g, tol=tol, max_iter=12, sw=sw)


# --------------------------------------------------- every bin, ragged sizes --

@pytest.mark.parametrize("case", ["sbm_cfg", "rmat14", "rmat16_w", "road64_w", "road_ragged"])
def test_mid_graphs_all_bins(gg, orc, lpa, ctx, case):
    if case == "sbm_cfg":
        g = gg.sbm(10000, 100, 0.1, 0.001, 1)
    elif case == "rmat14":
        g = gg.rmat(14, seed=14)
    elif case == "rmat16_w":
        g = gg.with_weights(gg.rmat(16, seed=16), 7, 1, 8)
    elif case == "road64_w":
        g = gg.road(64, 64, seed=64)
    else:
        g = gg.road(37, 211, seed=5)
    say(case, g.n, g.m)
    for sw in (0, 1):
        assert_same(orc, lpa, ctx, g, tol=0.05, max_iter=20, sw=sw)
    assert_same(orc, lpa, ctx, g, tol=0.0, max_iter=30, sw=1)


def test_long_rows_split_into_segments(gg, orc, lpa, ctx):
    # wave_max 40 sends rows above 40 arcs to the segment path; rows above 512
    # arcs are split over several wavefronts and merge through the slab
    g = gg.rmat(15, seed=15)
    deg = np.diff(g.row_ptr)
    assert (deg > 512).sum() > 20 and deg.max() > 2048
    for sw in (0, 1):
        assert_same(orc, lpa, ctx, g, tol=0.0, max_iter=15, sw=sw, wave_max=40, wide_max=40)
        assert_same(orc, lpa, ctx, g, tol=0.05, max_iter=15, sw=sw)
    gw = gg.with_weights(g, 11, 1, 6)
    assert_same(orc, lpa, ctx, gw, tol=0.0, max_iter=15, sw=1, wave_max=33, wide_max=33)


def test_long_rows_slab_merge(gg, orc, lpa, ctx):
    # merge_max 1: every row of two or more segments merges its full tallies
    # through the global slab instead of the top-K reports
    g = gg.rmat(15, seed=19)
    for sw in (0, 1):
        assert_same(orc, lpa, ctx, g, tol=0.0, max_iter=12, sw=sw, merge_max=1)
        assert_same(orc, lpa, ctx, g, tol=0.0, max_iter=12, sw=sw, merge_max=1, wave_max=40, wide_max=40)


def test_long_rows_undecided_reports_fall_back(gg, orc, lpa, ctx):
    # a hub whose neighbours carry labels in pairs: after round 1 every
    # segment reports eight labels of tally 2 and a bound of 2 for the rest,
    # so no leader can be proven and every round of the hub takes the slab
    # fallback.  The answer must still be exact.
    leaves = 6000
    hub = leaves
    edges = [(i, hub) for i in range(leaves)] + [(2 * j, 2 * j + 1) for j in range(leaves // 2)]
    g = gg.from_edges(leaves + 1, edges, weights=(5, 1, 1))
    for sw in (0, 1):
        assert_same(orc, lpa, ctx, g, tol=0.0, max_iter=6, sw=sw)
        assert_same(orc, lpa, ctx, g, tol=0.0, max_iter=6, sw=sw, group_max=8, wave_max=8, wide_max=8)


def test_repeated_neighbours_round_one(gg, orc, lpa, ctx):
    # rows that list a neighbour twice (multigraph arcs) may not take the
    # round-1 direct path; their tallies must add the repeated weights
    import graphgen
    base = gg.rmat(12, seed=31)
    src = np.repeat(np.arange(base.n), np.diff(base.row_ptr).astype(np.int64))
    rng = np.random.default_rng(2)
    dup = rng.random(base.m) < 0.05
    s2 = np.concatenate([src, src[dup]])
    d2 = np.concatenate([base.col.astype(np.int64), base.col[dup].astype(np.int64)])
    order = np.lexsort((rng.random(len(s2)), s2))  # rows unsorted inside
    s2, d2 = s2[order], d2[order]
    rp = np.zeros(base.n + 1, np.uint64)
    np.add.at(rp, s2 + 1, 1)
    rp = np.cumsum(rp).astype(np.uint64)
    g = graphgen.from_csr_arrays(base.n, rp, d2.astype(np.uint32), name="rmat12_multi")
    for sw in (0, 1):
        assert_same(orc, lpa, ctx, g, tol=0.0, max_iter=10, sw=sw)
        assert_same(orc, lpa, ctx, g, tol=0.0, max_iter=10, sw=sw, wave_max=40, wide_max=40)
        # the frontier engine votes the same queued rows in round 1
        assert_same(orc, lpa, ctx, g, tol=0.0, max_iter=10, sw=sw, frontier=1, wave_max=40, wide_max=40)


def test_long_rows_relabelled_by_slices(gg, orc, lpa, ctx):
    # the vertices of a weighted R-MAT graph spread over 9 M ids, so that the
    # long rows are relabelled slice by slice of the id space (at least 8
    # slices): most rows sorted, one reversed, one shuffled, one listing 40
    # neighbours twice (sorted, with repeats)
    import graphgen
    base = gg.with_weights(gg.rmat(14, 16, seed=14), 7, 1, 8)
    n = 9_000_000
    rng = np.random.default_rng(5)
    ids = rng.choice(n, base.n, replace=False).astype(np.int64)
    deg = np.diff(base.row_ptr).astype(np.int64)
    src = np.repeat(ids, deg)
    dst = ids[base.col.astype(np.int64)]
    wts = np.asarray(base.w, dtype=np.uint32)
    order = np.lexsort((dst, src))
    src, dst, wts = src[order], dst[order], wts[order]
    rp = np.zeros(n + 1, np.int64)
    np.add.at(rp, src + 1, 1)
    rp = np.cumsum(rp)
    longs = ids[np.flatnonzero(deg > 512)]
    assert len(longs) >= 3
    a0, a1 = rp[longs[0]], rp[longs[0] + 1]
    dst[a0:a1], wts[a0:a1] = dst[a0:a1][::-1].copy(), wts[a0:a1][::-1].copy()
    b0, b1 = rp[longs[1]], rp[longs[1] + 1]
    p = rng.permutation(b1 - b0)
    dst[b0:b1], wts[b0:b1] = dst[b0:b1][p], wts[b0:b1][p]
    r = longs[2]
    c0, c1 = rp[r], rp[r + 1]
    rc = np.concatenate([dst[c0:c1], dst[c0:c0 + 40]])
    rw = np.concatenate([wts[c0:c1], wts[c0:c0 + 40]])
    o = np.argsort(rc, kind="stable")
    dst = np.concatenate([dst[:c0], rc[o], dst[c1:]])
    wts = np.concatenate([wts[:c0], rw[o], wts[c1:]])
    rp[r + 1:] += 40
    g = graphgen.from_csr_arrays(n, rp.astype(np.uint64), dst.astype(np.uint32), wts, name="rmat14_spread9m")
    say("[slices]", g.n, g.m, "long rows", len(longs))
    for sw in (1, 0):
        ref, lab, st = assert_same(orc, lpa, ctx, g, tol=0.0, max_iter=6, sw=sw)
    ref, lab, st = assert_same(orc, lpa, ctx, g)
    q, terms = ctx.modularity(dev(lpa, g), _t(lab))
    mref = orc.modularity(g, ref.labels)
    assert (terms["two_m"], terms["sigma_in"], terms["sum_k2"]) == (mref.two_m, mref.sigma_in, mref.sum_k2)
    # a resumed run relabels without voting round 1 in the same pass
    dg = dev(lpa, g)
    part, st1 = ctx.run(dg, tol=0.0, max_iter=2)
    start = lpa.labels_to_numpy(part).copy()  # resume overwrites the labels in place
    rest, st2 = ctx.run_resume(dg, part, tol=0.0, max_iter=4)
    ref2 = orc.rak(g, tol=0.0, max_iter=4, init_labels=start)
    assert st2.changed == ref2.changed
    assert np.array_equal(lpa.labels_to_numpy(rest), ref2.labels)


def test_random_bin_thresholds_give_same_labels(gg, orc, lpa, ctx):
    g = gg.with_weights(gg.rmat(13, seed=21), 3, 1, 5)
    ref = orc.rak(g, tol=0.0, max_iter=12, self_weight=1)
    rng = np.random.default_rng(5)
    for _ in range(6):
        t = int(rng.integers(1, 9))
        gm = int(rng.integers(t, 33))
        wm = int(rng.integers(gm, 129))
        xm = int(rng.integers(wm, 513))
        lab, st = gpu_run(lpa, ctx, g, 0.0, 12, 1, thread_max=t, group_max=gm, wave_max=wm, wide_max=xm)
        assert np.array_equal(lab, ref.labels), (t, gm, wm, xm)
        assert st.changed == ref.changed


def test_repeated_runs_bit_identical(gg, lpa, ctx):
    g = dev(lpa, gg.rmat(15, seed=3))
    first, st0 = ctx.run(g, tol=0.0, max_iter=10)
    first = lpa.labels_to_numpy(first)
    for _ in range(3):
        lab, st = ctx.run(g, tol=0.0, max_iter=10)
        assert np.array_equal(lpa.labels_to_numpy(lab), first)
        assert st.changed == st0.changed


def test_resume_equals_uninterrupted(gg, orc, lpa, ctx):
    g = gg.rmat(13, seed=9)
    dg = dev(lpa, g)
    full, stf = ctx.run(dg, tol=0.0, max_iter=8)
    part, st1 = ctx.run(dg, tol=0.0, max_iter=3)
    start = lpa.labels_to_numpy(part).copy()  # resume overwrites the labels in place
    rest, st2 = ctx.run_resume(dg, part, tol=0.0, max_iter=5)
    assert np.array_equal(lpa.labels_to_numpy(rest), lpa.labels_to_numpy(full))
    assert st1.changed + st2.changed == stf.changed
    ref = orc.rak(g, tol=0.0, max_iter=5, init_labels=start)
    assert ref.changed == st2.changed
    assert np.array_equal(lpa.labels_to_numpy(rest), ref.labels)


# ------------------------------------------------------------- modularity --

@pytest.mark.parametrize("case", ["sbm", "rmat15", "road_w", "singletons", "one"])
def test_modularity_matches_oracle(gg, orc, lpa, ctx, case):
    if case in ("sbm", "singletons", "one"):
        g = gg.sbm(3000, 30, 0.1, 0.002, 2)
    elif case == "rmat15":
        g = gg.rmat(15, seed=4)
    else:
        g = gg.road(100, 80, seed=8)
    dg = dev(lpa, g)
    if case == "singletons":
        lab = np.arange(g.n, dtype=np.uint32)
    elif case == "one":
        lab = np.zeros(g.n, dtype=np.uint32)
    else:
        lab = orc.rak(g).labels
    ref = orc.modularity(g, lab)
    q, terms = ctx.modularity(dg, _t(lab))
    assert (terms["two_m"], terms["sigma_in"], terms["sum_k2"]) == (ref.two_m, ref.sigma_in, ref.sum_k2)
    assert abs(q - ref.q) <= 1e-9
    assert q == ref.q  # same exact integers, same FP64 expression


SMALL_BINS = {"thread_max": 2, "group_max": 6, "wave_max": 20, "wide_max": 40, "merge_max": 1}


@pytest.mark.parametrize("opts", [{}, {"self_weight": 0}, SMALL_BINS], ids=["default", "sw0", "small_bins"])
@pytest.mark.parametrize("max_iter,tol", [(1, 0.05), (2, 0.05), (3, 0.0), (20, 0.05), (30, 0.0)])
def test_run_reports_modularity(gg, orc, lpa, opts, max_iter, tol):
    # a run with modularity=1 reports Q of its result; after round 1 it is
    # computed from the last round's own-label sums and the arcs of the rows
    # that changed in it, which must give the full definition exactly
    star = [(0, i) for i in range(1, 700)] + [(i, i + 1) for i in range(1, 699, 3)]
    graphs = (gg.rmat(14, seed=6), gg.road(60, 70, seed=3),
              gg.with_weights(gg.sbm(2000, 20, 0.05, 0.003, seed=5), 9, 1, 7), gg.from_edges(700, star))
    sw = opts.get("self_weight", 1)
    with lpa.Context(0, modularity=1, **opts) as c:
        for g in graphs:
            ref = orc.rak(g, tol=tol, max_iter=max_iter, self_weight=sw)
            mref = orc.modularity(g, ref.labels)
            lab, st = c.run(dev(lpa, g), tol=tol, max_iter=max_iter)
            assert np.array_equal(lpa.labels_to_numpy(lab), ref.labels), g.name
            assert st.mod_terms == {"two_m": mref.two_m, "sigma_in": mref.sigma_in, "sum_k2": mref.sum_k2}, g.name
            assert st.modularity == mref.q


# ---------------------------------------------------------- edge + errors --

def test_degenerate_inputs(gg, lpa, ctx):
    import torch
    g0 = dev(lpa, gg.from_edges(0, []))
    lab, st = ctx.run(g0, tol=0.05, max_iter=5)
    assert lab.numel() == 0 and st.iterations == 0
    iso = dev(lpa, gg.from_edges(7, []))
    lab, st = ctx.run(iso, tol=0.0, max_iter=5)
    assert lpa.labels_to_numpy(lab).tolist() == list(range(7)) and st.changed == [0]
    q, terms = ctx.modularity(iso, lab)
    assert q == 0.0 and terms["two_m"] == 0
    g = dev(lpa, gg.sbm(500, 5, 0.2, 0.01, 3))
    lab, st = ctx.run(g, tol=0.05, max_iter=0)
    assert st.iterations == 0 and lpa.labels_to_numpy(lab).tolist() == list(range(500))
    assert torch.cuda.is_available()


def test_error_codes(gg, lpa, ctx):
    import torch

    def mk(n, rp, col, w=None):
        return lpa.DeviceGraph(n, torch.tensor(rp, dtype=torch.int64).cuda(),
                               torch.tensor(col, dtype=torch.int32).cuda(),
                               None if w is None else torch.tensor(w, dtype=torch.int64).to(torch.int32).cuda())

    with pytest.raises(lpa.LpaError) as e:
        ctx.run(mk(3, [0, 1, 2, 2], [1, 7]))  # col out of range
    assert e.value.code == -1
    with pytest.raises(lpa.LpaError) as e:
        ctx.run(mk(3, [0, 2, 1, 2], [1, 0]))  # row_ptr not monotone
    assert e.value.code == -1
    with pytest.raises(lpa.LpaError) as e:
        ctx.run(mk(2, [0, 1, 3], [1, 0]))  # row_ptr[n] != m
    assert e.value.code == -1
    heavy = mk(2, [0, 1, 2], [1, 0], [0xFFFFFFFF - 0x80000000, 0xFFFFFFFF - 0x80000000])
    with pytest.raises(lpa.LpaError) as e:
        lpa.Context(0, self_weight=0x80000001).run(heavy)
    assert e.value.code == -2
    ok = mk(3, [0, 1, 2, 2], [1, 0])
    with pytest.raises(lpa.LpaError):
        ctx.run(ok, tol=1.5)
    with pytest.raises(lpa.LpaError):
        ctx.run(ok, tol=float("nan"))
    bad = torch.tensor([0, 5, 1], dtype=torch.int32).cuda()
    with pytest.raises(lpa.LpaError):
        ctx.modularity(ok, bad)
    with pytest.raises(lpa.LpaError):
        ctx.run_resume(ok, bad.clone(), tol=0.0, max_iter=2)
    with pytest.raises(lpa.LpaError):
        lpa.Context(0, thread_max=9)
    with pytest.raises(lpa.LpaError):
        lpa.Context(0, wide_max=513)
    with pytest.raises(lpa.LpaError):
        lpa.Context(0, group_max=4, thread_max=8)
    # the context still works after errors
    lab, st = ctx.run(ok, tol=0.0, max_iter=2)
    assert st.iterations >= 1


# ------------------------------------ semi-synchronous rounds, hashed ties --
#
# lpa_options.order / .tie / .seed against the oracle's orc_rak_ext (the
# paper's non-strict mode made reproducible, and two half-rounds per round;
# Sections 3.2 and 3.3): labels, per-round changed counts and rounds equal.

MODES = [("semisync", "lowest"), ("sync", "hash"), ("semisync", "hash")]
ORDER = {"sync": 0, "semisync": 1}
TIE = {"lowest": 0, "hash": 1}


def assert_same_mode(orc, lpa, g, order, tie, seed, tol=0.05, max_iter=20, sw=1, **opts):
    ref = orc.rak_ext(g, tol=tol, max_iter=max_iter, self_weight=sw, order=order, tie=tie, seed=seed,
                      parallel=True)
    with lpa.Context(0, self_weight=sw, order=ORDER[order], tie=TIE[tie], seed=seed, **opts) as c:
        lab, st = c.run(dev(lpa, g), tol=tol, max_iter=max_iter)
    got = lpa.labels_to_numpy(lab)
    tag = (getattr(g, "name", ""), order, tie, seed, sw, opts)
    assert st.changed == ref.changed, (tag, st.changed, ref.changed)
    assert st.iterations == ref.iterations and st.converged == ref.converged, tag
    mism = np.flatnonzero(got != ref.labels)
    assert mism.size == 0, f"{tag}: {mism.size} labels differ, first {mism[:8]}"
    assert st.arcs_processed == g.m * st.iterations
    return ref, got, st


def mode_corpus(gg):
    star = gg.from_edges(1201, [(0, i) for i in range(1, 1201)])  # a 1200-arc row: three segments
    star.name = "star1200"
    return [gg.rmat(10, seed=3), gg.with_weights(gg.rmat(12, seed=4), 6, 1, 5), gg.sbm(2000, 20, 0.1, 0.005, seed=2),
            gg.road(64, 64, 0.3, 0.01, 1, 8, seed=5), star, gg.rmat(15, seed=15)]


@pytest.mark.parametrize("order,tie", MODES)
def test_modes_corpus(gg, orc, lpa, order, tie):
    for g in mode_corpus(gg):
        say("[modes]", order, tie, getattr(g, "name", ""), g.n, g.m)
        for sw, seed in ((1, 7), (0, 123456789)):
            assert_same_mode(orc, lpa, g, order, tie, seed, tol=0.0, max_iter=12, sw=sw)


@pytest.mark.parametrize("order,tie", MODES)
def test_modes_all_bins_and_slab(gg, orc, lpa, order, tie):
    """Every bin and long-row path under the new orders and tie rules:
    random thresholds, and merge_max 1 (every long row merged through the
    global slab)."""
    rng = np.random.default_rng(5)
    g = gg.with_weights(gg.rmat(14, seed=21), 8, 1, 3)
    for k in range(3):
        tm = int(rng.integers(1, 9))
        gm = int(rng.integers(tm, 33))
        wm = int(rng.integers(gm, 129))
        xm = int(rng.integers(wm, 513))
        say("[modes] bins", order, tie, tm, gm, wm, xm)
        assert_same_mode(orc, lpa, g, order, tie, 1000 + k, thread_max=tm, group_max=gm, wave_max=wm, wide_max=xm)
    assert_same_mode(orc, lpa, gg.rmat(15, seed=9), order, tie, 31, merge_max=1)


def test_modes_modularity_and_seeds(gg, orc, lpa):
    """The modularity lpa_run reports for a semi-synchronous run is the full
    definition's; different seeds give different (valid) results and the
    same seed the same result."""
    g = gg.road(96, 96, 0.3, 0.01, 1, 8, seed=8)
    ref, got, _ = assert_same_mode(orc, lpa, g, "semisync", "lowest", 5, modularity=1)
    with lpa.Context(0, order=1, seed=5, modularity=1) as c:
        lab, st = c.run(dev(lpa, g), tol=0.05, max_iter=20)
    m = orc.modularity(g, ref.labels)
    assert st.mod_terms == {"two_m": m.two_m, "sigma_in": m.sigma_in, "sum_k2": m.sum_k2}
    assert abs(st.modularity - m.q) <= 1e-9
    _, other, _ = assert_same_mode(orc, lpa, g, "semisync", "lowest", 6)
    assert not np.array_equal(got, other)


def test_modes_unsupported_combinations(gg, lpa):
    with pytest.raises(lpa.LpaError) as ei:
        lpa.Context(0, order=1, frontier=1)
    assert ei.value.code == lpa.LPA_EUNSUPPORTED
    with pytest.raises(lpa.LpaError) as ei:
        lpa.Context(0, order=2)
    assert ei.value.code == lpa.LPA_EINVAL
    b = gg.sbm_batch(G=4, n_min=50, n_max=100, seed=1)
    with lpa.Context(0, tie=1) as c:
        with pytest.raises(lpa.LpaError) as ei:
            c.run_batch(lpa.DeviceGraph.from_csr(b.csr, "cuda"), b.gv)
        assert ei.value.code == lpa.LPA_EUNSUPPORTED


def test_reuse_csr_equals_fresh(gg, orc, lpa):
    """reuse_csr keeps the binned, relabelled copy between calls on the same
    CSR (round 1 then runs in the round kernels): every call still equals
    the oracle, across graphs that replace the copy, resumes, modes and the
    reported modularity."""
    gs = [gg.with_weights(gg.rmat(14, seed=31), 4, 1, 6), gg.rmat(15, seed=9), gg.sbm(2000, 20, 0.1, 0.005, seed=3)]
    dgs = [dev(lpa, g) for g in gs]
    with lpa.Context(0, reuse_csr=1, modularity=1) as c:
        for rep in range(2):
            for g, dg in zip(gs, dgs):
                for _ in range(2):  # the second call reuses the copy
                    ref = orc.rak(g, tol=0.05, max_iter=20, self_weight=1)
                    lab, st = c.run(dg, tol=0.05, max_iter=20)
                    got = lpa.labels_to_numpy(lab)
                    assert st.changed == ref.changed and np.array_equal(got, ref.labels), (g.name, rep)
                    m = orc.modularity(g, ref.labels)
                    assert st.mod_terms == {"two_m": m.two_m, "sigma_in": m.sigma_in, "sum_k2": m.sum_k2}
        # resume through the kept copy: 2 rounds, then the rest
        g, dg = gs[1], dgs[1]
        lab, st1 = c.run(dg, tol=0.05, max_iter=2)
        lab, st2 = c.run_resume(dg, lab, tol=0.05, max_iter=20)
        ref = orc.rak(g, tol=0.05, max_iter=2, self_weight=1)
        ref = orc.rak(g, tol=0.05, max_iter=20, self_weight=1, init_labels=ref.labels)
        assert np.array_equal(lpa.labels_to_numpy(lab), ref.labels) and st2.changed == ref.changed
    for order, tie in (("semisync", "lowest"), ("sync", "hash")):
        with lpa.Context(0, reuse_csr=1, order=ORDER[order], tie=TIE[tie], seed=4) as c:
            for _ in range(2):
                lab, st = c.run(dgs[0], tol=0.0, max_iter=8)
                ref = orc.rak_ext(gs[0], tol=0.0, max_iter=8, self_weight=1, order=order, tie=tie, seed=4)
                assert st.changed == ref.changed and np.array_equal(lpa.labels_to_numpy(lab), ref.labels)
