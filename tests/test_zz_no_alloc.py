"""The allocation-free modularity entry point (lpa_modularity_noalloc)
against lpa_modularity, which allocates its scratch from the context, and
against the oracle: identical integer terms and Q (modularity, Section 1).

Calls follow each other on one GPU with smaller inputs after larger ones,
so each call finds the previous call's sums in the fixed scratch and must
clear what it uses.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


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


def both(lpa, ctx, orc, g, labels_np, weights=True):
    import torch
    dg = lpa.DeviceGraph.from_csr(g, "cuda", weights=weights)
    lab = torch.from_numpy(np.ascontiguousarray(labels_np, dtype=np.uint32).view(np.int32)).to("cuda")
    q_ref, t_ref = ctx.modularity(dg, lab)
    q_na, t_na = ctx.modularity_noalloc(dg, lab)
    say(f"[noalloc] {getattr(g, 'name', '')} n={g.n} m={g.m}: Q={q_na:.6f}")
    assert t_na == t_ref, (t_na, t_ref)
    assert q_na == q_ref
    gw = g if weights else type(g)(n=g.n, row_ptr=g.row_ptr, col=g.col, w=None)
    m = orc.modularity(gw, labels_np)
    assert t_na == {"two_m": m.two_m, "sigma_in": m.sigma_in, "sum_k2": m.sum_k2}
    assert abs(q_na - m.q) <= 1e-9
    return q_na


def test_noalloc_equals_modularity_calls_in_a_row(gg, orc, lpa):
    import torch
    with lpa.Context(0) as ctx:
        # the largest n the fixed scratch takes (R-MAT 22 has 2^22 vertices),
        # labels of a plain run
        g = gg.rmat(22, 16, 0.57, 0.19, 0.19, seed=22)
        assert g.n == lpa.LPA_NOALLOC_MAX_N
        dg = lpa.DeviceGraph.from_csr(g, "cuda")
        lab, _ = ctx.run(dg, tol=0.05, max_iter=20)
        both(lpa, ctx, orc, g, lpa.labels_to_numpy(lab))
        del dg
        # then smaller inputs: weighted, long rows (a 1200-arc star), isolated
        # vertices, random labels, unit weights
        rng = np.random.default_rng(11)
        gw = gg.with_weights(gg.rmat(14, seed=3), 5, 1, 8)
        both(lpa, ctx, orc, gw, rng.integers(0, 64, gw.n))
        star = gg.from_edges(1300, [(0, i) for i in range(1, 1201)])
        star.name = "star1200+100 isolated"
        both(lpa, ctx, orc, star, rng.integers(0, star.n, star.n))
        sbm = gg.sbm(2000, 20, 0.1, 0.005, seed=2)
        both(lpa, ctx, orc, sbm, np.arange(sbm.n) // 100)
        both(lpa, ctx, orc, sbm, np.zeros(sbm.n))
        one = gg.from_edges(1, [])
        q, t = ctx.modularity_noalloc(lpa.DeviceGraph.from_csr(one, "cuda"),
                                      torch.zeros(1, dtype=torch.int32, device="cuda"))
        assert q == 0.0 and t == {"two_m": 0, "sigma_in": 0, "sum_k2": 0}


def test_noalloc_errors(gg, lpa):
    import torch
    with lpa.Context(0) as ctx:
        g = gg.rmat(10, seed=5)
        dg = lpa.DeviceGraph.from_csr(g, "cuda")
        # one vertex past the fixed scratch: refused on the host, nothing launched
        big = lpa.DeviceGraph(lpa.LPA_NOALLOC_MAX_N + 1, dg.row_ptr, dg.col)
        lab_big = torch.zeros(1, dtype=torch.int32, device="cuda")
        with pytest.raises(lpa.LpaError) as ei:
            ctx.modularity_noalloc(big, lab_big)
        assert ei.value.code == lpa.LPA_ETOOLARGE
        # a label >= n is flagged by the kernel (counted as label 0 meanwhile)
        lab = torch.zeros(g.n, dtype=torch.int32, device="cuda")
        lab[7] = g.n
        with pytest.raises(lpa.LpaError) as ei:
            ctx.modularity_noalloc(dg, lab)
        assert ei.value.code == lpa.LPA_EINVAL
        # a row_ptr that does not end at m
        rp = dg.row_ptr.clone()
        rp[-1] = rp[-1] - 1
        bad = lpa.DeviceGraph(g.n, rp, dg.col)
        with pytest.raises(lpa.LpaError) as ei:
            ctx.modularity_noalloc(bad, torch.zeros(g.n, dtype=torch.int32, device="cuda"))
        assert ei.value.code == lpa.LPA_EINVAL
        # and the next good call is unaffected by the flagged ones
        q, t = ctx.modularity_noalloc(dg, torch.zeros(g.n, dtype=torch.int32, device="cuda"))
        q2, t2 = ctx.modularity(dg, torch.zeros(g.n, dtype=torch.int32, device="cuda"))
        assert t == t2 and q == q2
