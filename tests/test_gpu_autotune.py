"""GPU tests of the degree-bin autotuner (lpa_autotune): it times the
candidate thresholds, caches its choice per degree signature, and the runs
that follow still give the oracle's labels (RAK, arXiv 2301.09125, Section
3.2): the thresholds change the speed only.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lpa():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import paper_2301_09125_amd as P
    return P


def valid(o):
    return (1 <= o["thread_max"] <= 8 and o["thread_max"] <= o["group_max"] <= 32 and
            o["group_max"] <= o["wave_max"] <= 128 and o["wave_max"] <= o["wide_max"] <= 512)


def test_autotune_plain_then_cached(gg, orc, lpa):
    c = lpa.Context(0)
    try:
        for g in (gg.rmat(15, 16, seed=15), gg.with_weights(gg.sbm(4000, 40, 0.02, 0.002, seed=2), 1, 1, 5)):
            dg = lpa.DeviceGraph.from_csr(g, "cuda")
            o, n = c.autotune(dg)
            assert n == 16 and valid(o), (g.name, o)
            o2, n2 = c.autotune(dg)
            assert n2 == 0 and o2 == o
            ref = orc.rak(g, tol=0.05, max_iter=20)
            lab, st = c.run(dg, tol=0.05, max_iter=20)
            assert st.changed == ref.changed and np.array_equal(lpa.labels_to_numpy(lab), ref.labels), g.name
    finally:
        c.close()


def test_autotune_batch(gg, orc, lpa):
    b = gg.sbm_batch(G=48, n_min=50, n_max=2000, seed=9)
    c = lpa.Context(0)
    try:
        dg = lpa.DeviceGraph.from_csr(b.csr, "cuda")
        o, n = c.autotune(dg, b.gv)
        assert n == 16 and valid(o)
        lab, st = c.run_batch(dg, b.gv, tol=0.05, max_iter=20)
        lab = lpa.labels_to_numpy(lab)
        for k in range(0, b.G, 5):
            ref = orc.rak(b.graph(k), tol=0.05, max_iter=20)
            v0, v1 = int(b.gv[k]), int(b.gv[k + 1])
            assert np.array_equal(lab[v0:v1], ref.labels) and st.changed(k) == ref.changed
    finally:
        c.close()
