"""GPU parity at the full sizes of the benchmark workloads, in the launch
configuration bench.py times (default options, tol 0.05, max 20 rounds,
self weight 1): the planted-partition SBM, R-MAT scale 22 and the
4096 x 4096 road lattice are each run in full by the oracle and compared
bit-exactly (labels, per-round changed counts, iterations), and the
modularity integer terms are compared exactly.
"""
import sys
import time

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


@pytest.fixture(scope="module")
def ctx(lpa):
    c = lpa.Context(0)
    yield c
    c.close()


def full_compare(gg, orc, lpa, ctx, g):
    t = time.time()
    dg = lpa.DeviceGraph.from_csr(g, "cuda")
    lab, st = ctx.run(dg, tol=0.05, max_iter=20)
    got = lpa.labels_to_numpy(lab)
    q, terms = ctx.modularity(dg, lab)
    say(f"{g.name}: gpu {st.iterations} rounds {st.changed} in {st.ms_total:.1f} ms")
    ref = orc.rak(g, tol=0.05, max_iter=20, self_weight=1)
    say(f"{g.name}: oracle done in {time.time() - t:.1f}s")
    assert st.changed == ref.changed and st.iterations == ref.iterations and st.converged == ref.converged
    mism = np.flatnonzero(got != ref.labels)
    assert mism.size == 0, f"{mism.size} labels differ, first {mism[:8]}"
    mref = orc.modularity(g, ref.labels)
    assert (terms["two_m"], terms["sigma_in"], terms["sum_k2"]) == (mref.two_m, mref.sigma_in, mref.sum_k2)
    assert abs(q - mref.q) <= 1e-9


@pytest.mark.timeout(600)
def test_sbm_config_full(gg, orc, lpa, ctx):
    full_compare(gg, orc, lpa, ctx, gg.sbm(10000, 100, 0.1, 0.001, seed=1))


@pytest.mark.timeout(900)
def test_rmat22_full(gg, orc, lpa, ctx):
    t = time.time()
    g = gg.rmat(22, 16, 0.57, 0.19, 0.19, seed=22)
    say(f"rmat22 generated in {time.time() - t:.1f}s: n={g.n} m={g.m}")
    full_compare(gg, orc, lpa, ctx, g)


@pytest.mark.timeout(900)
def test_road4096_full(gg, orc, lpa, ctx):
    t = time.time()
    g = gg.road(4096, 4096, 0.3, 0.01, 1, 8, seed=4096)
    say(f"road generated in {time.time() - t:.1f}s: n={g.n} m={g.m}")
    full_compare(gg, orc, lpa, ctx, g)
