"""Pins of the oracle parts used by the learned frontier: the per-vertex
top-two tallies of a round, bfloat16 rounding, the MLP forward pass and the
gradients of its training loss.  Each is checked against something other
than the oracle's own formula: a dense brute-force tally, closed forms,
PyTorch's bfloat16 conversion and float64 autograd, and central finite
differences.
"""
import itertools

import numpy as np
import pytest


@pytest.fixture(scope="module")
def lrn():
    from oracle import learned
    return learned


def dense_top2(n, edges, weights, labels, sw):
    """Per vertex: the winning tally (lowest label among maxima) and the best
    tally of another label present in the closed neighbourhood."""
    T = {}
    for v in range(n):
        T[v] = {}
        if sw:
            T[v][labels[v]] = T[v].get(labels[v], 0) + sw
    for (a, b), w in zip(edges, weights):
        T[a][labels[b]] = T[a].get(labels[b], 0) + w
        T[b][labels[a]] = T[b].get(labels[a], 0) + w
    t1, t2, new = [], [], []
    for v in range(n):
        if not T[v]:
            t1.append(0), t2.append(0), new.append(labels[v])
            continue
        best = max(T[v].values())
        win = min(l for l, x in T[v].items() if x == best)
        others = [x for l, x in T[v].items() if l != win]
        t1.append(best), t2.append(max(others) if others else 0), new.append(win)
    return np.array(new), np.array(t1), np.array(t2)


@pytest.mark.parametrize("sw", [0, 1, 3])
def test_top2_brute_force(gg, orc, sw):
    rng = np.random.default_rng(100 + sw)
    for trial in range(60):
        n = int(rng.integers(1, 8))
        pairs = [(a, b) for a, b in itertools.combinations(range(n), 2) if rng.random() < 0.5]
        g = gg.from_edges(n, pairs, weights=(trial, 0, 4))
        src = np.repeat(np.arange(n), np.diff(g.row_ptr).astype(np.int64))
        wmap = {(int(a), int(b)): int(w) for a, b, w in zip(src, g.col, g.w)}
        edges = [(a, b) for a, b in pairs]
        weights = [wmap[(a, b)] for a, b in pairs]
        labels = rng.integers(0, n, n).astype(np.uint32)
        new, ch, t1, t2 = orc.rak_round_top2(g, labels, self_weight=sw)
        ref_new, ref_t1, ref_t2 = dense_top2(n, edges, weights, labels.tolist(), sw)
        assert np.array_equal(new, ref_new)
        assert np.array_equal(t1, ref_t1), (n, pairs, labels, t1, ref_t1)
        assert np.array_equal(t2, ref_t2), (n, pairs, labels, t2, ref_t2)
        assert ch == int(np.sum(new != labels))


def test_top2_closed_forms(gg, orc):
    # K_s from unique labels: every label once; with self weight 1 the own
    # label also has tally 1 -> top1 = top2 = 1; with self weight 2 the own
    # label wins with 2 over 1
    s = 6
    g = gg.from_edges(s, list(itertools.combinations(range(s), 2)))
    lab = np.arange(s, dtype=np.uint32)
    _, _, t1, t2 = orc.rak_round_top2(g, lab, 1)
    assert t1.tolist() == [1] * s and t2.tolist() == [1] * s
    new, ch, t1, t2 = orc.rak_round_top2(g, lab, 2)
    assert ch == 0 and t1.tolist() == [2] * s and t2.tolist() == [1] * s
    # one community: a single label, no runner-up
    _, _, t1, t2 = orc.rak_round_top2(g, np.zeros(s, np.uint32), 1)
    assert t1.tolist() == [s] * s and t2.tolist() == [0] * s
    # isolated vertex, self weight 0: empty vote
    g = gg.from_edges(2, [])
    new, ch, t1, t2 = orc.rak_round_top2(g, np.array([1, 0], np.uint32), 0)
    assert new.tolist() == [1, 0] and t1.tolist() == [0, 0] and t2.tolist() == [0, 0]


def test_bf16_round_matches_torch(lrn):
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-6, 6, 20000),
                        [0.0, -0.0, 1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -9, 3.0e38, -1e-40]]).astype(np.float32)
    # exact ties: values halfway between two bfloat16 numbers
    ties = (np.arange(1, 200, dtype=np.uint32) << 16 | 0x8000).view(np.float32)
    x = np.concatenate([x, ties, -ties])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(lrn.bf16_round(x), ref)


def test_forward_closed_form(lrn):
    m = {k: np.zeros_like(v) for k, v in lrn.init_model(0).items()}
    m["w1"][0, 0] = 1.0
    m["w2"][0, 0] = 1.0
    m["w3"][0] = 1.0
    m["b3"] = np.float32(0.25)
    X = np.zeros((4, 6))
    X[:, 0] = [0.5, 2.0, -3.0, 0.0]
    assert lrn.logits(X, m).tolist() == [0.75, 2.25, 0.25, 0.25]
    # biases pass through relu
    m["b1"][1] = 2.0
    m["w2"][1, 1] = 0.5
    m["w3"][1] = -1.0
    assert lrn.logits(X, m).tolist() == [-0.25, 1.25, -0.75, -0.75]


def _torch_model(torch, m, quantize):
    def q(a):
        t = torch.tensor(np.asarray(a, np.float32))
        return (t.to(torch.bfloat16) if quantize else t).to(torch.float64)
    return {k: (q(v) if k in ("w1", "w2", "w3") else torch.tensor(np.asarray(v, np.float64)))
            for k, v in m.items()}


@pytest.mark.parametrize("quantize", [False, True])
def test_forward_matches_torch(lrn, quantize):
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(7)
    m = lrn.init_model(3)
    m["b1"] = rng.standard_normal(32).astype(np.float32) * 0.1
    m["b2"] = rng.standard_normal(32).astype(np.float32) * 0.1
    X = rng.random((500, 6)) * np.array([16, 1, 1, 1, 1, 1])
    t = _torch_model(torch, m, quantize)
    x = (torch.tensor(X.astype(np.float32)).to(torch.bfloat16).to(torch.float64) if quantize
         else torch.tensor(X))
    h1 = torch.relu(x @ t["w1"] + t["b1"])
    if quantize:
        h1 = h1.to(torch.float32).to(torch.bfloat16).to(torch.float64)
    h2 = torch.relu(h1 @ t["w2"] + t["b2"])
    z = h2 @ t["w3"] + t["b3"]
    assert np.allclose(lrn.logits(X, m, quantize), z.numpy(), rtol=0, atol=1e-12)


def test_gradient_finite_differences(lrn):
    rng = np.random.default_rng(11)
    m = {k: np.asarray(v, np.float64) for k, v in lrn.init_model(5).items()}
    m["b1"] = rng.standard_normal(32) * 0.1
    m["b2"] = rng.standard_normal(32) * 0.1
    X = rng.random((64, 6)) * np.array([10, 1, 1, 1, 1, 1])
    y = (rng.random(64) < 0.3).astype(np.float64)
    L, g = lrn.loss_grad(X, y, m, pos_weight=3.0, quantize=False)
    assert abs(L - lrn.loss(X, y, m, 3.0, quantize=False)) < 1e-14
    h = 1e-6
    for k in ("w1", "b1", "w2", "b2", "w3", "b3"):
        base = np.array(m[k], dtype=np.float64)
        num = np.zeros_like(base)
        it = np.nditer(base, flags=["multi_index"]) if base.ndim else [None]
        for idx in (it if base.ndim else [()]):
            ix = it.multi_index if base.ndim else ()
            for sgn in (+1, -1):
                pert = base.copy()
                pert[ix] += sgn * h
                mm = dict(m)
                mm[k] = pert
                num[ix] += sgn * lrn.loss(X, y, mm, 3.0, quantize=False) / (2 * h)
        ana = np.asarray(g[k], dtype=np.float64)
        err = np.linalg.norm(ana - num) / max(np.linalg.norm(num), 1e-12)
        assert err < 1e-5, (k, err)


@pytest.mark.parametrize("quantize", [False, True])
def test_gradient_matches_torch_autograd(lrn, quantize):
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(12)
    m = lrn.init_model(6)
    m["b1"] = rng.standard_normal(32).astype(np.float32) * 0.1
    m["b2"] = rng.standard_normal(32).astype(np.float32) * 0.1
    X = rng.random((200, 6)) * np.array([12, 1, 1, 1, 1, 1])
    y = (rng.random(200) < 0.2).astype(np.float64)
    L, g = lrn.loss_grad(X, y, m, pos_weight=4.0, quantize=quantize)
    t = _torch_model(torch, m, quantize)
    for v in t.values():
        v.requires_grad_(True)
    x = (torch.tensor(X.astype(np.float32)).to(torch.bfloat16).to(torch.float64) if quantize
         else torch.tensor(X))
    h1 = torch.relu(x @ t["w1"] + t["b1"])
    if quantize:  # straight-through rounding
        h1 = h1 + (h1.detach().to(torch.float32).to(torch.bfloat16).to(torch.float64) - h1.detach())
    h2 = torch.relu(h1 @ t["w2"] + t["b2"])
    z = h2 @ t["w3"] + t["b3"]
    yt = torch.tensor(y)
    lt = torch.nn.functional.binary_cross_entropy_with_logits(z, yt, pos_weight=torch.tensor(4.0))
    lt.backward()
    assert abs(float(lt) - L) < 1e-12
    for k in ("w1", "b1", "w2", "b2", "w3", "b3"):
        assert np.allclose(np.asarray(g[k]), t[k].grad.numpy(), rtol=1e-10, atol=1e-14), k


def test_features_closed_form(lrn):
    X = lrn.features(deg=[3, 0, 7], kw=[3, 0, 14], top1=[3, 1, 10], top2=[1, 0, 4], changed_prev=[1, 0, 0],
                     frontier=[1, 0, 1], t=5, max_iter=20, self_weight=1)
    assert X[0].tolist() == [2.0, 0.5, 1.0, 0.75, 1.0, 0.25]
    assert X[1].tolist() == [0.0, 1.0, 0.0, 1.0, 0.0, 0.25]
    assert X[2].tolist() == [3.0, 6 / 15, 0.0, 10 / 15, 1.0, 0.25]


def test_tau_for_recall(lrn):
    z = np.arange(100, dtype=np.float64)
    tau = lrn.tau_for_recall(z, 0.99)
    thr = np.log(tau / (1 - tau))
    assert np.sum(z >= thr - 1e-9) == 99
    assert abs(thr - 1.0) < 1e-9
