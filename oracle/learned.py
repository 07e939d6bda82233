"""FP64 reference of the learned frontier's predictor: features, the MLP
forward pass and the gradients of its training loss.

TEST INFRASTRUCTURE ONLY, like the rest of this package: the GPU library
never imports it and shares none of its code.

The paper (arXiv 2301.09125) has no learned component; its Section 2 names
frontier-based label propagation as a way to visit fewer edges.  Here a
small network predicts which vertices of a round can change; the rules
below define it:

features of a candidate vertex v before round t (from the state after round
t-1; top1 / top2 = the winning tally and the best other tally of v's most
recent vote, k_v = weighted degree, sw = self weight):
    f1 = log2(1 + deg v)
    f2 = (top1 - top2) / (k_v + sw)
    f3 = 1 if v changed in round t-1 else 0
    f4 = top1 / (k_v + sw)
    f5 = 1 if v or a neighbour changed in round t-1 else 0
    f6 = t / max_iter
network (weights W1 6x32, W2 32x32, w3 32; biases b1, b2, b3):
    h1 = relu(x W1 + b1),  h2 = relu(bf16(h1) W2 + b2),  z = h2 . w3 + b3
with x, W1, W2, w3 rounded to bfloat16 (round to nearest, ties to even) and
everything else exact; v is kept iff z >= logit(tau).
loss: binary cross-entropy on the logit z with weight pos_weight on the
positive class (y = 1: v changed in round t), averaged over the samples.
Rounding is treated as the identity in the gradients (straight-through).
"""
from __future__ import annotations

import numpy as np

N_FEAT = 6
HIDDEN = 32


def bf16_round(x) -> np.ndarray:
    """Round to the nearest bfloat16 value (ties to even), returned as
    float64.  The value is first rounded to float32 (the precision the
    features and weights are held in)."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    nan = np.isnan(f)
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    if np.any(nan):
        out = np.where(nan, np.nan, out)
    return out


def features(deg, kw, top1, top2, changed_prev, frontier, t: int, max_iter: int, self_weight: int = 1):
    """Feature rows (float64, N x 6) of the rules above."""
    deg = np.asarray(deg, dtype=np.float64)
    den = np.asarray(kw, dtype=np.float64) + float(self_weight)
    den = np.where(den > 0, den, 1.0)
    t1 = np.asarray(top1, dtype=np.float64)
    t2 = np.asarray(top2, dtype=np.float64)
    X = np.empty((deg.size, N_FEAT), dtype=np.float64)
    X[:, 0] = np.log2(1.0 + deg)
    X[:, 1] = (t1 - t2) / den
    X[:, 2] = np.asarray(changed_prev, dtype=np.float64)
    X[:, 3] = t1 / den
    X[:, 4] = np.asarray(frontier, dtype=np.float64)
    X[:, 5] = float(t) / float(max_iter)
    return X


def init_model(seed: int = 0) -> dict:
    """He-initialised float32 master weights (what the trainer starts from)."""
    rng = np.random.default_rng(seed)
    return {
        "w1": (rng.standard_normal((N_FEAT, HIDDEN)) * np.sqrt(2.0 / N_FEAT)).astype(np.float32),
        "b1": np.zeros(HIDDEN, np.float32),
        "w2": (rng.standard_normal((HIDDEN, HIDDEN)) * np.sqrt(2.0 / HIDDEN)).astype(np.float32),
        "b2": np.zeros(HIDDEN, np.float32),
        "w3": (rng.standard_normal(HIDDEN) * np.sqrt(1.0 / HIDDEN)).astype(np.float32),
        "b3": np.float32(0.0),
    }


def _q(a, quantize: bool):
    return bf16_round(a) if quantize else np.asarray(a, dtype=np.float64)


def forward(X, model: dict, quantize: bool = True):
    """Logits z (float64, N) and the intermediate values."""
    x = _q(X, quantize)
    w1, w2, w3 = _q(model["w1"], quantize), _q(model["w2"], quantize), _q(model["w3"], quantize)
    b1 = np.asarray(model["b1"], np.float64)
    b2 = np.asarray(model["b2"], np.float64)
    b3 = float(model["b3"])
    a1 = x @ w1 + b1
    h1 = np.maximum(a1, 0.0)
    h1q = _q(h1, quantize)
    a2 = h1q @ w2 + b2
    h2 = np.maximum(a2, 0.0)
    z = h2 @ w3 + b3
    return z, {"x": x, "a1": a1, "h1q": h1q, "a2": a2, "h2": h2, "w2": w2, "w3": w3}


def logits(X, model: dict, quantize: bool = True) -> np.ndarray:
    return forward(X, model, quantize)[0]


def _softplus(x):
    return np.logaddexp(0.0, x)


def loss(X, y, model: dict, pos_weight: float = 1.0, quantize: bool = True) -> float:
    z = logits(X, model, quantize)
    y = np.asarray(y, dtype=np.float64)
    # -[pw y log s(z) + (1-y) log(1-s(z))],  log s(z) = -softplus(-z)
    return float(np.mean(pos_weight * y * _softplus(-z) + (1.0 - y) * _softplus(z)))


def loss_grad(X, y, model: dict, pos_weight: float = 1.0, quantize: bool = True):
    """(loss, gradients) of the mean weighted BCE with respect to every
    parameter, by the chain rule through the layers above."""
    z, c = forward(X, model, quantize)
    y = np.asarray(y, dtype=np.float64)
    N = z.size
    s = 1.0 / (1.0 + np.exp(-z))
    L = float(np.mean(pos_weight * y * _softplus(-z) + (1.0 - y) * _softplus(z)))
    dz = (s * (pos_weight * y + 1.0 - y) - pos_weight * y) / N
    g = {}
    g["w3"] = c["h2"].T @ dz
    g["b3"] = float(np.sum(dz))
    dh2 = np.outer(dz, c["w3"])
    da2 = dh2 * (c["a2"] > 0)
    g["w2"] = c["h1q"].T @ da2
    g["b2"] = np.sum(da2, axis=0)
    dh1 = da2 @ c["w2"].T
    da1 = dh1 * (c["a1"] > 0)
    g["w1"] = c["x"].T @ da1
    g["b1"] = np.sum(da1, axis=0)
    return L, g


def tau_for_recall(z_pos: np.ndarray, recall: float = 0.99) -> float:
    """The largest logit threshold that keeps at least `recall` of the
    positive samples (z >= threshold), as a probability tau."""
    z = np.sort(np.asarray(z_pos, dtype=np.float64))
    if z.size == 0:
        return 0.5
    k = int(np.floor((1.0 - recall) * z.size))
    thr = z[k]
    return float(1.0 / (1.0 + np.exp(-thr)))
