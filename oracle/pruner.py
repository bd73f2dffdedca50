"""FP64 reference of the frontier pruner's network.  TEST INFRASTRUCTURE ONLY.

The learned pruner ranks the frontier candidates of a query (s, t): a
first-hop candidate is an edge (s, r1, a) and a second-hop candidate an edge
(b, r3, t).  The paper's generic search keeps a bounded frontier per level
(section 5); here a small network learns which candidates lie on the exact
top-K paths.  For a candidate with vertex v and relation r, u the query
endpoint its edge touches (s for the first hop, t for the second) and w the
other endpoint:

    f  = [X[u], X[w], X[v], Y[r]]                     (4d inputs)
    h1 = relu(W1 f + b1)                              W1: [H, 4d]
    h2 = relu(W2 h1 + b2)                             W2: [H, H]
    z  = w3 . h2 + b3                                 w3: [H]
    p  = sigmoid(z)

Training loss: binary cross-entropy with a weight w_pos on the positive
class, averaged over the N samples of a step:

    L = (1/N) sum_i -( w_pos y_i log p_i + (1 - y_i) log(1 - p_i) )
    dL/dz_i = ( w_pos y_i (p_i - 1) + (1 - y_i) p_i ) / N

Gradients follow by the chain rule; the optimiser is Adam with bias
correction (Kingma & Ba, 2015).

Parameters are one flat float vector in the order W1 (row-major), b1, W2
(row-major), b2, w3, b3.

``bf16=True`` evaluates the same formulas with the operands of every matrix
product rounded to bfloat16 (round to nearest, ties to even) where the GPU
kernels round them: the features, W1, W2 and w3, the activations h1 and h2,
and the back-propagated dz2 = dL/d(W2 h1 + b2) and dz1.  Products and sums
are then exact in FP64, so what remains between this and the GPU is only
the order and precision of the FP32 accumulation.
"""

from __future__ import annotations

import numpy as np


def param_count(d: int, H: int) -> int:
    return H * 4 * d + H + H * H + H + H + 1


def unpack(theta: np.ndarray, d: int, H: int):
    """Views (W1, b1, W2, b2, w3, b3) of the flat parameter vector."""
    theta = np.asarray(theta)
    o = 0
    W1 = theta[o:o + H * 4 * d].reshape(H, 4 * d); o += H * 4 * d
    b1 = theta[o:o + H]; o += H
    W2 = theta[o:o + H * H].reshape(H, H); o += H * H
    b2 = theta[o:o + H]; o += H
    w3 = theta[o:o + H]; o += H
    b3 = theta[o:o + 1]; o += 1
    assert o == len(theta)
    return W1, b1, W2, b2, w3, b3


def pack(W1, b1, W2, b2, w3, b3) -> np.ndarray:
    return np.concatenate([np.ravel(W1), np.ravel(b1), np.ravel(W2), np.ravel(b2), np.ravel(w3),
                           np.ravel(b3)]).astype(np.float64)


def round_bf16(x: np.ndarray) -> np.ndarray:
    """Nearest bfloat16 value (ties to even), returned as float64.  The
    input is first rounded to float32 (the precision the kernels hold)."""
    b = np.ascontiguousarray(np.asarray(x, dtype=np.float32)).view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    b = ((b + 0x7FFF + lsb) >> 16) << 16
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def features(X, Y, s, t, v, r, hop2=None) -> np.ndarray:
    """f_i = [X[u_i], X[w_i], X[v_i], Y[r_i]] in float64 (tables as stored:
    float32 values, or bfloat16 values widened exactly), with (u, w) = (s, t)
    for first-hop candidates and (t, s) where hop2 is true."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    s = np.asarray(s)
    t = np.asarray(t)
    if hop2 is not None:
        hop2 = np.asarray(hop2, dtype=bool)
        s, t = np.where(hop2, t, s), np.where(hop2, s, t)
    return np.concatenate([X[s], X[t], X[v], Y[r]], axis=1)


def sigmoid(z):
    z = np.asarray(z, dtype=np.float64)
    return np.where(z >= 0, 1.0 / (1.0 + np.exp(-np.abs(z))), np.exp(-np.abs(z)) / (1.0 + np.exp(-np.abs(z))))


def forward(theta, F, d, H, bf16=False):
    """Returns z [N] and the intermediate values the backward pass needs."""
    W1, b1, W2, b2, w3, b3 = unpack(theta, d, H)
    rnd = round_bf16 if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    Fq, W1q, W2q, w3q = rnd(F), rnd(W1), rnd(W2), rnd(w3)
    z1 = Fq @ W1q.T + b1
    h1 = rnd(np.maximum(z1, 0.0))
    z2 = h1 @ W2q.T + b2
    h2 = rnd(np.maximum(z2, 0.0))
    z = h2 @ w3q + b3[0]
    cache = dict(F=Fq, W1=W1q, W2=W2q, w3=w3q, z1=z1, h1=h1, z2=z2, h2=h2)
    return z, cache


def bce_loss(z, y, w_pos=1.0):
    """Mean weighted binary cross-entropy of sigmoid(z) against labels y,
    with log p = -log(1 + exp(-z)) evaluated stably."""
    z = np.asarray(z, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    log_p = -np.logaddexp(0.0, -z)        # log sigmoid(z)
    log_1mp = -np.logaddexp(0.0, z)       # log (1 - sigmoid(z))
    return float(np.mean(-(w_pos * y * log_p + (1.0 - y) * log_1mp)))


def bce_grad(z, y, w_pos=1.0):
    """dL/dz for the mean loss above."""
    p = sigmoid(z)
    y = np.asarray(y, dtype=np.float64)
    return (w_pos * y * (p - 1.0) + (1.0 - y) * p) / len(p)


def backward(theta, cache, dz, d, H, bf16=False):
    """Gradient of the loss with respect to the flat parameters, given
    dL/dz for every sample."""
    rnd = round_bf16 if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    dz = np.asarray(dz, dtype=np.float64)
    h1, h2, z1, z2 = cache["h1"], cache["h2"], cache["z1"], cache["z2"]
    g_w3 = h2.T @ dz
    g_b3 = np.array([dz.sum()])
    dz2 = rnd(np.outer(dz, cache["w3"]) * (z2 > 0))
    g_W2 = dz2.T @ h1
    g_b2 = dz2.sum(axis=0)
    dz1 = rnd((dz2 @ cache["W2"]) * (z1 > 0))
    g_W1 = dz1.T @ cache["F"]
    g_b1 = dz1.sum(axis=0)
    return pack(g_W1, g_b1, g_W2, g_b2, g_w3, g_b3)


def adam_step(theta, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def keep_count(n: int, permille: int) -> int:
    """ceil(n * permille / 1000) in integers, at least 1 when n > 0."""
    if n == 0:
        return 0
    return max(1, (n * permille + 999) // 1000)


def keep_top_fraction(scores, permille):
    """Indices of the keep_count(n, permille) highest scores together with
    every score equal to the lowest one kept (ties are all kept)."""
    scores = np.asarray(scores)
    n = len(scores)
    if n == 0:
        return np.zeros(0, dtype=np.int64)
    m = keep_count(n, permille)
    thr = np.sort(scores)[::-1][m - 1]
    return np.nonzero(scores >= thr)[0]
