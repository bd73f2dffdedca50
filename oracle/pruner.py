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


# ---------------------------------------------------------------------------
# Element-wise error bounds for a computation that follows the formulas above
# with bfloat16-rounded operands and FP32 accumulation in any order (as the
# GPU kernels do).  Each quantity travels with a bound e on |x_gpu - x|,
# where x is the FP64 value of forward / backward with bf16=True:
#   product C = A B (inner length k), |A' - A| <= eA, |B' - B| <= eB:
#     |C' - C| <= |A| eB + eA |B| + eA eB + gamma_k (|A| + eA)(|B| + eB)
#     (gamma_k = k u / (1 - k u), u = 2^-24, bounds any summation order)
#   bfloat16 rounding to nearest of x' vs of x: rounding is monotone, so
#     rnd(x') lies between rnd(x - e) and rnd(x + e)
#   relu is 1-Lipschitz; a 0/1 mask (x > 0) is certain only where |x| > e,
#   elsewhere the masked value may be kept or dropped.
#   exact sums: where both operands are known exactly and every term
#     A_ij B_jk (and the added bias) is a multiple of one power of two q
#     with sum |terms| < 2^24 q, every partial sum in any order is a
#     multiple of q below 2^24 q in magnitude, hence an FP32 number: the
#     product is computed without rounding and its bound is zero.
# ---------------------------------------------------------------------------

U32 = 2.0 ** -24


def gamma(k):
    return k * U32 / (1.0 - k * U32)


def quantum(x):
    """Largest power of two dividing each element of x (float64 holding
    FP32 values); +inf for zeros."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)
    M = np.abs(m * 2.0 ** 53).astype(np.int64)
    low = (M & -M).astype(np.float64)
    with np.errstate(divide="ignore"):
        q = np.ldexp(low, e - 53)
    return np.where(x == 0, np.inf, q)


def _exact_mask(A, eA, B, eB, S, bias=None):
    """True where the product element (i, k) is provably exact: row i of A
    and column k of B (and the bias) are exact and S_ik < 2^24 q_ik, S the
    sum of the terms' magnitudes and q_ik the smallest quantum among the
    terms, bounded below by qA_i qB_k (q the smallest quantum of the row /
    column) and the bias's own quantum."""
    qa = quantum(A).min(axis=1)
    qb = quantum(B).min(axis=0)
    exact_rows = ~np.any(eA != 0, axis=1)
    exact_cols = ~np.any(eB != 0, axis=0)
    with np.errstate(invalid="ignore", over="ignore"):
        q = np.outer(qa, qb)
        if bias is not None:
            q = np.minimum(q, quantum(bias)[None, :])
        ok = (S < 2.0 ** 24 * q) | (S == 0)
    return ok & exact_rows[:, None] & exact_cols[None, :]


def _prod_err(A, eA, B, eB, k, bias=None):
    """Bound on |C' - C| for C = A B (+ bias per column, exact), k terms
    per element in any order (one more with a bias)."""
    aA, aB = np.abs(A), np.abs(B)
    S = aA @ aB
    err = aA @ eB + eA @ aB + eA @ eB
    if bias is not None:
        bias = np.asarray(bias, dtype=np.float64).reshape(-1)
        err = err + gamma(k) * ((aA + eA) @ (aB + eB) + np.abs(bias)[None, :])
        S = S + np.abs(bias)[None, :]
    else:
        err = err + gamma(k) * ((aA + eA) @ (aB + eB))
    return np.where(_exact_mask(A, eA, B, eB, S, bias), 0.0, err)


def _rnd_err(x, e):
    """Bound on |rnd(x') - rnd(x)| for |x' - x| <= e: rounding to nearest is
    monotone, so rnd(x') lies between rnd(x - e) and rnd(x + e) (zero when
    no rounding boundary falls within the interval)."""
    r = round_bf16(x)
    return np.maximum(round_bf16(x + e) - r, r - round_bf16(x - e))


def forward_bounds(theta, F, d, H):
    """(z, bound on |z_gpu - z|, cache with per-quantity bounds) for the
    bfloat16-operand forward pass; FP32 parameters as held on the device
    (theta exactly representable in FP32)."""
    z, c = forward(theta, F, d, H, bf16=True)
    W1, b1, W2, b2, w3, b3 = unpack(theta, d, H)
    zero = lambda a: np.zeros_like(a)
    # the features and weights are rounded from exact inputs: no error
    e_z1 = _prod_err(c["F"], zero(c["F"]), c["W1"].T, zero(c["W1"].T), 4 * d + 1, bias=b1)
    e_h1 = _rnd_err(np.maximum(c["z1"], 0.0), e_z1)
    e_z2 = _prod_err(c["h1"], e_h1, c["W2"].T, zero(c["W2"].T), H + 1, bias=b2)
    e_h2 = _rnd_err(np.maximum(c["z2"], 0.0), e_z2)
    e_z = _prod_err(c["h2"], e_h2, c["w3"][:, None], zero(c["w3"][:, None]), H + 1, bias=b3)[:, 0]
    c.update(e_z1=e_z1, e_h1=e_h1, e_z2=e_z2, e_h2=e_h2)
    return z, e_z, c


def backward_bounds(theta, cache, z, e_z, y, w_pos, d, H):
    """(gradient, element-wise bound) for the bfloat16-operand backward
    pass from the logits' bounds e_z (BCE with sigmoid: dL/dz is 1/4-
    Lipschitz in z per sample, scaled by the weight and 1/N, plus the FP32
    evaluation's few roundings)."""
    N = len(z)
    g = backward(theta, cache, bce_grad(z, y, w_pos), d, H, bf16=True)
    dz = bce_grad(z, y, w_pos)
    wmax = np.where(np.asarray(y) > 0, w_pos, 1.0)
    e_dz = 0.25 * wmax * e_z / N + 8 * U32 * np.abs(dz) + 1e-45
    h1, h2, z1, z2 = cache["h1"], cache["h2"], cache["z1"], cache["z2"]
    e_h1, e_h2, e_z1, e_z2 = cache["e_h1"], cache["e_h2"], cache["e_z1"], cache["e_z2"]
    w3, W2, F = cache["w3"], cache["W2"], cache["F"]
    # output layer: g_w3 = h2^T dz, g_b3 = sum dz
    e_gw3 = _prod_err(h2.T, e_h2.T, dz[:, None], e_dz[:, None], N + 1)[:, 0]
    e_gb3 = np.array([e_dz.sum() + gamma(N) * np.abs(dz).sum()])
    # dz2 = bf16(dz w3^T * [z2 > 0])
    pre2 = np.outer(dz, w3)
    e_pre2 = np.outer(e_dz, np.abs(w3)) + gamma(1) * np.abs(pre2)
    m2 = z2 > 0
    unsure2 = (e_z2 > 0) & (np.abs(z2) <= e_z2)   # an exact z2 decides its mask
    dz2 = round_bf16(pre2 * m2)
    e_dz2 = np.where(unsure2, np.abs(pre2) + e_pre2, _rnd_err(pre2 * m2, e_pre2 * m2))
    e_gW2 = _prod_err(dz2.T, e_dz2.T, h1, e_h1, N + 1)
    e_gb2 = e_dz2.sum(0) + gamma(N) * np.abs(dz2).sum(0)
    # dz1 = bf16((dz2 W2) * [z1 > 0])
    pre1 = dz2 @ W2
    e_pre1 = _prod_err(dz2, e_dz2, W2, np.zeros_like(W2), H + 1)
    m1 = z1 > 0
    unsure1 = (e_z1 > 0) & (np.abs(z1) <= e_z1)
    dz1 = round_bf16(pre1 * m1)
    e_dz1 = np.where(unsure1, np.abs(pre1) + e_pre1, _rnd_err(pre1 * m1, e_pre1 * m1))
    e_gW1 = _prod_err(dz1.T, e_dz1.T, F, np.zeros_like(F), N + 1)
    e_gb1 = e_dz1.sum(0) + gamma(N) * np.abs(dz1).sum(0)
    return g, pack(e_gW1, e_gb1, e_gW2, e_gb2, e_gw3, e_gb3)


def adam_interval(theta, g, e_g, m, v, step, lr, beta1, beta2, eps):
    """Element-wise intervals (lo, hi) for the parameters, first and second
    moments after one Adam step evaluated in FP32 from exact FP32 state
    (theta, m, v, step) and constants, whose gradient lies within e_g of g.

    Every quantity is bounded by interval arithmetic: the moments are
    monotone in g (the second through g^2), and the step r = m_hat /
    (sqrt(v_hat) + eps) is increasing in m_hat and, for a fixed sign of
    m_hat, decreasing in |.| with v_hat.  FP32 evaluation is allowed a
    relative error of 4u per moment update, 8u per bias correction term
    1 - beta^t (pow within 4 ulp, then one subtraction, relative to the
    difference), 4u for the square root and eps, 4u for the step's
    products and quotient and u for the final subtraction (u = 2^-24)."""
    u = U32
    g = np.asarray(g, dtype=np.float64)
    glo, ghi = g - e_g, g + e_g
    m1lo = beta1 * m + (1 - beta1) * glo
    m1hi = beta1 * m + (1 - beta1) * ghi
    am = 4 * u * (np.abs(beta1 * m) + (1 - beta1) * np.maximum(np.abs(glo), np.abs(ghi)))
    m1lo, m1hi = m1lo - am, m1hi + am
    g2hi = np.maximum(glo * glo, ghi * ghi)
    g2lo = np.where((glo <= 0) & (ghi >= 0), 0.0, np.minimum(glo * glo, ghi * ghi))
    v1lo = beta2 * v + (1 - beta2) * g2lo
    v1hi = beta2 * v + (1 - beta2) * g2hi
    av = 4 * u * (np.abs(beta2 * v) + (1 - beta2) * g2hi)
    v1lo, v1hi = np.maximum(v1lo - av, 0.0), v1hi + av
    p1, p2 = beta1 ** step, beta2 ** step
    bc1, bc2 = 1 - p1, 1 - p2
    r1 = (8 * u * p1 + u) / bc1 + u      # relative error of the FP32 bias corrections
    r2 = (8 * u * p2 + u) / bc2 + u
    mh = np.stack([m1lo / (bc1 * (1 + r1)), m1lo / (bc1 * (1 - r1)),
                   m1hi / (bc1 * (1 + r1)), m1hi / (bc1 * (1 - r1))])
    mhlo, mhhi = mh.min(0), mh.max(0)
    dlo = np.sqrt(v1lo / (bc2 * (1 + r2))) * (1 - 4 * u) + eps * (1 - u)
    dhi = np.sqrt(v1hi / (bc2 * (1 - r2))) * (1 + 4 * u) + eps * (1 + u)
    rr = np.stack([mhlo / dlo, mhlo / dhi, mhhi / dlo, mhhi / dhi])
    rlo, rhi = rr.min(0), rr.max(0)
    rlo = rlo - 4 * u * np.abs(rlo)
    rhi = rhi + 4 * u * np.abs(rhi)
    tlo, thi = theta - lr * rhi, theta - lr * rlo
    at = u * np.maximum(np.abs(tlo), np.abs(thi))
    return (tlo - at, thi + at), (m1lo, m1hi), (v1lo, v1hi)
