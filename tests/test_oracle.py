"""Pins for the CPU oracle: each check is fixed by the paper's problem
statement and by mathematics, not by the oracle itself.

* closed forms of the log-sigmoid, evaluated independently in 60-digit
  decimal arithmetic;
* a hand-worked example (tests/golden/handworked_d2.json);
* the path count |P(s,t)| = (A^3)[s,t] with A the relation-multiplicity
  matrix, computed by scipy.sparse;
* the sum-of-degree-products identity over all targets;
* all-zero embeddings: every score is -3 ln 2 and the ranking is the plain
  lexicographic order of the paths, enumerated independently with numpy;
* K = 1 against a (max, +) matrix product with weights computed by numpy;
* K-monotonicity, transposed-graph symmetry, relabelling and edge-order /
  duplicate invariance;
* the C oracle and the pure-Python oracle agree.
"""

import decimal
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

import kgsynth
import oracle
from oracle import pyoracle

GOLD = os.path.join(os.path.dirname(__file__), "golden", "handworked_d2.json")
LN2 = 0.6931471805599453


def dec_logsigmoid(x) -> float:
    """-ln(1 + e^(-x)) in 60-digit decimal arithmetic."""
    with decimal.localcontext() as ctx:
        ctx.prec = 60
        X = decimal.Decimal(x)
        return float(-(1 + (-X).exp()).ln())


def small_graph(name):
    cfg = kgsynth.CONFIGS[name]
    h, r, t = kgsynth.make_graph(cfg.graph)
    X, Y = kgsynth.embeddings(cfg.graph.n, cfg.graph.R, cfg.emb)
    s, d, k = kgsynth.queries(h, cfg.graph.n, cfg.query)
    return cfg, (h, r, t), oracle.as_f32_table(X, cfg.emb.dtype), oracle.as_f32_table(Y, cfg.emb.dtype), (s, d, k)


def multiplicity(n, h, r, t):
    keys = np.unique((h.astype(np.int64) * n + t) * 64 + r)
    uv = keys // 64
    return sp.csr_matrix((np.ones(len(uv)), (uv // n, uv % n)), shape=(n, n))


@pytest.mark.parametrize("x", [0.0, 1.0, -1.0, 2.0, -2.0, 0.5, -0.5, 1e-3, -1e-3, 10.0, -10.0, 40.0, -40.0])
def test_logsigmoid_closed_forms(oracle_lib, x):
    ref = dec_logsigmoid(x)
    for f in (oracle_lib.logsigmoid, pyoracle.logsigmoid):
        got = f(x)
        assert abs(got - ref) <= 4e-16 * max(1.0, abs(ref)), (x, got, ref)


def test_logsigmoid_printed_constants(oracle_lib):
    # logsigmoid(0) = -ln 2 and the integer values used by the hand-worked fixture
    assert oracle_lib.logsigmoid(0.0) == -LN2
    assert abs(oracle_lib.logsigmoid(1.0) - (-0.31326168751822286)) < 1e-16
    assert abs(oracle_lib.logsigmoid(-1.0) - (-1.3132616875182228)) < 1e-15
    assert abs(oracle_lib.logsigmoid(2.0) - (-0.1269280110429725)) < 1e-16
    assert abs(oracle_lib.logsigmoid(-2.0) - (-2.1269280110429727)) < 1e-15


def _gold():
    with open(GOLD) as f:
        return json.load(f)


def test_handworked_fixture_c_oracle(oracle_lib):
    j = _gold()
    e = np.array(j["edges"], dtype=np.uint32)
    g = oracle_lib.Graph(j["n"], j["R"], e[:, 0], e[:, 1], e[:, 2])
    X = np.array(j["X"], np.float32)
    Y = np.array(j["Y"], np.float32)
    for q in j["queries"]:
        out, cnt, tot = g.topk(X, Y, [q["s"]], [q["t"]], 16)
        assert int(tot[0]) == q["total"]
        assert int(cnt[0]) == len(q["paths"])
        for got, exp in zip(out[0][:cnt[0]], q["paths"]):
            assert (got["a"], got["b"], got["r1"], got["r2"], got["r3"]) == \
                (exp["a"], exp["b"], exp["r1"], exp["r2"], exp["r3"])
            ref = sum(dec_logsigmoid(x) for x in exp["x"])
            assert abs(got["s"] - ref) < 1e-14


def test_handworked_fixture_py_oracle():
    j = _gold()
    for q in j["queries"]:
        paths, total = pyoracle.topk_paths(j["edges"], j["X"], j["Y"], q["s"], q["t"], 16)
        assert total == q["total"]
        assert [p[1:] for p in paths] == [(e["a"], e["b"], e["r1"], e["r2"], e["r3"]) for e in q["paths"]]
        for p, e in zip(paths, q["paths"]):
            assert abs(p[0] - sum(dec_logsigmoid(x) for x in e["x"])) < 1e-14


def test_fsum_is_correctly_rounded(oracle_lib):
    """The path-score sum against Python's math.fsum (an independent
    correctly rounded summation) on adversarial and random triples."""
    rng = np.random.Generator(np.random.PCG64(8))
    cases = [(1.0, 1e-16, 1e-16), (1e16, 1.0, -1e16), (-0.6931471805599453,) * 3,
             (1.0, 2.0 ** -53, 2.0 ** -106), (0.1, 0.2, 0.3), (-1e-300, 1e-300, 5e-324)]
    cases += [tuple(rng.standard_normal(3) * 10.0 ** rng.integers(-20, 20, 3)) for _ in range(2000)]
    cases += [tuple(-0.69 + rng.standard_normal(3) * 1e-3) for _ in range(2000)]
    for c in cases:
        assert oracle_lib.fsum(c) == math.fsum(c), c
        # a function of the multiset only
        assert oracle_lib.fsum(c[::-1]) == oracle_lib.fsum(c) == oracle_lib.fsum((c[1], c[2], c[0]))


def test_permuted_weights_tie(oracle_lib):
    """When a = t, DistMult symmetry makes the paths (r2, r3) = (x, y) and
    (y, x) through the same b carry the same three weights in another
    order: their scores are equal and the ids break the tie."""
    n, R, d = 6, 2, 8
    rng = np.random.Generator(np.random.PCG64(12))
    X = rng.standard_normal((n, d)).astype(np.float32)
    Y = rng.standard_normal((R, d)).astype(np.float32)
    s, t, b = 0, 3, 4
    edges = [(s, 0, t), (t, 0, b), (t, 1, b), (b, 0, t), (b, 1, t)]
    h = np.array([e[0] for e in edges], np.uint32)
    r = np.array([e[1] for e in edges], np.uint32)
    tt = np.array([e[2] for e in edges], np.uint32)
    g = oracle_lib.Graph(n, R, h, r, tt)
    out, cnt, tot = g.topk(X, Y, [s], [t], 8)
    got = out[0][:cnt[0]]
    key = {(p["r2"], p["r3"]): p["s"] for p in got}
    assert key[(0, 1)] == key[(1, 0)]
    i01 = [i for i, p in enumerate(got) if (p["r2"], p["r3"]) == (0, 1)][0]
    i10 = [i for i, p in enumerate(got) if (p["r2"], p["r3"]) == (1, 0)][0]
    assert i01 < i10
    paths, _ = pyoracle.topk_paths(edges, X.tolist(), Y.tolist(), s, t, 8)
    assert [p[1:] for p in paths] == list(zip(got["a"].tolist(), got["b"].tolist(), got["r1"].tolist(),
                                               got["r2"].tolist(), got["r3"].tolist()))


@pytest.mark.parametrize("name", ["tiny", "dense_tiny", "hub_tiny"])
def test_count_equals_adjacency_cube(oracle_lib, name):
    cfg, (h, r, t), X, Y, (s, d, k) = small_graph(name)
    n = cfg.graph.n
    g = oracle_lib.Graph(n, cfg.graph.R, h, r, t)
    A = multiplicity(n, h, r, t)
    A3 = (A @ A @ A).tocsr()
    _, cnt, tot = g.topk(X, Y, s, d, 1)
    for q in range(len(s)):
        assert int(tot[q]) == int(round(A3[int(s[q]), int(d[q])]))
        assert int(cnt[q]) == min(1, int(tot[q]))


def test_sum_of_degree_products(oracle_lib):
    cfg, (h, r, t), X, Y, _ = small_graph("dense_tiny")
    n = cfg.graph.n
    g = oracle_lib.Graph(n, cfg.graph.R, h, r, t)
    rp, tail, rel = g.csr()
    outdeg = np.diff(rp).astype(np.int64)
    for s in (0, 7, 33):
        _, _, tot = g.topk(X, Y, np.full(n, s), np.arange(n), 1)
        expect = 0
        for e1 in range(int(rp[s]), int(rp[s + 1])):
            a = int(tail[e1])
            for e2 in range(int(rp[a]), int(rp[a + 1])):
                expect += int(outdeg[int(tail[e2])])
        assert int(tot.sum()) == expect


def _all_walks_numpy(n, h, r, t, s, tt):
    """Every walk s->a->b->tt as rows (a, b, r1, r2, r3), by numpy joins."""
    E = np.unique(np.stack([h, r, t], 1).astype(np.int64), axis=0)
    e1 = E[E[:, 0] == s]
    e3 = E[E[:, 2] == tt]
    rows = []
    for (_, r1, a) in e1:
        e2 = E[E[:, 0] == a]
        for (_, r2, b) in e2:
            for (bb, r3, _) in e3[e3[:, 0] == b]:
                rows.append((a, b, r1, r2, r3))
    return np.array(rows, dtype=np.int64).reshape(-1, 5)


def test_all_zero_embeddings_tie_break(oracle_lib):
    cfg, (h, r, t), X, Y, (s, d, k) = small_graph("dense_tiny")
    n = cfg.graph.n
    g = oracle_lib.Graph(n, cfg.graph.R, h, r, t)
    Z = np.zeros_like(X)
    ZY = np.zeros_like(Y)
    out, cnt, tot = g.topk(Z, ZY, s[:6], d[:6], 25)
    three = math.fsum([-LN2] * 3)
    for q in range(6):
        walks = _all_walks_numpy(n, h, r, t, int(s[q]), int(d[q]))
        assert len(walks) == int(tot[q])
        order = np.lexsort(walks.T[::-1])
        exp = walks[order][:25]
        got = out[q][:cnt[q]]
        assert np.all(got["s"] == three)
        assert np.array_equal(np.stack([got["a"], got["b"], got["r1"], got["r2"], got["r3"]], 1), exp)


def _np_weights(X, Y, u, r, v):
    x = np.einsum("ij,ij,ij->i", X[u].astype(np.float64), Y[r].astype(np.float64), X[v].astype(np.float64))
    return -np.logaddexp(0.0, -x)


def test_top1_equals_maxplus_product(oracle_lib):
    cfg, (h, r, t), X, Y, (s, d, k) = small_graph("dense_tiny")
    n = cfg.graph.n
    g = oracle_lib.Graph(n, cfg.graph.R, h, r, t)
    E = np.unique(np.stack([h, r, t], 1).astype(np.int64), axis=0)
    w = _np_weights(X, Y, E[:, 0], E[:, 1], E[:, 2])
    W = np.full((n, n), -np.inf)
    np.maximum.at(W, (E[:, 0], E[:, 2]), w)
    out, cnt, tot = g.topk(X, Y, s, d, 1)
    for q in range(len(s)):
        sq, tq = int(s[q]), int(d[q])
        best = np.max(W[sq][:, None] + W + W[:, tq][None, :])
        if tot[q] == 0:
            assert not np.isfinite(best)
        else:
            assert abs(out[q][0]["s"] - best) < 1e-12


def test_k_monotone_prefix(oracle_lib):
    cfg, (h, r, t), X, Y, (s, d, k) = small_graph("dense_tiny")
    g = oracle_lib.Graph(cfg.graph.n, cfg.graph.R, h, r, t)
    prev = None
    for K in (1, 2, 5, 10, 31, 32, 200):
        out, cnt, tot = g.topk(X, Y, s, d, K)
        assert np.array_equal(cnt, np.minimum(K, tot).astype(np.uint32))
        if prev is not None:
            pout, pcnt = prev
            for q in range(len(s)):
                assert np.array_equal(out[q][:pcnt[q]], pout[q][:pcnt[q]])
        prev = (out, cnt)


def test_transposed_graph_symmetry(oracle_lib):
    cfg, (h, r, t), X, Y, (s, d, k) = small_graph("dense_tiny")
    n = cfg.graph.n
    g = oracle_lib.Graph(n, cfg.graph.R, h, r, t)
    gt = oracle_lib.Graph(n, cfg.graph.R, t, r, h)
    K = 40
    out, cnt, tot = g.topk(X, Y, s, d, K)
    outt, cntt, tott = gt.topk(X, Y, d, s, K)
    assert np.array_equal(tot, tott)
    for q in range(len(s)):
        a = {(p["a"], p["b"], p["r1"], p["r2"], p["r3"]): p["s"] for p in out[q][:cnt[q]]}
        b = {(p["b"], p["a"], p["r3"], p["r2"], p["r1"]): p["s"] for p in outt[q][:cntt[q]]}
        if cnt[q] == tot[q]:
            assert a.keys() == b.keys()
        for key in a.keys() & b.keys():
            assert abs(a[key] - b[key]) <= 4e-16 * 3


def test_relabel_and_edge_order_invariance(oracle_lib):
    cfg, (h, r, t), X, Y, (s, d, k) = small_graph("hub_tiny")
    n = cfg.graph.n
    g = oracle_lib.Graph(n, cfg.graph.R, h, r, t)
    out, cnt, tot = g.topk(X, Y, s, d, 12)
    rng = np.random.Generator(np.random.PCG64(99))
    # shuffled edge order plus duplicated triples
    perm = rng.permutation(len(h))
    dup = rng.integers(0, len(h), 500)
    h2 = np.concatenate([h[perm], h[dup]]); r2 = np.concatenate([r[perm], r[dup]])
    t2 = np.concatenate([t[perm], t[dup]])
    g2 = oracle_lib.Graph(n, cfg.graph.R, h2, r2, t2)
    o2, c2, tt2 = g2.topk(X, Y, s, d, 12)
    assert np.array_equal(out, o2) and np.array_equal(cnt, c2) and np.array_equal(tot, tt2)
    # vertex relabelling pi: scores map exactly, ids map by pi (no exact ties here)
    pi = rng.permutation(n).astype(np.uint32)
    Xp = np.empty_like(X); Xp[pi] = X
    g3 = oracle_lib.Graph(n, cfg.graph.R, pi[h], r, pi[t])
    o3, c3, t3 = g3.topk(Xp, Y, pi[s], pi[d], 12)
    assert np.array_equal(tot, t3)
    for q in range(len(s)):
        ra = out[q][:cnt[q]]
        rb = o3[q][:c3[q]]
        assert np.array_equal(ra["s"], rb["s"])
        assert np.array_equal(pi[ra["a"]], rb["a"]) and np.array_equal(pi[ra["b"]], rb["b"])


@pytest.mark.parametrize("name,nq", [("tiny", 64), ("dense_tiny", 12), ("hub_tiny", 16)])
def test_c_oracle_equals_python_oracle(oracle_lib, name, nq):
    cfg, (h, r, t), X, Y, (s, d, k) = small_graph(name)
    g = oracle_lib.Graph(cfg.graph.n, cfg.graph.R, h, r, t)
    K = int(k[0])
    out, cnt, tot = g.topk(X, Y, s[:nq], d[:nq], K)
    edges = list(zip(h.tolist(), r.tolist(), t.tolist()))
    Xl, Yl = X.tolist(), Y.tolist()
    for q in range(nq):
        paths, total = pyoracle.topk_paths(edges, Xl, Yl, int(s[q]), int(d[q]), K)
        assert total == int(tot[q])
        got = out[q][:cnt[q]]
        assert [p[1:] for p in paths] == list(zip(got["a"].tolist(), got["b"].tolist(), got["r1"].tolist(),
                                                    got["r2"].tolist(), got["r3"].tolist()))
        assert np.allclose([p[0] for p in paths], got["s"], rtol=0, atol=1e-15)


def test_truncation_is_exercised(oracle_lib):
    """The test-only graphs must actually truncate at K (the tiny config
    averages well under one path per query)."""
    for name in ("dense_tiny", "hub_tiny"):
        cfg, (h, r, t), X, Y, (s, d, k) = small_graph(name)
        g = oracle_lib.Graph(cfg.graph.n, cfg.graph.R, h, r, t)
        _, cnt, tot = g.topk(X, Y, s, d, k)
        assert (tot > k).sum() >= len(s) // 4


def test_bad_arguments(oracle_lib):
    with pytest.raises(ValueError):
        oracle_lib.Graph(4, 1, np.array([0, 5], np.uint32), np.array([0, 0], np.uint32), np.array([1, 2], np.uint32))
    g = oracle_lib.Graph(4, 1, np.array([0, 1], np.uint32), np.array([0, 0], np.uint32), np.array([1, 2], np.uint32))
    X = np.zeros((4, 8), np.float32); Y = np.zeros((1, 8), np.float32)
    with pytest.raises(ValueError):
        g.topk(X, Y, [0], [9], 1)
    with pytest.raises(ValueError):
        g.topk(X, Y, [0], [1], 0)
