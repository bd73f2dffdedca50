"""Pins for the oracle's TransE-L1 scorer (the paper's own edge score,
section 3.3: gamma minus the L1 distance between head plus relation and
tail, gamma = 1.0 in the paper).  Each check is fixed by the definition and
by arithmetic, not by the oracle itself:

* a hand-worked example with integer embeddings (tests/golden/
  transe_handworked.json): every distance and score is an exact integer,
  worked out by hand, including a tie broken by the ids and a self-loop;
  the same example with gamma = 2.5 shifts every score by 3 * 1.5;
* edge weights equal gamma - |h + r - t|_1 at single points where the value
  is known exactly (dyadic operands);
* translating every entity embedding by one vector leaves every weight,
  hence every ranking and score, unchanged (exact with dyadic operands);
* direction: reversing an edge and negating the relation gives the same
  distance, while the hand-worked graph's asymmetric weights pin which
  operand is the head;
* K = 1 equals a (max, +) matrix product over max_r w(u, r, v);
* path counts do not depend on the scorer; C and pure-Python oracles agree.
"""

import json
import os

import numpy as np
import pytest

import kgsynth
import oracle
from oracle import pyoracle

GOLD = os.path.join(os.path.dirname(__file__), "golden", "transe_handworked.json")


def _gold():
    with open(GOLD) as f:
        return json.load(f)


@pytest.mark.parametrize("gamma", [1.0, 2.5])
def test_handworked_transe_c_oracle(oracle_lib, gamma):
    j = _gold()
    e = np.array(j["edges"], dtype=np.uint32)
    g = oracle_lib.Graph(j["n"], j["R"], e[:, 0], e[:, 1], e[:, 2])
    X = np.array(j["X"], np.float32)
    Y = np.array(j["Y"], np.float32)
    for q in j["queries"]:
        out, cnt, tot = g.topk(X, Y, [q["s"]], [q["t"]], 16, scorer="transe_l1", gamma=gamma)
        assert int(tot[0]) == q["total"] and int(cnt[0]) == len(q["paths"])
        for got, exp in zip(out[0][:cnt[0]], q["paths"]):
            assert (got["a"], got["b"], got["r1"], got["r2"], got["r3"]) == \
                (exp["a"], exp["b"], exp["r1"], exp["r2"], exp["r3"])
            assert got["s"] == 3 * gamma - sum(exp["l1"])


@pytest.mark.parametrize("gamma", [1.0, 2.5])
def test_handworked_transe_py_oracle(gamma):
    j = _gold()
    for q in j["queries"]:
        paths, total = pyoracle.topk_paths(j["edges"], j["X"], j["Y"], q["s"], q["t"], 16,
                                           scorer="transe_l1", gamma=gamma)
        assert total == q["total"]
        assert [p[1:] for p in paths] == [(e["a"], e["b"], e["r1"], e["r2"], e["r3"]) for e in q["paths"]]
        assert [p[0] for p in paths] == [3 * gamma - sum(e["l1"]) for e in q["paths"]]


def test_edge_weight_points(oracle_lib):
    """Single edges with dyadic operands: the distance is exact."""
    X = np.array([[0.5, -1.25, 3.0, 0.0], [2.0, 0.75, -0.5, 1.0]], np.float32)
    Y = np.array([[1.5, 0.25, -2.5, 0.125]], np.float32)
    g = oracle_lib.Graph(2, 1, np.array([0], np.uint32), np.array([0], np.uint32), np.array([1], np.uint32))
    x, w = g.edge_weights(X, Y, [0, 1, 0], [0, 0, 0], [1, 0, 0], scorer="transe_l1", gamma=1.0)
    # (0.5+1.5-2, -1.25+0.25-0.75, 3-2.5+0.5, 0+0.125-1) = (0, -1.75, 1, -0.875)
    assert x[0] == 3.625 and w[0] == 1.0 - 3.625
    # (2+1.5-0.5, 0.75+0.25+1.25, -0.5-2.5-3, 1+0.125-0) = (3, 2.25, -6, 1.125)
    assert x[1] == 12.375 and w[1] == -11.375
    # a self-loop: the distance is |r|_1
    assert x[2] == 1.5 + 0.25 + 2.5 + 0.125
    # the DistMult scorer is unchanged by the option
    xd, _ = g.edge_weights(X, Y, [0], [0], [1])
    assert xd[0] == 0.5 * 1.5 * 2.0 + (-1.25) * 0.25 * 0.75 + 3.0 * (-2.5) * (-0.5) + 0.0
    with pytest.raises(ValueError):
        g.edge_weights(X, Y, [0], [0], [1], scorer="nope")


def _dyadic_case(seed, n=48, R=3, d=8, m=700):
    """A dense uniform graph with embeddings on the grid 2^-6 in [-2, 2]:
    every sum and difference below is exact in FP64."""
    h, r, t = kgsynth.uniform_graph(n, R, m, seed)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    X = (rng.integers(-128, 129, (n, d)) / 64.0).astype(np.float32)
    Y = (rng.integers(-128, 129, (R, d)) / 64.0).astype(np.float32)
    s = rng.integers(0, n, 24).astype(np.uint32)
    tt = rng.integers(0, n, 24).astype(np.uint32)
    return n, R, (h, r, t), X, Y, s, tt


def test_translation_invariance(oracle_lib):
    n, R, (h, r, t), X, Y, s, tt = _dyadic_case(5)
    g = oracle_lib.Graph(n, R, h, r, t)
    c = (np.arange(X.shape[1]) / 8.0 - 0.5).astype(np.float32)
    a = g.topk(X, Y, s, tt, 20, scorer="transe_l1")
    b = g.topk(X + c, Y, s, tt, 20, scorer="transe_l1")
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
    # not a property of DistMult: the scores move
    ad = g.topk(X, Y, s, tt, 20)
    bd = g.topk(X + c, Y, s, tt, 20)
    assert not np.array_equal(ad[0]["s"], bd[0]["s"])


def test_reversed_edge_with_negated_relation(oracle_lib):
    n, R, (h, r, t), X, Y, s, tt = _dyadic_case(6)
    g = oracle_lib.Graph(n, R, h, r, t)
    x1, w1 = g.edge_weights(X, Y, h, r, t, scorer="transe_l1")
    x2, w2 = g.edge_weights(X, -Y, t, r, h, scorer="transe_l1")
    assert np.array_equal(x1, x2)
    x3, _ = g.edge_weights(X, Y, t, r, h, scorer="transe_l1")
    assert not np.array_equal(x1, x3)   # the weight is directed


def test_top1_equals_maxplus_product_transe(oracle_lib):
    n, R, (h, r, t), X, Y, s, tt = _dyadic_case(7)
    g = oracle_lib.Graph(n, R, h, r, t)
    E = np.unique(np.stack([h, r, t], 1).astype(np.int64), axis=0)
    w = 1.0 - np.abs(X[E[:, 0]].astype(np.float64) + Y[E[:, 1]] - X[E[:, 2]]).sum(1)
    W = np.full((n, n), -np.inf)
    np.maximum.at(W, (E[:, 0], E[:, 2]), w)
    out, cnt, tot = g.topk(X, Y, s, tt, 1, scorer="transe_l1")
    for q in range(len(s)):
        best = np.max(W[s[q]][:, None] + W + W[:, tt[q]][None, :])
        if tot[q] == 0:
            assert not np.isfinite(best)
        else:
            assert out[q][0]["s"] == best   # integer-grid values: exact


@pytest.mark.parametrize("name,nq", [("dense_tiny", 12), ("hub_tiny", 16)])
def test_c_equals_python_and_counts_independent_of_scorer(oracle_lib, name, nq):
    cfg = kgsynth.CONFIGS[name]
    h, r, t = kgsynth.make_graph(cfg.graph)
    X, Y = kgsynth.embeddings(cfg.graph.n, cfg.graph.R, cfg.emb)
    s, d, k = kgsynth.queries(h, cfg.graph.n, cfg.query)
    g = oracle_lib.Graph(cfg.graph.n, cfg.graph.R, h, r, t)
    K = int(k[0])
    out, cnt, tot = g.topk(X, Y, s[:nq], d[:nq], K, scorer="transe_l1")
    _, _, tot_d = g.topk(X, Y, s[:nq], d[:nq], K)
    assert np.array_equal(tot, tot_d)
    edges = list(zip(h.tolist(), r.tolist(), t.tolist()))
    Xl, Yl = X.tolist(), Y.tolist()
    for q in range(nq):
        paths, total = pyoracle.topk_paths(edges, Xl, Yl, int(s[q]), int(d[q]), K, scorer="transe_l1")
        assert total == int(tot[q])
        got = out[q][:cnt[q]]
        assert [p[1:] for p in paths] == list(zip(got["a"].tolist(), got["b"].tolist(), got["r1"].tolist(),
                                                    got["r2"].tolist(), got["r3"].tolist()))
        assert np.allclose([p[0] for p in paths], got["s"], rtol=0, atol=1e-13)
