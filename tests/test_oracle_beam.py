"""Pins for the oracle's generic multi-hop search (section 5: level-by-level
expansion with cycle exclusion, target-reaching paths recorded as found,
the best K children of each parent passed on):

* a hand-worked example on the TransE-L1 example graph (integer scores)
  for K = 1, 2, 3 and a K that keeps every child;
* with K at least the largest branching the beam prunes nothing, so the
  result is the best K of all simple paths of at most H edges, enumerated
  here by an independent depth-first search;
* H = 1 returns the direct edges s -> t ranked by weight;
* the best score found never drops as K grows (a wider beam explores a
  superset);
* the C and pure-Python oracles agree.
"""

import json
import os

import numpy as np
import pytest

import kgsynth
import oracle
from oracle import pyoracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _graph():
    j = json.load(open(os.path.join(GOLD, "transe_handworked.json")))
    e = np.array(j["edges"], dtype=np.uint32)
    return j, e, np.array(j["X"], np.float32), np.array(j["Y"], np.float32)


def _rows(out, cnt):
    p = out[:cnt]
    return [(float(x["s"]), tuple(int(v) for v in x["v"][:x["len"]]), tuple(int(r) for r in x["r"][:x["len"]]))
            for x in p]


def test_handworked_beam(oracle_lib):
    j, e, X, Y = _graph()
    case = json.load(open(os.path.join(GOLD, "beam_handworked.json")))
    g = oracle_lib.Graph(j["n"], j["R"], e[:, 0], e[:, 1], e[:, 2])
    for c in case["cases"]:
        out, cnt, rec = g.beam(X, Y, [case["s"]], [case["t"]], case["H"], c["K"], scorer="transe_l1")
        exp = [(float(p["score"]), tuple(p["v"]), tuple(p["r"])) for p in c["paths"]]
        assert _rows(out[0], cnt[0]) == exp, c["K"]
        assert int(rec[0]) == c["recorded"]
        py, nrec = pyoracle.beam_paths(j["edges"], j["X"], j["Y"], case["s"], case["t"], case["H"], c["K"],
                                       scorer="transe_l1")
        assert py == exp and nrec == c["recorded"]


def _dyadic(seed, n=40, R=3, m=400, d=8):
    h, r, t = kgsynth.uniform_graph(n, R, m, seed)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    X = (rng.integers(-64, 65, (n, d)) / 32.0).astype(np.float32)
    Y = (rng.integers(-64, 65, (R, d)) / 32.0).astype(np.float32)
    return n, R, (h, r, t), X, Y, rng


def _all_simple_paths(n, h, r, t, X, Y, s, tt, H):
    """Every simple path s -> tt of at most H edges (depth-first search over
    the distinct triples), with the score summed along it."""
    E = sorted(set(zip(h.tolist(), r.tolist(), t.tolist())))
    adj = {}
    for (u, rr, v) in E:
        adj.setdefault(u, []).append((v, rr))
    w = lambda u, rr, v: 1.0 - float(np.abs(X[u].astype(np.float64) + Y[rr] - X[v]).sum())
    out = []

    def dfs(u, score, vs, rs):
        if len(vs) == H:
            return
        for (v, rr) in adj.get(u, []):
            if v == s or v in vs:
                continue
            sc = score + w(u, rr, v)
            if v == tt:
                out.append((sc, vs + (v,), rs + (rr,)))
            else:
                dfs(v, sc, vs + (v,), rs + (rr,))
    dfs(s, 0.0, (), ())
    out.sort(key=lambda p: (-p[0], list(p[1]), list(p[2])))
    return out


@pytest.mark.parametrize("H", [2, 3, 4])
def test_wide_beam_equals_all_simple_paths(oracle_lib, H):
    n, R, (h, r, t), X, Y, rng = _dyadic(11 + H, n=24, m=150)
    g = oracle_lib.Graph(n, R, h, r, t)
    outdeg = np.bincount(h, minlength=n)
    Kwide = int(outdeg.max()) * R + 1
    src = rng.integers(0, n, 6).astype(np.uint32)
    dst = rng.integers(0, n, 6).astype(np.uint32)
    out, cnt, rec = g.beam(X, Y, src, dst, H, Kwide, scorer="transe_l1")
    for q in range(6):
        allp = _all_simple_paths(n, h, r, t, X, Y, int(src[q]), int(dst[q]), H)
        assert int(rec[q]) == len(allp)
        assert _rows(out[q], cnt[q]) == allp[:Kwide]


def test_one_hop_is_the_direct_edges(oracle_lib):
    n, R, (h, r, t), X, Y, rng = _dyadic(21)
    g = oracle_lib.Graph(n, R, h, r, t)
    E = sorted(set(zip(h.tolist(), r.tolist(), t.tolist())))
    for (s, tt) in [(E[0][0], E[0][2]), (E[5][0], E[5][2])]:
        out, cnt, _ = g.beam(X, Y, [s], [tt], 1, 8, scorer="transe_l1")
        direct = sorted([(1.0 - float(np.abs(X[s].astype(np.float64) + Y[rr] - X[tt]).sum()), (tt,), (rr,))
                         for (u, rr, v) in E if u == s and v == tt], key=lambda p: (-p[0], list(p[2])))
        assert _rows(out[0], cnt[0]) == direct


def test_best_score_monotone_in_k(oracle_lib):
    n, R, (h, r, t), X, Y, rng = _dyadic(31, n=60, m=900)
    g = oracle_lib.Graph(n, R, h, r, t)
    src = rng.integers(0, n, 10).astype(np.uint32)
    dst = rng.integers(0, n, 10).astype(np.uint32)
    prev = None
    for K in (1, 2, 4, 8, 16):
        out, cnt, _ = g.beam(X, Y, src, dst, 3, K, scorer="transe_l1")
        best = np.where(cnt > 0, out["s"][:, 0], -np.inf)
        if prev is not None:
            assert np.all(best >= prev)
        prev = best


@pytest.mark.parametrize("scorer", ["distmult", "transe_l1"])
def test_c_beam_equals_python(oracle_lib, scorer):
    cfg = kgsynth.CONFIGS["dense_tiny"]
    h, r, t = kgsynth.make_graph(cfg.graph)
    X, Y = kgsynth.embeddings(cfg.graph.n, cfg.graph.R, cfg.emb)
    s, d, _ = kgsynth.queries(h, cfg.graph.n, cfg.query)
    g = oracle_lib.Graph(cfg.graph.n, cfg.graph.R, h, r, t)
    edges = list(zip(h.tolist(), r.tolist(), t.tolist()))
    for H, K in ((2, 3), (3, 4)):
        out, cnt, rec = g.beam(X, Y, s[:8], d[:8], H, K, scorer=scorer)
        for q in range(8):
            py, nrec = pyoracle.beam_paths(edges, X.tolist(), Y.tolist(), int(s[q]), int(d[q]), H, K, scorer=scorer)
            got = _rows(out[q], cnt[q])
            assert [p[1:] for p in got] == [p[1:] for p in py] and nrec == int(rec[q])
            assert np.allclose([p[0] for p in got], [p[0] for p in py], rtol=0, atol=1e-14)
