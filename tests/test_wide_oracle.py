"""The oracle on wide-relation graphs (more than 32 relations, the scale
regime of the paper's WikiKG90Mv2 experiments, section 4.1), on the CPU:
pinned by a pure-Python brute force over all three-edge walks with
TransE-L1 weights and math.fsum path scores, and the per-query subgraph
that the full-size parity checks feed the oracle gives the same answers as
the whole graph."""

import math

import numpy as np

import kgsynth
import oracle


def _brute(h, r, t, X, Y, s, tq, K, gamma=1.0):
    """Every walk s -r1-> a -r2-> b -r3-> tq over the distinct triples, the
    TransE-L1 weight gamma - sum_i |x_u + y_r - x_v| of each edge in Python
    floats, the path score the correctly rounded sum of the three weights;
    sorted by score descending, then a, b, r1, r2, r3."""
    trip = sorted(set(zip(h.tolist(), r.tolist(), t.tolist())))
    out_e = {}
    for u, rr, v in trip:
        out_e.setdefault(u, []).append((rr, v))

    def w(u, rr, v):
        acc = 0.0
        for i in range(X.shape[1]):
            acc += abs((float(X[u, i]) + float(Y[rr, i])) - float(X[v, i]))
        return gamma - acc

    paths = []
    for r1, a in out_e.get(s, []):
        for r2, b in out_e.get(a, []):
            for r3, v in out_e.get(b, []):
                if v == tq:
                    paths.append((math.fsum([w(s, r1, a), w(a, r2, b), w(b, r3, tq)]), a, b, r1, r2, r3))
    paths.sort(key=lambda p: (-p[0], p[1], p[2], p[3], p[4], p[5]))
    return paths[:K], len(paths)


def test_oracle_matches_brute_force_on_a_wide_graph():
    sp = kgsynth.WIDE["wide_tiny"]
    h, r, t = kgsynth.wide_graph(sp)
    X, Y = kgsynth.wide_embeddings(sp)
    g = oracle.Graph(sp.n, sp.R, h, r, t)
    rng = np.random.Generator(np.random.PCG64(3))
    src = rng.integers(0, sp.n, 40).astype(np.uint32)
    dst = rng.integers(0, sp.n, 40).astype(np.uint32)
    K = 12
    paths, cnt, tot = g.topk(X, Y, src, dst, K, scorer="transe_l1", gamma=1.0)
    nonempty = 0
    for q in range(len(src)):
        exp, n = _brute(h, r, t, X, Y, int(src[q]), int(dst[q]), K)
        assert int(tot[q]) == n and int(cnt[q]) == len(exp)
        got = [(float(p["s"]), int(p["a"]), int(p["b"]), int(p["r1"]), int(p["r2"]), int(p["r3"]))
               for p in paths[q][:cnt[q]]]
        assert got == exp
        nonempty += n > 0
    assert nonempty >= 10
    assert int(r.max()) >= 32   # relation ids past one 32-bit mask


def test_query_subgraph_gives_the_full_graph_answer():
    sp = kgsynth.WIDE["wide_small"]
    h, r, t = kgsynth.wide_graph(sp)
    X, Y = kgsynth.wide_embeddings(sp)
    src, dst = kgsynth.wide_queries(h, t, 12, seed=5)
    full = oracle.Graph(sp.n, sp.R, h, r, t).topk(X, Y, src, dst, 32, scorer="transe_l1")
    for q in range(len(src)):
        sh, sr, st = kgsynth.wide_subgraph(h, r, t, int(src[q]), int(dst[q]))
        sub = oracle.Graph(sp.n, sp.R, sh, sr, st).topk(X, Y, src[q:q + 1], dst[q:q + 1], 32, scorer="transe_l1")
        assert int(sub[2][0]) == int(full[2][q]) and int(sub[1][0]) == int(full[1][q])
        assert np.array_equal(sub[0][0][:sub[1][0]], full[0][q][:full[1][q]])
    assert int(full[2].sum()) > 0
