"""Synthetic inputs: determinism, shape and the stated laws."""

import hashlib

import numpy as np

import kgsynth


def _digest(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def test_same_seed_same_arrays():
    for name in ("tiny", "dense_tiny", "hub_tiny"):
        cfg = kgsynth.CONFIGS[name]
        a = kgsynth.make_graph(cfg.graph)
        b = kgsynth.make_graph(cfg.graph)
        assert _digest(*a) == _digest(*b)
        Xa, Ya = kgsynth.embeddings(cfg.graph.n, cfg.graph.R, cfg.emb)
        Xb, Yb = kgsynth.embeddings(cfg.graph.n, cfg.graph.R, cfg.emb)
        assert _digest(Xa, Ya) == _digest(Xb, Yb)


def test_graph_laws():
    for name in ("tiny", "dense_tiny", "hub_tiny"):
        cfg = kgsynth.CONFIGS[name]
        h, r, t = kgsynth.make_graph(cfg.graph)
        assert len(h) == cfg.graph.m
        assert h.dtype == np.uint32 and r.dtype == np.uint32 and t.dtype == np.uint32
        assert h.max() < cfg.graph.n and t.max() < cfg.graph.n and r.max() < cfg.graph.R
        assert not np.any(h == t)
        key = (h.astype(np.int64) * cfg.graph.n + t) * cfg.graph.R + r
        assert len(np.unique(key)) == len(key)


def test_chung_lu_weights_solve():
    w, i0, C = kgsynth.chung_lu_weights(1_000_000, 20_000_000, 2.1, 1e5)
    assert abs(w.sum() - 2e7) / 2e7 < 1e-9
    assert abs(w[0] - 1e5) / 1e5 < 1e-9
    assert np.all(np.diff(w) < 0)


def test_chung_lu_is_heavy_tailed():
    cfg = kgsynth.CONFIGS["hub_tiny"]
    h, r, t = kgsynth.make_graph(cfg.graph)
    deg = np.bincount(h, minlength=cfg.graph.n)
    assert deg.max() > 20 * np.median(deg)


def test_embedding_law_and_bf16_rounding():
    spec = kgsynth.EmbSpec(64, "f32", seed=5)
    X, Y = kgsynth.embeddings(4000, 8, spec)
    assert X.shape == (4000, 64) and Y.shape == (8, 64) and X.dtype == np.float32
    assert abs(X.var() * 64 - 1.0) < 0.05
    bspec = kgsynth.EmbSpec(64, "bf16", seed=5)
    Xb, Yb = kgsynth.embeddings(4000, 8, bspec)
    assert Xb.dtype == np.uint16
    # round-to-nearest-even: the bf16 value is the nearest representable one
    back = kgsynth.bf16_bits_to_f32(Xb)
    err = np.abs(back.astype(np.float64) - X.astype(np.float64))
    ulp = np.abs(back).view(np.uint32) & 0x7F800000
    half_ulp = (ulp.view(np.float32).astype(np.float64)) * 2.0 ** -8
    assert np.all(err <= half_ulp * 1.0000001)
    # ties go to even
    tie = np.array([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8], np.float32)
    got = kgsynth.bf16_bits_to_f32(kgsynth.f32_to_bf16_bits(tie))
    assert got[0] == 1.0 and got[1] == 1.0 + 2 ** -6


def test_query_laws():
    cfg = kgsynth.CONFIGS["hub_tiny"]
    h, r, t = kgsynth.make_graph(cfg.graph)
    s, d, k = kgsynth.queries(h, cfg.graph.n, cfg.query)
    assert len(s) == cfg.query.nq and np.all(s != d) and np.all(k == cfg.query.k)
    deg = np.bincount(h, minlength=cfg.graph.n)
    assert np.all(deg[s] > 0)
    spec = kgsynth.QuerySpec(2000, "hubmix", 64, seed=4, k_choices=(1, 8, 64), hub_top=50)
    s, d, k = kgsynth.queries(h, cfg.graph.n, spec)
    assert set(np.unique(k).tolist()) == {1, 8, 64}
    hubs = np.lexsort((np.arange(cfg.graph.n), -deg))[:50]
    assert np.isin(s, hubs).mean() > 0.10
