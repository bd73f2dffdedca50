"""GPU parity of the TransE-L1 scorer (the paper's own edge score, section
3.3: gamma minus the L1 distance of head plus relation from tail) against
the FP64 oracle: the hand-worked integer example, the test workloads in
FP32 and bfloat16 storage, both search directions with hash and directory
probes, K from 1 to 200, a wide band, the exhaustive pass on all-equal scores, single edge
weights with their bounds, and a full-size sample of the realistic graph."""

import json
import os

import numpy as np
import pytest

import kgsynth
import oracle
from tests.parity import assert_same_result, compare, gpu_graph, run_gpu, run_oracle, say, workload

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "transe_handworked.json")
TE = "transe_l1"


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2406_07727_amd  # noqa: F401
    oracle.build(force=False)


def _small(name, k=None, nq=None, opts=None, zero=False, gamma=1.0):
    cfg, (h, r, t), (X, Y), (s, d, kk) = workload(name)
    if nq:
        s, d, kk = s[:nq], d[:nq], kk[:nq]
    if k is not None:
        kk = np.full(len(s), k, np.uint32)
    if zero:
        X = np.zeros_like(X)
        Y = np.zeros_like(Y)
    n, R = cfg.graph.n, cfg.graph.R
    say(f"case transe {name} nq={len(s)} k={int(kk.max())} zero={zero} gamma={gamma}")
    g = gpu_graph(n, R, h, r, t, X, Y, cfg.emb.dtype, scorer=TE, gamma=gamma)
    gpu = run_gpu(g, s, d, kk, k_max=int(kk.max()), opts=opts)
    orc = run_oracle(n, R, h, r, t, X, Y, s, d, kk, cfg.emb.dtype, scorer=TE, gamma=gamma)
    return gpu, orc


@pytest.mark.parametrize("gamma", [1.0, 2.5])
def test_handworked_transe(gamma):
    j = json.load(open(GOLD))
    e = np.array(j["edges"], dtype=np.uint32)
    X = np.zeros((j["n"], 8), np.float32)
    X[:, :2] = np.array(j["X"], np.float32)   # zero padding adds |0 + 0 - 0| = 0 to every distance
    Y = np.zeros((j["R"], 8), np.float32)
    Y[:, :2] = np.array(j["Y"], np.float32)
    say(f"case transe handworked gamma={gamma}")
    g = gpu_graph(j["n"], j["R"], e[:, 0], e[:, 1], e[:, 2], X, Y, scorer=TE, gamma=gamma)
    s = [q["s"] for q in j["queries"]]
    d = [q["t"] for q in j["queries"]]
    p, c, tot, st = run_gpu(g, s, d, 16)
    for qi, q in enumerate(j["queries"]):
        assert int(tot[qi]) == q["total"] and int(c[qi]) == len(q["paths"]) and st[qi] == 0
        for got, exp in zip(p[qi][:c[qi]], q["paths"]):
            assert (got["a"], got["b"], got["r1"], got["r2"], got["r3"]) == \
                (exp["a"], exp["b"], exp["r1"], exp["r2"], exp["r3"])
            assert float(got["score"]) == 3 * gamma - sum(exp["l1"])


@pytest.mark.parametrize("name", ["tiny", "dense_tiny", "hub_tiny", "dense_tiny_bf16", "hub_tiny_bf16",
                                  "hub_r32_bf16"])
def test_transe_small_workloads(name):
    gpu, orc = _small(name)
    compare(gpu, orc)


@pytest.mark.parametrize("k", [1, 7, 64, 200])
def test_transe_k_values(k):
    gpu, orc = _small("dense_tiny", k=k, gamma=0.75)
    compare(gpu, orc)


def test_transe_all_equal_scores():
    """All-zero embeddings: every weight is gamma, every score 3 gamma, so
    the ranking is the lexicographic order of the ids (exhaustive pass)."""
    gpu, orc = _small("dense_tiny", k=10, zero=True)
    compare(gpu, orc)
    p, c, tot, st = gpu
    assert np.all(p["score"][c > 0, 0] == np.float32(3.0))


def test_transe_wide_band_keeps_results():
    """A band of 4.0, about the spread of the paths' scores, so it outgrows
    the tile lists: the results equal the oracle's and are the same bytes as
    with the rigorous band alone."""
    import paper_2406_07727_amd as mhr
    opts = mhr.QueryOpts()
    opts.band_abs = 4.0
    gpu, orc = _small("hub_r32_bf16", opts=opts)
    compare(gpu, orc)
    base, _ = _small("hub_r32_bf16")
    assert_same_result(gpu, base)


def test_transe_forward_direction_and_heavy_probe():
    """The weight is directed, so the forward plan (scanning out-rows) and
    the backward plan (in-rows) orient the three edges differently; both run
    here, with hash and directory probes."""
    import paper_2406_07727_amd as mhr
    n, R = 6000, 4
    h, r, t = kgsynth.chung_lu_graph(n, R, 60000, 2.1, 2500.0, seed=41)
    X, Y = kgsynth.embeddings(n, R, kgsynth.EmbSpec(16, "f32", seed=42))
    indeg = np.bincount(t, minlength=n)
    outdeg = np.bincount(h, minlength=n)
    hubs = np.argsort(-indeg)[:8].astype(np.uint32)
    rng = np.random.Generator(np.random.PCG64(3))
    src = rng.integers(0, n, 40).astype(np.uint32)
    dst = hubs[rng.integers(0, len(hubs), 40)]
    src = np.concatenate([src, np.argsort(-outdeg)[:8].astype(np.uint32)])
    dst = np.concatenate([dst, rng.integers(0, n, 8).astype(np.uint32)])
    say("case transe forward/heavy")
    g = gpu_graph(n, R, h, r, t, X, Y, scorer=TE)
    orc = run_oracle(n, R, h, r, t, X, Y, src, dst, 16, scorer=TE)
    for hl in (10, 12):
        gpu = run_gpu(g, src, dst, 16, opts=mhr.QueryOpts(0, 0, 0, hl))
        compare(gpu, orc)


@pytest.mark.parametrize("name", ["hub_tiny", "hub_r32_bf16"])
def test_transe_edge_weights(name):
    cfg, (h, r, t), (X, Y), _ = workload(name)
    n, R = cfg.graph.n, cfg.graph.R
    rng = np.random.Generator(np.random.PCG64(11))
    m = 4096
    u = rng.integers(0, n, m).astype(np.uint32)
    rr = rng.integers(0, R, m).astype(np.uint32)
    v = rng.integers(0, n, m).astype(np.uint32)
    say(f"case transe edge weights {name}")
    g = gpu_graph(n, R, h, r, t, X, Y, cfg.emb.dtype, scorer=TE, gamma=1.0)
    w, e, hi, lo = (x.cpu().numpy() for x in g.edge_weights(u, rr, v))
    og = oracle.Graph(n, R, h, r, t)
    _, w64 = og.edge_weights(oracle.as_f32_table(X, cfg.emb.dtype), oracle.as_f32_table(Y, cfg.emb.dtype),
                             u, rr, v, scorer=TE, gamma=1.0)
    err32 = np.abs(w.astype(np.float64) - w64)
    assert np.all(err32 <= e.astype(np.float64) + 1e-15), err32.max()
    assert np.all(e <= 1e-4 * (1 + np.abs(w64)))
    errff = np.abs(hi.astype(np.float64) + lo.astype(np.float64) - w64)
    assert np.all(errff <= 1e-12 * (1 + np.abs(w64))), errff.max()


@pytest.mark.timeout(600)
def test_transe_realistic_full_size_sample():
    """The 1M-vertex / 20M-edge graph, d=128 FP32, all 1,024 queries in one
    launch with the TransE-L1 scorer; 256 sampled queries checked against
    the oracle."""
    cfg, (h, r, t), (X, Y), (s, d, kk) = workload("realistic")
    n, R = cfg.graph.n, cfg.graph.R
    say("case transe realistic full batch")
    g = gpu_graph(n, R, h, r, t, X, Y, scorer=TE)
    gpu = run_gpu(g, s, d, 32)
    p, c, tot, st = gpu
    assert np.all((st & ~np.uint32(4)) == 0)
    assert np.all(c == np.minimum(32, tot))
    rng = np.random.Generator(np.random.PCG64(29))
    sample = np.sort(rng.choice(len(s), 256, replace=False))
    og = oracle.Graph(n, R, h, r, t)
    parts = []
    for i in range(0, 256, 64):
        sq = sample[i:i + 64]
        parts.append((sq, run_oracle(n, R, h, r, t, X, Y, s[sq], d[sq], 32, og=og, scorer=TE)))
        say(f"oracle {i + 64}/256")
    ties = 0
    for sq, orc in parts:
        ties += compare(gpu, orc, queries=list(sq))
    say(f"transe realistic: 256 sampled queries equal the oracle ({ties} precision ties)")
