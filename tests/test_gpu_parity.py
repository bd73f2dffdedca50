"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle on
the same seeded inputs.  Sets and order must match exactly (permutations
only inside flagged precision ties), scores within 1e-5 relative and within
each result's own error bound."""

import json
import os

import numpy as np
import pytest

import kgsynth
import oracle
from tests.parity import (OracleResult, assert_same_result, compare, gpu_graph, run_gpu, run_oracle, say,
                          tied_tables, workload)

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "handworked_d2.json")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2406_07727_amd  # noqa: F401  (fails loudly if the library is missing)
    oracle.build(force=False)


def _small(name, k=None, nq=None, opts=None, zero=False):
    cfg, (h, r, t), (X, Y), (s, d, kk) = workload(name)
    if nq:
        s, d, kk = s[:nq], d[:nq], kk[:nq]
    if k is not None:
        kk = np.full(len(s), k, np.uint32)
    if zero:
        X = np.zeros_like(X)
        Y = np.zeros_like(Y)
    n, R = cfg.graph.n, cfg.graph.R
    say(f"case {name} nq={len(s)} k={int(kk.max())} zero={zero}")
    g = gpu_graph(n, R, h, r, t, X, Y, cfg.emb.dtype)
    gpu = run_gpu(g, s, d, kk, k_max=int(kk.max()), opts=opts)
    orc = run_oracle(n, R, h, r, t, X, Y, s, d, kk, cfg.emb.dtype)
    return gpu, orc


def test_handworked_fixture():
    j = json.load(open(GOLD))
    e = np.array(j["edges"], dtype=np.uint32)
    X = np.zeros((j["n"], 8), np.float32)
    X[:, :2] = np.array(j["X"], np.float32)   # zero padding leaves every score unchanged
    Y = np.zeros((j["R"], 8), np.float32)
    Y[:, :2] = np.array(j["Y"], np.float32)
    say("case handworked")
    g = gpu_graph(j["n"], j["R"], e[:, 0], e[:, 1], e[:, 2], X, Y)
    s = [q["s"] for q in j["queries"]]
    d = [q["t"] for q in j["queries"]]
    p, c, tot, st = run_gpu(g, s, d, 16)
    import decimal
    for qi, q in enumerate(j["queries"]):
        assert int(tot[qi]) == q["total"] and int(c[qi]) == len(q["paths"]) and st[qi] == 0
        for got, exp in zip(p[qi][:c[qi]], q["paths"]):
            assert (got["a"], got["b"], got["r1"], got["r2"], got["r3"]) == \
                (exp["a"], exp["b"], exp["r1"], exp["r2"], exp["r3"])
            with decimal.localcontext() as ctx:
                ctx.prec = 50
                ref = float(sum(-(1 + (-decimal.Decimal(x)).exp()).ln() for x in exp["x"]))
            assert abs(float(got["score"]) - ref) <= float(got["err_bound"]) + 1e-13


@pytest.mark.parametrize("name", ["tiny", "dense_tiny", "hub_tiny", "dense_tiny_bf16", "hub_tiny_bf16",
                                  "hub_r32_bf16"])
def test_small_workloads(name):
    gpu, orc = _small(name)
    compare(gpu, orc)


@pytest.mark.parametrize("k", [1, 2, 7, 32, 64, 200])
def test_k_values_dense(k):
    gpu, orc = _small("dense_tiny", k=k)
    compare(gpu, orc)


def test_per_query_k_mixed():
    cfg, (h, r, t), (X, Y), (s, d, _) = workload("hub_tiny")
    rng = np.random.Generator(np.random.PCG64(7))
    kk = rng.choice(np.array([1, 8, 64], np.uint32), size=len(s))
    say("case per-query k")
    g = gpu_graph(cfg.graph.n, cfg.graph.R, h, r, t, X, Y)
    gpu = run_gpu(g, s, d, kk, k_max=64)
    orc = run_oracle(cfg.graph.n, cfg.graph.R, h, r, t, X, Y, s, d, kk)
    compare(gpu, orc)


def test_all_zero_embeddings_exhaustive_pass():
    """Every path scores -3 ln 2 exactly: the FP32 band holds every path, so
    truncated tiles force the exhaustive float-float pass; the ranking is
    then the lexicographic order of (a, b, r1, r2, r3)."""
    gpu, orc = _small("dense_tiny", k=10, zero=True)
    compare(gpu, orc)
    p, c, tot, st = gpu
    assert np.all(p["score"][c > 0, 0] == np.float32(-3 * np.log(2)))


def test_forward_direction_and_heavy_probe():
    """Queries from low-degree sources to hub targets make the forward plan
    cheaper; hash_log2=10 forces long probe rows onto the bucket
    directories."""
    import paper_2406_07727_amd as mhr
    cfg = kgsynth.CONFIGS["hub_tiny"]
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
    say(f"case forward/heavy max_in={indeg.max()} max_out={outdeg.max()}")
    g = gpu_graph(n, R, h, r, t, X, Y)
    assert g.stats()["heavy_rows_in"] > 0 and g.stats()["heavy_rows_out"] > 0
    orc = run_oracle(n, R, h, r, t, X, Y, src, dst, 16)
    for hl in (10, 12):
        opts = mhr.QueryOpts(0, 0, 0, hl)
        gpu = run_gpu(g, src, dst, 16, opts=opts)
        compare(gpu, orc)


def test_tiling_and_grid_do_not_change_results():
    import paper_2406_07727_amd as mhr
    cfg, (h, r, t), (X, Y), (s, d, kk) = workload("hub_tiny")
    say("case tiling invariance")
    g = gpu_graph(cfg.graph.n, cfg.graph.R, h, r, t, X, Y)
    ref = run_gpu(g, s, d, 16)
    for te, gb, hl in ((64, 3, 10), (500, 7, 11), (1 << 20, 1, 12), (0, 0, 0)):
        got = run_gpu(g, s, d, 16, opts=mhr.QueryOpts(0, te, gb, hl))
        for a, b in zip(ref, got):
            assert np.array_equal(a, b), (te, gb, hl)
    again = run_gpu(g, s[::-1].copy(), d[::-1].copy(), 16)
    for a, b in zip(ref, again):
        assert np.array_equal(a, b[::-1])


def _tiles_per_query(n, h, t, src, dst, tile_edges, nq):
    """Tile counts the schedule gives each query: the scan cost of the
    cheaper direction over distinct (u, v) pairs, tiles of tile_edges entries
    (at most 4096 per query), the tile size doubled while the batch exceeds
    the workspace's max(4 nq, 16384) tiles."""
    pairs = np.unique(np.stack([h, t], 1).astype(np.int64), axis=0)
    u, v = pairs[:, 0], pairs[:, 1]
    outdeg = np.bincount(u, minlength=n)
    indeg = np.bincount(v, minlength=n)
    cost = []
    for s_, t_ in zip(src, dst):
        cb = int(indeg[u[v == t_]].sum())
        cf = int(outdeg[v[u == s_]].sum())
        probe = outdeg[s_] if cf >= cb else indeg[t_]
        cost.append(min(cf, cb) if probe > 0 else 0)
    cost = np.array(cost, np.int64)
    te, cap = tile_edges, max(4 * nq, 16384)
    while True:
        nt = np.where(cost > 0, np.minimum((cost + te - 1) // te, 4096), 0)
        if nt.sum() <= cap:
            return nt
        te *= 2


def test_merge_selects_over_many_tiles():
    """The fast merge's radix select over the tile lists, with the keys held
    in LDS (at most 8192 list slots) and streamed from memory (more), against
    the oracle and the default tiling."""
    import paper_2406_07727_amd as mhr
    cfg, (h, r, t), (X, Y), (s, d, kk) = workload("hub_tiny")
    n, R = cfg.graph.n, cfg.graph.R
    nt = _tiles_per_query(n, h, t, s, d, 4, len(s))
    say(f"case many tiles: max tiles/query {nt.max()}, queries with 2..128 tiles {int(((nt > 1) & (nt <= 128)).sum())}")
    assert nt.max() > 128 and ((nt > 1) & (nt <= 128)).any()
    g = gpu_graph(n, R, h, r, t, X, Y)
    ref = run_gpu(g, s, d, 16)
    got = run_gpu(g, s, d, 16, opts=mhr.QueryOpts(0, 4, 0, 0))
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)
    compare(got, run_oracle(n, R, h, r, t, X, Y, s, d, 16))


def test_large_batch_matches_split_batches():
    """Batches above 4,096 queries schedule from the plans in HBM, smaller
    ones from a copy in LDS: one batch of 5,000 queries and the same queries
    in two halves give identical results."""
    cfg, (h, r, t), (X, Y), (s, d, kk) = workload("hub_tiny")
    n, R = cfg.graph.n, cfg.graph.R
    rng = np.random.Generator(np.random.PCG64(7))
    pick = rng.integers(0, len(s), 5000)
    s5, d5 = s[pick].copy(), d[pick].copy()
    say("case large batch vs split batches (5000 queries)")
    g = gpu_graph(n, R, h, r, t, X, Y)
    whole = run_gpu(g, s5, d5, 16)
    a = run_gpu(g, s5[:2500].copy(), d5[:2500].copy(), 16)
    b = run_gpu(g, s5[2500:].copy(), d5[2500:].copy(), 16)
    for w, x, y in zip(whole, a, b):
        assert np.array_equal(w, np.concatenate([x, y]))
    sub = np.arange(0, 5000, 250)
    compare(tuple(arr[sub] for arr in whole), run_oracle(n, R, h, r, t, X, Y, s5[sub], d5[sub], 16))


def test_bad_queries_and_empty_results():
    import paper_2406_07727_amd as mhr
    cfg, (h, r, t), (X, Y), _ = workload("tiny")
    n = cfg.graph.n
    say("case bad queries")
    g = gpu_graph(n, cfg.graph.R, h, r, t, X, Y)
    src = np.array([0, n, 5, 3, 3], np.uint32)
    dst = np.array([1, 2, n + 7, 3, 4], np.uint32)
    kk = np.array([4, 4, 4, 4, 0], np.uint32)
    p, c, tot, st = run_gpu(g, src, dst, kk, k_max=4)
    assert st[1] & mhr.Q_BAD_ID and st[2] & mhr.Q_BAD_ID and st[4] & mhr.Q_BAD_K
    assert c[1] == 0 and c[2] == 0 and c[4] == 0
    assert np.all(p["a"][1] == 0xFFFFFFFF) and np.all(np.isneginf(p["score"][4]))
    orc = run_oracle(n, cfg.graph.R, h, r, t, X, Y, src[[0, 3]], dst[[0, 3]], 4)
    compare((p, c, tot, st), orc, queries=[0, 3])


def test_permuted_weight_ties_on_gpu():
    """a = t: the two paths whose middle and last relations swap carry the
    same weights; both sides must report an exact tie broken by the ids."""
    n, R, d = 6, 2, 8
    rng = np.random.Generator(np.random.PCG64(12))
    X = rng.standard_normal((n, d)).astype(np.float32) * 0.3
    Y = rng.standard_normal((R, d)).astype(np.float32) * 0.3
    s, t, b = 0, 3, 4
    edges = np.array([(s, 0, t), (t, 0, b), (t, 1, b), (b, 0, t), (b, 1, t)], np.uint32)
    say("case permuted-weight tie")
    g = gpu_graph(n, R, edges[:, 0], edges[:, 1], edges[:, 2], X, Y)
    gpu = run_gpu(g, [s], [t], 8)
    orc = run_oracle(n, R, edges[:, 0], edges[:, 1], edges[:, 2], X, Y, [s], [t], 8)
    compare(gpu, orc)
    p, c, _, _ = gpu
    sc = {(int(x["r2"]), int(x["r3"])): x["score"] for x in p[0][:c[0]]}
    assert sc[(0, 1)] == sc[(1, 0)]


def test_graph_without_edges():
    say("case empty graph")
    X = np.ones((10, 8), np.float32)
    Y = np.ones((2, 8), np.float32)
    e = np.zeros(0, np.uint32)
    g = gpu_graph(10, 2, e, e, e, X, Y)
    p, c, tot, st = run_gpu(g, [0, 1], [1, 0], 3)
    assert np.all(c == 0) and np.all(tot == 0) and np.all(st == 0)


def test_bad_edge_ids_rejected():
    import paper_2406_07727_amd as mhr
    say("case bad edges")
    with pytest.raises(mhr.MhrError):
        mhr.Graph(np.array([0, 11], np.uint32), np.array([0, 0], np.uint32), np.array([1, 2], np.uint32), 10, 1)
    with pytest.raises(mhr.MhrError):
        mhr.Graph(np.array([0, 1], np.uint32), np.array([0, 3], np.uint32), np.array([1, 2], np.uint32), 10, 2)


def test_csr_matches_numpy_construction():
    cfg, (h, r, t), (X, Y), _ = workload("hub_tiny")
    n, R = cfg.graph.n, cfg.graph.R
    rng = np.random.Generator(np.random.PCG64(5))
    dup = rng.integers(0, len(h), 1000)
    perm = rng.permutation(len(h) + 1000)
    H = np.concatenate([h, h[dup]])[perm]
    Rr = np.concatenate([r, r[dup]])[perm]
    T = np.concatenate([t, t[dup]])[perm]
    say("case csr")
    g = gpu_graph(n, R, H, Rr, T, X, Y)
    for rev in (False, True):
        rp, col, rm = (x.cpu().numpy().view(np.uint32) for x in g.export_csr(reverse=rev))
        u, v = (T, H) if rev else (H, T)
        key = u.astype(np.int64) * n + v
        pairs, inv = np.unique(key, return_inverse=True)
        mask = np.zeros(len(pairs), np.uint64)
        np.bitwise_or.at(mask, inv, (np.uint64(1) << Rr.astype(np.uint64)))
        exp_rp = np.searchsorted(pairs // n, np.arange(n + 1), side="left")
        assert np.array_equal(rp, exp_rp.astype(np.uint32))
        assert np.array_equal(col, (pairs % n).astype(np.uint32))
        assert np.array_equal(rm, mask.astype(np.uint32))
    st = g.stats()
    assert st["num_triples"] == len(np.unique((h.astype(np.int64) * n + t) * R + r))


def test_caller_buffer_graph_matches_library_allocation():
    """A graph built in caller buffers (mhr_graph_create_in) holds the same
    CSRs as one the library allocates itself, long rows and their
    directories included, and answers queries identically."""
    import torch
    import paper_2406_07727_amd as mhr
    cfg, (h, r, t), (X, Y), (s, d, k) = workload("hub_tiny")
    n, R = cfg.graph.n, cfg.graph.R
    # two hubs of 1,500 out- and in-neighbours: rows long enough for directories
    rng = np.random.Generator(np.random.PCG64(21))
    hub_out = rng.choice(n, 1500, replace=False).astype(np.uint32)
    hub_in = rng.choice(n, 1500, replace=False).astype(np.uint32)
    H = np.concatenate([h, np.full(1500, 3, np.uint32), hub_in]).astype(np.uint32)
    T = np.concatenate([t, hub_out, np.full(1500, 5, np.uint32)]).astype(np.uint32)
    Rr = np.concatenate([r, rng.integers(0, R, 3000).astype(np.uint32)]).astype(np.uint32)
    say("case caller-buffer graph")
    own = mhr.Graph(H, Rr, T, n, R)
    cal = mhr.Graph(H, Rr, T, n, R, caller_buffers=True)
    so, sc = own.stats(), cal.stats()
    for f in ("num_triples", "num_pairs", "max_out_degree", "max_in_degree", "heavy_rows_out", "heavy_rows_in"):
        assert so[f] == sc[f], f
    assert sc["heavy_rows_out"] >= 1 and sc["heavy_rows_in"] >= 1
    assert 0 < sc["device_bytes"] <= mhr.graph_buffer_sizes(n, R, len(H))[0]
    for rev in (False, True):
        for a, b in zip(own.export_csr(reverse=rev), cal.export_csr(reverse=rev)):
            assert torch.equal(a, b)
    Xd, Yd = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
    own.set_embeddings(Xd, Yd)
    cal.set_embeddings(Xd, Yd)
    qs = np.concatenate([s, np.array([3, 3, 7], np.uint32)]).astype(np.uint32)
    qd = np.concatenate([d, np.array([5, 9, 5], np.uint32)]).astype(np.uint32)
    ro = own.topk(qs, qd, 16).to_numpy()
    rc = cal.topk(qs, qd, 16).to_numpy()
    for a, b in zip(ro, rc):
        assert np.array_equal(np.asarray(a).view(np.uint8), np.asarray(b).view(np.uint8))
    cal.close()
    own.close()


@pytest.mark.parametrize("name", ["tiny", "hub_tiny"])
def test_edge_weights_against_oracle(name):
    cfg, (h, r, t), (X, Y), _ = workload(name)
    n, R = cfg.graph.n, cfg.graph.R
    rng = np.random.Generator(np.random.PCG64(11))
    m = 4096
    u = rng.integers(0, n, m).astype(np.uint32)
    rr = rng.integers(0, R, m).astype(np.uint32)
    v = rng.integers(0, n, m).astype(np.uint32)
    # larger |x| too: scaled copies of the tables
    for scale in (1.0, 8.0, 64.0):
        Xs = (X * np.float32(scale)).astype(np.float32)
        say(f"case edge weights {name} scale={scale}")
        g = gpu_graph(n, R, h, r, t, Xs, Y)
        w, e, hi, lo = (x.cpu().numpy() for x in g.edge_weights(u, rr, v))
        og = oracle.Graph(n, R, h, r, t)
        _, w64 = og.edge_weights(Xs, Y, u, rr, v)
        err32 = np.abs(w.astype(np.float64) - w64)
        assert np.all(err32 <= e.astype(np.float64) + 1e-15), err32.max()
        errff = np.abs(hi.astype(np.float64) + lo.astype(np.float64) - w64)
        assert np.all(errff <= 1e-12 * (1 + np.abs(w64))), errff.max()


@pytest.mark.parametrize("k", [1, 16, 64])
def test_bf16_two_relation_blocks_k(k):
    gpu, orc = _small("hub_r32_bf16", k=k)
    compare(gpu, orc)


def test_bf16_edge_weights_against_oracle():
    cfg, (h, r, t), (Xb, Yb), _ = workload("hub_r32_bf16")
    n, R = cfg.graph.n, cfg.graph.R
    rng = np.random.Generator(np.random.PCG64(12))
    m = 4096
    u = rng.integers(0, n, m).astype(np.uint32)
    rr = rng.integers(0, R, m).astype(np.uint32)
    v = rng.integers(0, n, m).astype(np.uint32)
    X = oracle.as_f32_table(Xb, "bf16")
    for scale in (1.0, 16.0):   # power-of-two scaling keeps the values bfloat16
        Xs = (X * np.float32(scale)).astype(np.float32)
        Xsb = kgsynth.f32_to_bf16_bits(Xs)
        assert np.array_equal(kgsynth.bf16_bits_to_f32(Xsb), Xs)
        say(f"case bf16 edge weights scale={scale}")
        g = gpu_graph(n, R, h, r, t, Xsb, Yb, "bf16")
        w, e, hi, lo = (x.cpu().numpy() for x in g.edge_weights(u, rr, v))
        og = oracle.Graph(n, R, h, r, t)
        _, w64 = og.edge_weights(Xs, oracle.as_f32_table(Yb, "bf16"), u, rr, v)
        err32 = np.abs(w.astype(np.float64) - w64)
        assert np.all(err32 <= e.astype(np.float64) + 1e-15), err32.max()
        errff = np.abs(hi.astype(np.float64) + lo.astype(np.float64) - w64)
        assert np.all(errff <= 1e-12 * (1 + np.abs(w64))), errff.max()


def _oracle_in_chunks(name, n, R, h, r, t, X, Y, s, d, k, dtype="f32", chunk=128):
    """The oracle over a large sample, in chunks with a progress line each
    (a full-size sample takes tens of seconds); results cached per process
    under `name`."""
    key = (name, len(s), int(np.asarray(s, np.int64).sum()), int(np.asarray(k, np.int64).sum()))
    if key in _ORACLE_CACHE:
        return _ORACLE_CACHE[key]
    og = oracle.Graph(n, R, h, r, t)
    kk = np.broadcast_to(np.asarray(k, dtype=np.uint32), (len(s),)).copy()
    parts = []
    for i in range(0, len(s), chunk):
        parts.append(run_oracle(n, R, h, r, t, X, Y, s[i:i + chunk], d[i:i + chunk], kk[i:i + chunk], dtype, og=og))
        say(f"oracle {min(i + chunk, len(s))}/{len(s)}")
    width = max(p.paths.shape[1] for p in parts)
    paths = np.zeros((len(s), width), oracle.PATH_DTYPE)
    o = 0
    for p in parts:
        paths[o:o + len(p.count), :p.paths.shape[1]] = p.paths
        o += len(p.count)
    res = OracleResult(paths, *(np.concatenate([getattr(p, f) for p in parts]) for f in ("count", "total", "full")))
    _ORACLE_CACHE[key] = res
    return res


_ORACLE_CACHE = {}


@pytest.mark.timeout(600)
def test_realistic_full_size_all_queries():
    """The 1M-vertex / 20M-edge graph, d=128, K=32, in the launch the
    benchmark times: all 1,024 queries are checked against the oracle."""
    cfg, (h, r, t), (X, Y), (s, d, kk) = workload("realistic")
    n, R = cfg.graph.n, cfg.graph.R
    say("case realistic full batch")
    g = gpu_graph(n, R, h, r, t, X, Y)
    gpu = run_gpu(g, s, d, 32)
    p, c, tot, st = gpu
    assert np.all(st == 0)
    assert np.all(c == np.minimum(32, tot))
    orc = _oracle_in_chunks("realistic", n, R, h, r, t, X, Y, s, d, 32)
    ties = compare(gpu, orc)
    say(f"realistic: {len(s)} queries equal the oracle ({ties} precision ties)")


def _precision_sample():
    cfg, (h, r, t), (X, Y), (s, d, kk) = workload("precision")
    n, R = cfg.graph.n, cfg.graph.R
    sample = np.arange(256)   # the first 256 queries
    orc = _oracle_in_chunks("precision", n, R, h, r, t, X, Y, s[sample], d[sample], 32, "bf16")
    return cfg, (h, r, t), (X, Y), (s, d), sample, orc


@pytest.mark.timeout(600)
@pytest.mark.parametrize("band", [0.0, 1e-2])
def test_precision_full_size_subsample(band):
    """The 4M-vertex / 64M-edge graph with d=256 bfloat16 embeddings and 32
    relations, all 4,096 queries at K=32 in one launch (bfloat16 MFMA
    scoring), with the rigorous band alone and with the fixed 1e-2 band; the
    first 256 queries are checked against the oracle.  The wider band
    rescores more kept candidates but returns the same bytes and sends no
    more queries to the exhaustive pass."""
    import paper_2406_07727_amd as mhr
    say(f"case precision full batch band={band}")
    cfg, (h, r, t), (X, Y), (s, d), sample, orc = _precision_sample()
    n, R = cfg.graph.n, cfg.graph.R
    g = gpu_graph(n, R, h, r, t, X, Y, "bf16")
    opts = mhr.QueryOpts()
    opts.band_abs = band
    gpu = run_gpu(g, s, d, 32, opts=opts)
    p, c, tot, st = gpu
    assert np.all((st & ~np.uint32(4)) == 0)
    assert np.all(c == np.minimum(32, tot))
    ties = compare(gpu, orc, queries=list(sample))
    nx = int(np.sum((st & 4) != 0))
    say(f"precision band={band}: {len(sample)} queries equal the oracle; {nx} queries took the exhaustive pass; "
        f"{ties} precision ties")
    if band > 0:
        assert_same_result(gpu, run_gpu(g, s, d, 32))


@pytest.mark.timeout(900)
def test_precision_full_size_tied_exhaustive():
    """The precision graph at full size with tables that make the best paths
    tie (tied_tables: half the entity rows zero, every DistMult value <= 0):
    the paths of score -3 ln 2 outnumber the tile lists, so queries take the
    exhaustive float-float pass, which skips the lower paths and ranks the
    tied ones by ids.  All 4,096 queries in one launch; the first 64 against
    the oracle."""
    say("case precision full batch, tied top")
    cfg, (h, r, t), (X, Y), (s, d, _) = workload("precision")
    n, R = cfg.graph.n, cfg.graph.R
    Xt, Yt = tied_tables(X, Y, "bf16", 0.5, seed=5)
    g = gpu_graph(n, R, h, r, t, Xt, Yt, "bf16")
    gpu = run_gpu(g, s, d, 32)
    p, c, tot, st = gpu
    assert np.all((st & ~np.uint32(4)) == 0)
    assert np.all(c == np.minimum(32, tot))
    sample = np.arange(64)
    orc = _oracle_in_chunks("precision_tied", n, R, h, r, t, Xt, Yt, s[sample], d[sample], 32, "bf16", chunk=32)
    ties = compare(gpu, orc, queries=list(sample))
    nx = int(np.sum((st & 4) != 0))
    say(f"precision tied: {nx} queries took the exhaustive pass, {int(np.sum((st[sample] & 4) != 0))} of the "
        f"sample; {ties} precision ties")
    assert nx > 0 and np.sum((st[sample] & 4) != 0) > 0
    # every value is <= 0, so no path beats -3 ln 2; most queries reach it
    top = p["score"][c > 0, 0]
    tie = np.float32(-3 * np.log(2))
    assert np.all(top <= tie) and np.mean(top == tie) > 0.5


def test_plan_replays_match_eager():
    """A captured plan replayed several times, with eager calls and
    synchronisations between the replays, returns the eager results each
    time; a new batch written into its buffers is answered too."""
    import torch
    cfg, (h, r, t), (X, Y), (s, d, kk) = workload("hub_tiny")
    say("case plan replays")
    g = gpu_graph(cfg.graph.n, cfg.graph.R, h, r, t, X, Y)
    kq = (np.arange(len(s)) % 3 * 7 + 1).astype(np.uint32)   # K in {1, 8, 15}
    ref = run_gpu(g, s, d, kq, k_max=16)
    rs, rd = s[::-1].copy(), d[::-1].copy()
    ref_rev = run_gpu(g, rs, rd, kq[::-1].copy(), k_max=16)
    plan = g.plan(s, d, kq, k_max=16)
    for rep in range(3):
        got = plan.launch()
        torch.cuda.synchronize()
        for a, b in zip(ref, got.to_numpy()):
            assert np.array_equal(a, b), f"replay {rep}"
        run_gpu(g, rs, rd, 16)   # eager work between replays
        torch.cuda.synchronize()
    plan.set_queries(rs, rd, kq[::-1].copy())
    got = plan.launch()
    torch.cuda.synchronize()
    for a, b in zip(ref_rev, got.to_numpy()):
        assert np.array_equal(a, b)
    plan.close()


def test_autotune_keeps_results():
    cfg, (h, r, t), (X, Y), (s, d, kk) = workload("hub_tiny")
    say("case autotune")
    g = gpu_graph(cfg.graph.n, cfg.graph.R, h, r, t, X, Y)
    ref = run_gpu(g, s, d, 16)
    tuned, ms = g.autotune(s, d, 16, reps=2)
    assert tuned.tile_edges in (8192, 16384, 32768, 65536, 131072, 262144, 524288)
    assert tuned.hash_log2 in (10, 11, 12)
    assert ms > 0
    got = run_gpu(g, s, d, 16, opts=tuned)
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)


@pytest.mark.timeout(600)
def test_batched_full_size_sample():
    """The batched workload: the 1M-vertex graph with 16,384 queries (10%
    hub sources), K drawn from {1, 8, 64}, autotuned and run as one captured
    plan; a 512-query sample is checked against the oracle."""
    import torch
    cfg, (h, r, t), (X, Y), (s, d, kk) = workload("batched")
    n, R = cfg.graph.n, cfg.graph.R
    say("case batched full size")
    g = gpu_graph(n, R, h, r, t, X, Y)
    tuned, ms = g.autotune(s, d, kk, k_max=64, reps=1)
    say(f"tuned tile_edges={tuned.tile_edges} hash_log2={tuned.hash_log2} ({ms:.2f} ms)")
    plan = g.plan(s, d, kk, k_max=64, opts=tuned)
    plan.launch()
    torch.cuda.synchronize()
    gpu = plan.out.to_numpy()
    rng = np.random.Generator(np.random.PCG64(23))
    sample = np.sort(rng.choice(len(s), 512, replace=False))
    orc = _oracle_in_chunks("batched", n, R, h, r, t, X, Y, s[sample], d[sample], kk[sample])
    ties = compare(gpu, orc, queries=list(sample))
    say(f"batched: {len(sample)} sampled queries equal the oracle ({ties} precision ties)")
    p, c, tot, st = gpu
    assert np.all((st & ~np.uint32(4)) == 0)
    assert np.all(c == np.minimum(kk, tot))
    plan.close()


@pytest.mark.parametrize("name", ["dense_tiny", "hub_r32_bf16"])
def test_wide_rescoring_band_keeps_results(name):
    """A fixed rescoring band of 1e-2 below the K-th score (the precision
    form's margin), far wider than the rigorous band and, at d = 64, wider
    than the tile lists: the results equal the oracle's and are the same
    bytes as with the rigorous band alone."""
    import paper_2406_07727_amd as mhr
    opts = mhr.QueryOpts()
    opts.band_abs = 1e-2
    gpu, orc = _small(name, opts=opts)
    compare(gpu, orc)
    base, _ = _small(name)
    assert_same_result(gpu, base)


@pytest.mark.parametrize("name", ["hub_tiny", "hub_r32_bf16"])
def test_tied_top_exhaustive_pass(name):
    """Tables whose best paths tie (tied_tables): the tied paths outnumber
    the tile lists, so queries take the exhaustive pass; it skips the paths
    below the tie and ranks the tied ones by (a, b, r1, r2, r3)."""
    cfg, (h, r, t), (X, Y), (s, d, kk) = workload(name)
    n, R = cfg.graph.n, cfg.graph.R
    Xt, Yt = tied_tables(X, Y, cfg.emb.dtype, 0.5, seed=3)
    say(f"case tied top {name}")
    g = gpu_graph(n, R, h, r, t, Xt, Yt, cfg.emb.dtype)
    gpu = run_gpu(g, s, d, kk, k_max=int(kk.max()))
    orc = run_oracle(n, R, h, r, t, Xt, Yt, s, d, kk, cfg.emb.dtype)
    compare(gpu, orc)
    nx = int(np.sum((gpu[3] & 4) != 0))
    say(f"tied top {name}: {nx} of {len(s)} queries took the exhaustive pass")
    assert nx > 0
