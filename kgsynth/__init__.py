"""Seeded synthetic typed knowledge graphs, embeddings and query batches.

This module is shared by the CPU oracle and by the GPU path, so it holds only
random draws and storage rounding: no edge weight, no path, no top-K.
Every draw uses numpy's PCG64 with a fixed seed, so the same call gives the
same arrays on every machine.

Graphs are returned as three ``uint32`` arrays ``(head, rel, tail)``: the
edge list of the problem statement (section 3.1: triples (h, r, t), a
relation embedding table and an entity embedding table).  The synthetic laws
stand in for WikiKG90Mv2, which the paper measures on (section 4.1) and which
is not available here.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Optional, Tuple

import numpy as np

__all__ = [
    "GraphSpec", "EmbSpec", "QuerySpec", "Workload", "CONFIGS",
    "uniform_graph", "chung_lu_weights", "chung_lu_graph", "make_graph",
    "embeddings", "queries", "f32_to_bf16_bits", "bf16_bits_to_f32",
    "out_degree", "in_degree", "TuringSpec", "TURING", "turing_workload",
]


# ---------------------------------------------------------------------------
# specs
# ---------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class GraphSpec:
    kind: str            # "uniform" or "chunglu"
    n: int               # vertices
    R: int               # relation types
    m: int               # distinct directed typed edges
    seed: int
    gamma: float = 2.1   # Chung-Lu degree exponent
    wmax: float = 1e5    # Chung-Lu largest expected degree


@dataclasses.dataclass(frozen=True)
class EmbSpec:
    d: int
    dtype: str           # "f32" or "bf16" (storage type)
    seed: int


@dataclasses.dataclass(frozen=True)
class QuerySpec:
    nq: int
    law: str             # "uniform", "degree" or "hubmix"
    k: int               # K when k_choices is None
    seed: int
    k_choices: Optional[Tuple[int, ...]] = None
    hub_frac: float = 0.10
    hub_top: int = 1000


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    graph: GraphSpec
    emb: EmbSpec
    query: QuerySpec


CONFIGS = {
    # 2,000 vertices, 4 relations, 20,000 uniform edges, d=32 FP32, 64 queries, K=10
    "tiny": Workload(
        "tiny",
        GraphSpec("uniform", 2000, 4, 20000, seed=1),
        EmbSpec(32, "f32", seed=2),
        QuerySpec(64, "uniform", 10, seed=3)),
    # 1M vertices, 16 relations, 20M Chung-Lu edges (exponent 2.1), d=128 FP32,
    # 1,024 queries with degree-proportional sources, K=32
    "realistic": Workload(
        "realistic",
        GraphSpec("chunglu", 1_000_000, 16, 20_000_000, seed=2406),
        EmbSpec(128, "f32", seed=7727),
        QuerySpec(1024, "degree", 32, seed=11)),
    # 4M vertices, 32 relations, 64M Chung-Lu edges, d=256 BF16, 4,096 queries, K=32
    "precision": Workload(
        "precision",
        GraphSpec("chunglu", 4_000_000, 32, 64_000_000, seed=2407),
        EmbSpec(256, "bf16", seed=7728),
        QuerySpec(4096, "degree", 32, seed=12)),
    # the realistic graph with 16,384 mixed hub / degree-proportional queries,
    # K drawn from {1, 8, 64}
    "batched": Workload(
        "batched",
        GraphSpec("chunglu", 1_000_000, 16, 20_000_000, seed=2406),
        EmbSpec(128, "f32", seed=7727),
        QuerySpec(16384, "hubmix", 64, seed=13, k_choices=(1, 8, 64))),
    # test-only graphs: small enough for the pure-Python oracle, dense enough
    # that K truncation is exercised
    "dense_tiny": Workload(
        "dense_tiny",
        GraphSpec("uniform", 64, 4, 2000, seed=21),
        EmbSpec(8, "f32", seed=22),
        QuerySpec(32, "uniform", 10, seed=23)),
    "hub_tiny": Workload(
        "hub_tiny",
        GraphSpec("chunglu", 3000, 4, 30000, seed=31, wmax=600.0),
        EmbSpec(16, "f32", seed=32),
        QuerySpec(48, "degree", 16, seed=33)),
    # bfloat16 storage at test sizes: d = 8 and 16 (short per-lane slices),
    # and d = 64 with 32 relations (two relation blocks per match)
    "dense_tiny_bf16": Workload(
        "dense_tiny_bf16",
        GraphSpec("uniform", 64, 4, 2000, seed=21),
        EmbSpec(8, "bf16", seed=24),
        QuerySpec(32, "uniform", 10, seed=23)),
    "hub_tiny_bf16": Workload(
        "hub_tiny_bf16",
        GraphSpec("chunglu", 3000, 4, 30000, seed=31, wmax=600.0),
        EmbSpec(16, "bf16", seed=34),
        QuerySpec(48, "degree", 16, seed=33)),
    # learned-pruner tests: a mid-sized Chung-Lu graph, d=64 bfloat16; the
    # query spec is the held-out evaluation set (training queries use seed 82)
    "pruner_small": Workload(
        "pruner_small",
        GraphSpec("chunglu", 200_000, 16, 4_000_000, seed=77, wmax=20_000.0),
        EmbSpec(64, "bf16", seed=78),
        QuerySpec(2000, "degree", 32, seed=80)),
    # the learned-pruner form: the precision graph; held-out evaluation
    # queries (training queries use seed 15)
    "pruner": Workload(
        "pruner",
        GraphSpec("chunglu", 4_000_000, 32, 64_000_000, seed=2407),
        EmbSpec(256, "bf16", seed=7728),
        QuerySpec(8192, "degree", 32, seed=14)),
    "hub_r32_bf16": Workload(
        "hub_r32_bf16",
        GraphSpec("chunglu", 4000, 32, 60000, seed=41, wmax=800.0),
        EmbSpec(64, "bf16", seed=42),
        QuerySpec(48, "degree", 32, seed=43)),
}


# ---------------------------------------------------------------------------
# graphs
# ---------------------------------------------------------------------------

def _pack(u, r, v, n, R):
    return (u.astype(np.int64) * n + v.astype(np.int64)) * R + r.astype(np.int64)


def _draw_distinct(m, n, R, seed, draw_uv):
    """Draw (u, r, v) triples with u != v in batches until at least m distinct
    ones exist, then keep a uniformly random subset of exactly m of them.
    The triples come back sorted by (u, v, r); the edge order carries no
    meaning for the method."""
    rng = np.random.Generator(np.random.PCG64(seed))
    keys = np.empty(0, dtype=np.int64)
    while len(keys) < m:
        batch = int((m - len(keys)) * 1.12) + 1024
        u, v = draw_uv(rng, batch)
        r = rng.integers(0, R, size=batch, dtype=np.int64)
        ok = u != v
        keys = np.unique(np.concatenate([keys, _pack(u[ok], r[ok], v[ok], n, R)]))
    if len(keys) > m:
        pri = rng.random(len(keys))
        thr = np.partition(pri, m - 1)[m - 1]
        keys = keys[pri <= thr][:m]
    r = (keys % R).astype(np.uint32)
    uv = keys // R
    return ((uv // n).astype(np.uint32), r, (uv % n).astype(np.uint32))


def _weighted_sampler(w):
    """Sampler of indices i with probability w_i / sum(w): inverse CDF with a
    guide table of len(w) equal-width buckets, then a short forward walk to
    the first i whose cumulative weight exceeds the uniform draw."""
    cdf = np.cumsum(w)
    tot = cdf[-1]
    G = len(w)
    guide = np.searchsorted(cdf, np.arange(G, dtype=np.float64) * (tot / G), side="right")

    guide = np.append(guide, G - 1)

    def sample(rng, b):
        x = rng.random(b) * tot
        g = np.minimum((x * (G / tot)).astype(np.int64), G - 1)
        lo = guide[g]          # first i with cdf[i] > left edge of bucket g
        hi = guide[g + 1]      # the answer lies in [lo, hi]
        while True:
            open_ = lo < hi
            if not open_.any():
                break
            mid = (lo + hi) >> 1
            c = cdf[mid] <= x
            lo = np.where(open_ & c, mid + 1, lo)
            hi = np.where(open_ & ~c, mid, hi)
        return np.minimum(lo, G - 1)
    return sample


def uniform_graph(n: int, R: int, m: int, seed: int):
    """Endpoints and relation i.i.d. uniform; self-loops and duplicate triples
    rejected.  Returns (head, rel, tail) as uint32 arrays of length m."""
    if m > n * (n - 1) * R:
        raise ValueError("more distinct edges requested than exist")

    def draw(rng, b):
        return (rng.integers(0, n, size=b, dtype=np.int64),
                rng.integers(0, n, size=b, dtype=np.int64))
    return _draw_distinct(m, n, R, seed, draw)


def chung_lu_weights(n: int, m: int, gamma: float, wmax: float):
    """Expected degrees w_i = C (i + i0)^(-1/(gamma-1)) with w_0 = wmax and
    sum(w) = m; i0 solved by bisection.  Returns (w, i0, C)."""
    alpha = 1.0 / (gamma - 1.0)
    i = np.arange(n, dtype=np.float64)

    def total(i0):
        return wmax * i0 ** alpha * np.sum((i + i0) ** (-alpha))

    lo, hi = 1e-9, 1.0
    while total(hi) < m:
        hi *= 2.0
        if hi > 1e18:
            raise ValueError("cannot reach the requested edge count")
    for _ in range(200):
        mid = math.sqrt(lo * hi)
        if total(mid) < m:
            lo = mid
        else:
            hi = mid
    i0 = hi
    C = wmax * i0 ** alpha
    return C * (i + i0) ** (-alpha), i0, C


def chung_lu_graph(n: int, R: int, m: int, gamma: float, wmax: float, seed: int):
    """Chung-Lu graph: both endpoints drawn independently with probability
    proportional to w (the same weights for in and out), the weights placed
    on a random permutation of the ids so that id order carries no degree
    information; relation uniform; self-loops and duplicates rejected."""
    w, _, _ = chung_lu_weights(n, m, gamma, wmax)
    rng0 = np.random.Generator(np.random.PCG64(seed + 0x9E3779B1))
    perm = rng0.permutation(n)
    wp = np.empty(n, dtype=np.float64)
    wp[perm] = w
    sample = _weighted_sampler(wp)

    def draw(rng, b):
        return sample(rng, b), sample(rng, b)
    return _draw_distinct(m, n, R, seed, draw)


def make_graph(spec: GraphSpec):
    if spec.kind == "uniform":
        return uniform_graph(spec.n, spec.R, spec.m, spec.seed)
    if spec.kind == "chunglu":
        return chung_lu_graph(spec.n, spec.R, spec.m, spec.gamma, spec.wmax, spec.seed)
    raise ValueError(spec.kind)


def out_degree(head, n):
    return np.bincount(head, minlength=n)


def in_degree(tail, n):
    return np.bincount(tail, minlength=n)


# ---------------------------------------------------------------------------
# embeddings
# ---------------------------------------------------------------------------

def f32_to_bf16_bits(x: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (round to nearest, ties to even) and
    return the 16-bit patterns as uint16.  Inputs here are finite."""
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    b = (b + 0x7FFF + lsb) >> 16
    return b.astype(np.uint16)


def bf16_bits_to_f32(h: np.ndarray) -> np.ndarray:
    return (h.astype(np.uint32) << 16).view(np.float32)


def grid_values(rng, shape, levels: int, exp: int, density: float = 1.0) -> np.ndarray:
    """Integers drawn uniformly from [-levels, levels] times 2^exp (zeroed
    with probability 1 - density), as float64: values exactly representable
    in bfloat16 for levels <= 256, so that sums of their products stay on a
    known power-of-two grid."""
    v = rng.integers(-levels, levels + 1, shape).astype(np.float64)
    if density < 1.0:
        v *= rng.random(shape) < density
    return np.ldexp(v, exp)


def embeddings(n: int, R: int, spec: EmbSpec, chunk_rows: int = 1 << 16):
    """Entity table X[n][d] and relation table Y[R][d], entries drawn from a
    normal law with variance 1/d in float64 and rounded to the storage type.
    float32 storage returns float32 arrays; bf16 storage returns the uint16
    bit patterns.  Rows are drawn in chunks of ``chunk_rows`` from one
    generator (entity rows first, then relation rows)."""
    d = spec.d
    rng = np.random.Generator(np.random.PCG64(spec.seed))
    scale = 1.0 / math.sqrt(d)
    odt = np.float32 if spec.dtype == "f32" else np.uint16

    def table(rows):
        out = np.empty((rows, d), dtype=odt)
        for r0 in range(0, rows, chunk_rows):
            r1 = min(rows, r0 + chunk_rows)
            blk = (rng.standard_normal((r1 - r0, d)) * scale).astype(np.float32)
            out[r0:r1] = blk if spec.dtype == "f32" else f32_to_bf16_bits(blk)
        return out
    X = table(n)
    Y = table(R)
    return X, Y


# ---------------------------------------------------------------------------
# queries
# ---------------------------------------------------------------------------

def queries(head: np.ndarray, n: int, spec: QuerySpec):
    """(src, dst, k) arrays.  ``uniform``: s uniform; ``degree``: s drawn with
    probability proportional to its realized out-degree; ``hubmix``: a
    fraction hub_frac of the sources uniform over the hub_top vertices of
    largest out-degree (ties by id), the rest degree-proportional.  t is
    uniform over the vertices other than s.  k is spec.k, or uniform over
    spec.k_choices."""
    rng = np.random.Generator(np.random.PCG64(spec.seed))
    nq = spec.nq
    if spec.law == "uniform":
        s = rng.integers(0, n, size=nq, dtype=np.int64)
    else:
        deg = np.bincount(head, minlength=n).astype(np.float64)
        cdf = np.cumsum(deg)
        s = np.searchsorted(cdf, rng.random(nq) * cdf[-1], side="right")
        np.minimum(s, n - 1, out=s)
        if spec.law == "hubmix":
            order = np.lexsort((np.arange(n), -deg))
            hubs = order[:spec.hub_top]
            is_hub = rng.random(nq) < spec.hub_frac
            s = np.where(is_hub, hubs[rng.integers(0, len(hubs), size=nq)], s)
        elif spec.law != "degree":
            raise ValueError(spec.law)
    t = rng.integers(0, n - 1, size=nq, dtype=np.int64)
    t = t + (t >= s)
    if spec.k_choices:
        k = np.asarray(spec.k_choices, dtype=np.int64)[
            rng.integers(0, len(spec.k_choices), size=nq)]
    else:
        k = np.full(nq, spec.k, dtype=np.int64)
    return s.astype(np.uint32), t.astype(np.uint32), k.astype(np.uint32)


# ---------------------------------------------------------------------------
# the award-pipeline candidate scan (paper sections 3.2-3.3, section 4.1)
# ---------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class TuringSpec:
    n: int               # entities
    R: int               # relations
    d: int               # embedding dimension
    n_persons: int       # candidate persons (first hop)
    n_univ: int          # candidate universities (third hop)
    k: int
    seed: int


# The paper's workload shape: WikiKG90Mv2's 91,230,610 entities and 1,387
# relations, embeddings trimmed to d = 8, 539,603 persons, 89,689 universities,
# K = 50.  Synthetic tables stand in for the dataset.
TURING = {
    "turing": TuringSpec(91_230_610, 1387, 8, 539_603, 89_689, 50, seed=41),
    "turing_small": TuringSpec(2_000_000, 64, 8, 60_000, 12_000, 50, seed=43),
    "turing_tiny": TuringSpec(20_000, 8, 8, 3_000, 700, 16, seed=45),
}


def turing_workload(spec: TuringSpec):
    """Entity and relation tables (N(0, 1/d), FP32), disjoint random person
    and university id lists, the award and field entities and three distinct
    relations (award winner, works in, affiliated with).  Returns
    (X, Y, persons, universities, award, field, (r_award, r_works, r_affil))."""
    X, Y = embeddings(spec.n, spec.R, EmbSpec(spec.d, "f32", seed=spec.seed))
    rng = np.random.Generator(np.random.PCG64(spec.seed + 1))
    ids = rng.choice(spec.n, spec.n_persons + spec.n_univ + 2, replace=False).astype(np.uint32)
    persons = ids[:spec.n_persons]
    univ = ids[spec.n_persons:spec.n_persons + spec.n_univ]
    award, field = int(ids[-2]), int(ids[-1])
    rels = rng.choice(spec.R, 3, replace=False)
    return X, Y, persons, univ, award, field, tuple(int(x) for x in rels)


# ---------------------------------------------------------------------------
# wide-relation knowledge graphs (the scale of the paper's WikiKG90Mv2
# experiments: 91,230,610 entities, 1,387 relations, 601,062,811 triples,
# 8-dimensional embeddings; section 4.1)
# ---------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class WideSpec:
    n: int
    R: int
    m: int                  # triples drawn (duplicates are merged at ingest)
    seed: int
    out_gamma: float = 2.5  # power-law exponent of the out-degree distribution
    in_gamma: float = 2.2   # and of the in-degree distribution (hubs are targets)
    rel_power: float = 4.0  # relation rank = floor(R * u^rel_power): a few relations dominate
    d: int = 8
    dtype: str = "f32"


WIDE = {
    # the paper's graph size
    "paper_kg": WideSpec(91_230_610, 1_387, 601_062_811, seed=2406),
    # one sixteenth of it, same shape
    "paper_kg_16th": WideSpec(5_701_913, 1_387, 37_566_425, seed=2407),
    # small graphs for parity tests: many relations per pair, hubs past one tile
    "wide_tiny": WideSpec(60, 40, 1_500, seed=11, out_gamma=3.0, in_gamma=3.0, rel_power=1.5),
    "wide_small": WideSpec(20_000, 1_387, 300_000, seed=12),
    "wide_hub": WideSpec(6_000, 300, 500_000, seed=13, out_gamma=2.1, in_gamma=2.0),
    "wide_small_bf16": WideSpec(20_000, 1_387, 300_000, seed=14, dtype="bf16"),
}


def _scatter_ids(rank: np.ndarray, n: int, mult: int, add: int) -> np.ndarray:
    """A fixed bijection of [0, n) (x -> (mult x + add) mod n with mult
    coprime to n), so that the highest-weight ranks land on unrelated ids."""
    while math.gcd(mult, n) != 1:
        mult += 2
    return ((rank.astype(np.uint64) * np.uint64(mult) + np.uint64(add)) % np.uint64(n)).astype(np.uint32)


def powerlaw_ranks(u: np.ndarray, n: int, gamma: float) -> np.ndarray:
    """Vertex ranks drawn with probability density proportional to
    (x + 1)^(-1 / (gamma - 1)) on [0, n) (the expected-degree sequence of a
    Chung-Lu graph whose degrees follow a power law of exponent gamma), by
    inverting the continuous distribution function at the uniforms u."""
    beta = 1.0 / (gamma - 1.0)
    e = 1.0 - beta
    if abs(e) < 1e-9:   # density 1 / (x + 1): the distribution function is logarithmic
        x = (n + 1.0) ** u - 1.0
    else:
        lo, hi = 1.0, (n + 1.0) ** e
        x = (lo + u * (hi - lo)) ** (1.0 / e) - 1.0
    return np.minimum(x.astype(np.int64), n - 1)


def wide_graph(spec: WideSpec, chunk: int = 1 << 24):
    """(head, rel, tail) uint32 arrays of spec.m triples, drawn in chunks
    from one generator: heads and tails from power laws over scattered ids,
    relations by rank."""
    rng = np.random.Generator(np.random.PCG64(spec.seed))
    head = np.empty(spec.m, np.uint32)
    rel = np.empty(spec.m, np.uint32)
    tail = np.empty(spec.m, np.uint32)
    for c0 in range(0, spec.m, chunk):
        c1 = min(spec.m, c0 + chunk)
        u = rng.random((3, c1 - c0))
        head[c0:c1] = _scatter_ids(powerlaw_ranks(u[0], spec.n, spec.out_gamma), spec.n, 2654435761, 12345)
        tail[c0:c1] = _scatter_ids(powerlaw_ranks(u[1], spec.n, spec.in_gamma), spec.n, 40503 * 65537, 777)
        rel[c0:c1] = np.minimum((spec.R * u[2] ** spec.rel_power).astype(np.int64), spec.R - 1)
    return head, rel, tail


def wide_embeddings(spec: WideSpec, chunk_rows: int = 1 << 22):
    """X [n][d], Y [R][d]: normal entries of variance 1/d, float32 (or
    bfloat16 bit patterns)."""
    return embeddings(spec.n, spec.R, EmbSpec(spec.d, spec.dtype, seed=spec.seed + 1), chunk_rows)


def wide_queries(head: np.ndarray, tail: np.ndarray, nq: int, seed: int):
    """Query pairs (s, t): the head of one uniformly drawn triple and the
    tail of another (sources and targets in proportion to their degrees)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    i = rng.integers(0, len(head), nq)
    j = rng.integers(0, len(tail), nq)
    return head[i].astype(np.uint32), tail[j].astype(np.uint32)


def wide_subgraph(head, rel, tail, s: int, t: int):
    """The triples any three-hop path s -> a -> b -> t can use: the out-edges
    of s, the out-edges of its out-neighbours and the in-edges of t."""
    first = head == s
    mids = np.unique(tail[first])
    keep = first | np.isin(head, mids) | (tail == t)
    return head[keep], rel[keep], tail[keep]
