"""CPU oracle for exact three-hop top-K path search over a typed knowledge graph.

TEST INFRASTRUCTURE ONLY.  The tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` use it; the product path (the HIP library
and its binding) never imports, calls or links anything here, and nothing
here imports the product.

Two independent implementations of the same plain definition:

* ``mhr_oracle.c`` (loaded through ctypes): FP64 brute force, OpenMP over
  queries.  Every walk s -> a -> b -> t is enumerated, scored and sorted.
* ``pyoracle`` : the same definition in pure Python loops over edge lists,
  for tiny graphs only.

The definition (what both compute):
  edge weight  scorer "distmult" (the default):
               w(u,r,v) = logsigmoid( sum_i (X[u,i]*Y[r,i])*X[v,i] )  in FP64,
               logsigmoid(x) = min(x,0) - log1p(exp(-|x|));
               scorer "transe_l1" (the paper's own score, section 3.3):
               w(u,r,v) = gamma - sum_i |(X[u,i] + Y[r,i]) - X[v,i]|  in FP64,
               gamma = 1.0 by default as in the paper;
  path score   S = w(s,r1,a) + w(a,r2,b) + w(b,r3,t), the exact sum rounded
               once to FP64, over walks of exactly three edges (the
               three-hop query of section 3.1);
  order        S descending, then a, b, r1, r2, r3 ascending;
  result       the first min(K, |P(s,t)|) paths (a ranked top-K list, as the
               generic multi-hop algorithm of section 5 returns).
Embeddings are read exactly: float32 values, or bfloat16 values widened to
float32, are converted to FP64 without rounding.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mhr_oracle.c")
_LIB = os.path.join(_HERE, "libmhr_oracle.so")

MAX_HOPS = 8
BEAM_DTYPE = np.dtype([("s", np.float64), ("len", np.uint32), ("v", np.uint32, (MAX_HOPS,)),
                       ("r", np.uint32, (MAX_HOPS,))], align=True)

PATH_DTYPE = np.dtype([("s", np.float64), ("a", np.uint32), ("b", np.uint32),
                       ("r1", np.uint32), ("r2", np.uint32), ("r3", np.uint32)],
                      align=True)


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (-O2, OpenMP).  Building the checker is
    not using it: the build step compiles it beside the HIP library."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        vp, u32, u64 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64
        lib.og_graph_build.restype = vp
        lib.og_graph_build.argtypes = [u32, u32, u64, vp, vp, vp]
        lib.og_graph_free.argtypes = [vp]
        lib.og_graph_edges.restype = u64
        lib.og_graph_edges.argtypes = [vp]
        lib.og_graph_export.argtypes = [vp, vp, vp, vp]
        lib.og_logsigmoid.restype = ctypes.c_double
        lib.og_logsigmoid.argtypes = [ctypes.c_double]
        lib.og_edge_weights.argtypes = [u32, vp, vp, u64, vp, vp, vp, vp, vp]
        lib.og_edge_weights_s.argtypes = [ctypes.c_int, ctypes.c_double, u32, vp, vp, u64, vp, vp, vp, vp, vp]
        lib.og_topk_s.restype = ctypes.c_int
        lib.og_topk_s.argtypes = [vp, ctypes.c_int, ctypes.c_double, u32, vp, vp, u32, vp, vp, vp, u32,
                                  ctypes.c_int, vp, vp, vp]
        lib.og_topk.restype = ctypes.c_int
        lib.og_topk.argtypes = [vp, u32, vp, vp, u32, vp, vp, vp, u32, ctypes.c_int,
                                vp, vp, vp]
        lib.og_beam.restype = ctypes.c_int
        lib.og_beam.argtypes = [vp, ctypes.c_int, ctypes.c_double, u32, vp, vp, u32, vp, vp, u32, u32, vp, vp, vp]
        lib.og_scan_topk.restype = ctypes.c_int
        lib.og_scan_topk.argtypes = [u32, vp, vp, u32, vp, vp, vp, u32, u32, ctypes.c_double, vp, vp]
        lib.og_max_threads.restype = ctypes.c_int
        lib.og_fsum.restype = ctypes.c_double
        lib.og_fsum.argtypes = [vp, ctypes.c_int]
        _lib = lib
    return _lib


SCORERS = {"distmult": 0, "transe_l1": 1}


def _scorer(name):
    if name not in SCORERS:
        raise ValueError(f"unknown scorer {name!r}")
    return SCORERS[name]


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def as_f32_table(t: np.ndarray, dtype: str) -> np.ndarray:
    """Stored embedding table -> float32 values (bfloat16 bit patterns are
    widened exactly)."""
    if dtype == "bf16":
        return (np.ascontiguousarray(t, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)
    return np.ascontiguousarray(t, dtype=np.float32)


def logsigmoid(x: float) -> float:
    return _load().og_logsigmoid(float(x))


def fsum(values) -> float:
    """The C oracle's correctly rounded sum (used for path scores)."""
    v = np.ascontiguousarray(values, dtype=np.float64)
    if len(v) > 8:
        raise ValueError("at most 8 terms")
    return _load().og_fsum(_ptr(v), len(v))


class Graph:
    """Canonical graph (sorted, identical triples removed) held by the C oracle."""

    def __init__(self, n, R, head, rel, tail):
        lib = _load()
        self.n, self.R = int(n), int(R)
        self._h = np.ascontiguousarray(head, dtype=np.uint32)
        self._r = np.ascontiguousarray(rel, dtype=np.uint32)
        self._t = np.ascontiguousarray(tail, dtype=np.uint32)
        self._g = lib.og_graph_build(self.n, self.R, len(self._h),
                                     _ptr(self._h), _ptr(self._r), _ptr(self._t))
        if not self._g:
            raise ValueError("bad edge list (id out of range) or out of memory")
        self.m = int(lib.og_graph_edges(self._g))

    def __del__(self):
        if getattr(self, "_g", None) and _lib is not None:
            _lib.og_graph_free(self._g)
            self._g = None

    def csr(self):
        rp = np.empty(self.n + 1, np.uint64)
        t = np.empty(self.m, np.uint32)
        r = np.empty(self.m, np.uint32)
        _load().og_graph_export(self._g, _ptr(rp), _ptr(t), _ptr(r))
        return rp, t, r

    def beam(self, X, Y, src, dst, H, K, scorer: str = "distmult", gamma: float = 1.0):
        """The generic multi-hop search of section 5 (level-by-level
        expansion, cycles excluded, paths to the target recorded as found,
        the best K children of each parent passed on): per query the best K
        recorded paths of at most H edges.  Returns (paths [nq][K] of
        BEAM_DTYPE, count [nq], recorded [nq])."""
        X = np.ascontiguousarray(X, np.float32)
        Y = np.ascontiguousarray(Y, np.float32)
        src = np.ascontiguousarray(src, np.uint32)
        dst = np.ascontiguousarray(dst, np.uint32)
        nq = len(src)
        out = np.zeros((nq, K), BEAM_DTYPE)
        cnt = np.zeros(nq, np.uint32)
        rec = np.zeros(nq, np.uint64)
        rc = _load().og_beam(self._g, _scorer(scorer), float(gamma), X.shape[1], _ptr(X), _ptr(Y), nq, _ptr(src),
                             _ptr(dst), int(H), int(K), _ptr(out), _ptr(cnt), _ptr(rec))
        if rc != 0:
            raise ValueError("oracle beam search failed (bad argument or out of memory)")
        return out, cnt, rec

    def edge_weights(self, X, Y, u, r, v, scorer: str = "distmult", gamma: float = 1.0):
        """(x, w) of arbitrary edges: the scorer's raw value (DistMult score
        or L1 distance) and the edge weight, in FP64."""
        X = np.ascontiguousarray(X, np.float32)
        Y = np.ascontiguousarray(Y, np.float32)
        u = np.ascontiguousarray(u, np.uint32)
        r = np.ascontiguousarray(r, np.uint32)
        v = np.ascontiguousarray(v, np.uint32)
        x = np.empty(len(u), np.float64)
        w = np.empty(len(u), np.float64)
        _load().og_edge_weights_s(_scorer(scorer), float(gamma), X.shape[1], _ptr(X), _ptr(Y), len(u),
                                  _ptr(u), _ptr(r), _ptr(v), _ptr(x), _ptr(w))
        return x, w

    def topk(self, X, Y, src, dst, k, nthreads: int = 0, scorer: str = "distmult", gamma: float = 1.0):
        """Top-K paths for each query.  X, Y: float32 tables (use
        ``as_f32_table`` for bfloat16 storage).  k: scalar or per-query array.
        Returns (paths[nq][kmax] structured array, count[nq], total[nq])."""
        X = np.ascontiguousarray(X, np.float32)
        Y = np.ascontiguousarray(Y, np.float32)
        if X.ndim != 2 or Y.ndim != 2 or X.shape[1] != Y.shape[1]:
            raise ValueError("embedding tables must be [n][d] and [R][d]")
        if X.shape[0] != self.n or Y.shape[0] != self.R:
            raise ValueError("embedding table row counts do not match the graph")
        src = np.ascontiguousarray(src, np.uint32)
        dst = np.ascontiguousarray(dst, np.uint32)
        nq = len(src)
        kk = np.broadcast_to(np.asarray(k, dtype=np.uint32), (nq,)).copy()
        kmax = int(kk.max()) if nq else 1
        out = np.zeros((nq, kmax), PATH_DTYPE)
        cnt = np.zeros(nq, np.uint32)
        tot = np.zeros(nq, np.uint64)
        rc = _load().og_topk_s(self._g, _scorer(scorer), float(gamma), X.shape[1], _ptr(X), _ptr(Y), nq,
                               _ptr(src), _ptr(dst), _ptr(kk), kmax, int(nthreads), _ptr(out), _ptr(cnt),
                               _ptr(tot))
        if rc != 0:
            raise ValueError("oracle query failed (bad id, k out of range, or out of memory)")
        return out, cnt, tot


def scan_topk(X, Y, head, rel, cand, K, gamma=1.0):
    """Candidate scan of the paper's Turing-award pipeline (section 3.3):
    for each query q, the TransE-L1 score gamma - |X[head[q]] + Y[rel[q]] -
    X[c]|_1 (FP64) of every candidate c in `cand`, and the best min(K,
    len(cand)) under (score descending, id ascending).  Returns (ids
    [nq][K], scores [nq][K]); unused slots hold 0xFFFFFFFF and -inf."""
    X = np.ascontiguousarray(X, np.float32)
    Y = np.ascontiguousarray(Y, np.float32)
    head = np.ascontiguousarray(head, np.uint32)
    rel = np.ascontiguousarray(rel, np.uint32)
    cand = np.ascontiguousarray(cand, np.uint32)
    nq = len(head)
    ids = np.empty((nq, K), np.uint32)
    sc = np.empty((nq, K), np.float64)
    if _load().og_scan_topk(X.shape[1], _ptr(X), _ptr(Y), nq, _ptr(head), _ptr(rel), _ptr(cand), len(cand),
                            int(K), float(gamma), _ptr(ids), _ptr(sc)) != 0:
        raise MemoryError("oracle scan: allocation failed")
    return ids, sc


def turing_pipeline(X, Y, persons, universities, award, field, r_award, r_works, r_affil, K, gamma=1.0):
    """The three hops of the paper's pipeline (section 3.2, the simple
    algorithm; section 3.3 for the scores):
      1. score every person against (award + r_award) and keep the top K;
      2. score those K against (field + r_works) and rank them by it;
      3. for each of them, in that order, score every university against
         (person + r_affil) and keep the top K.
    Returns (hop1 ids/scores [K], hop2 ids/scores [K], hop3 ids/scores [K][K])."""
    h1_id, h1_s = scan_topk(X, Y, [award], [r_award], persons, K, gamma)
    top = h1_id[0][h1_id[0] != 0xFFFFFFFF]
    h2_id, h2_s = scan_topk(X, Y, [field], [r_works], top, K, gamma)
    ranked = h2_id[0][h2_id[0] != 0xFFFFFFFF]
    h3_id, h3_s = scan_topk(X, Y, ranked, np.full(len(ranked), r_affil, np.uint32), universities, K, gamma)
    return (h1_id[0], h1_s[0]), (h2_id[0], h2_s[0]), (h3_id, h3_s)


def max_threads() -> int:
    return int(_load().og_max_threads())
