"""Training and inference of the learned frontier pruner (include/mhr.h).

Training.  For a batch of training queries:
1. The exact search's top-K labels the candidates: a candidate is positive
   when its vertex is the a (first hop) or the b (second hop) of one of the
   exact top-K paths.
2. All positives, and about ``neg_per_hop`` negatives per hop and query, are
   the batch's samples.
3. The network is trained on them with binary cross-entropy, weighting the
   positives by the batch's negative/positive ratio, and with Adam.

Inference.
1. Enumerate the candidates and compute their logits.
2. Keep the top ``keep_permille`` of each query's candidates per hop.
3. Run the exact search restricted to the kept first and last pairs.
4. Answer with the unrestricted exact search every query that fails the
   confidence test: fewer than K paths found, or a kept share of the
   predicted mass below ``tau`` at either hop.

Every step of both runs in the library's kernels.  Training is one library
call (mhr_pruner_train); for inference this module sequences the calls and
sizes buffers from the counts the kernels report.
"""

from __future__ import annotations

import ctypes
import time

import numpy as np

from . import (Graph, Pruner, TopK, TrainOpts, _check, _dev_u32, _lib, _ptr, _stream_ptr, _torch, candidates,
               select)


def init_params(dim: int, hidden: int, seed: int) -> np.ndarray:
    """He-normal weights (fan-in), zero biases, as one flat FP32 vector."""
    rng = np.random.Generator(np.random.PCG64(seed))
    W1 = rng.normal(0.0, np.sqrt(2.0 / (4 * dim)), (hidden, 4 * dim))
    W2 = rng.normal(0.0, np.sqrt(2.0 / hidden), (hidden, hidden))
    w3 = rng.normal(0.0, np.sqrt(1.0 / hidden), hidden)
    z = np.zeros(hidden)
    return np.concatenate([W1.ravel(), z, W2.ravel(), z, w3, [0.0]]).astype(np.float32)


class LearnedPruner:
    def __init__(self, graph: Graph, dim: int, hidden: int = 512, seed: int = 1):
        self.graph = graph
        self.net = Pruner(dim, hidden)
        self.net.set_params(init_params(dim, hidden, seed))
        self.seed = seed

    # ---- training -----------------------------------------------------------
    def samples(self, src, dst, K: int, neg_per_hop: int, seed: int):
        """Labelled samples of one query batch: (q, v, r, label, src, dst)
        device tensors, q indexing the batch."""
        torch = _torch()
        g = self.graph
        s, d = _dev_u32(src), _dev_u32(dst)
        nq = s.numel()
        exact = g.topk(s, d, K)
        c = candidates(g, s, d)
        pos = torch.empty(max(c.n_entries, 1), dtype=torch.uint8, device="cuda")
        st = _stream_ptr()
        _check(_lib.mhr_pruner_label(g._h, nq, _ptr(s), _ptr(d), _ptr(c.entry_off), _ptr(exact.paths),
                                     _ptr(exact.count), K, _ptr(pos), st), "mhr_pruner_label")
        n = c.n
        sq = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
        sv = torch.empty_like(sq)
        sr = torch.empty_like(sq)
        sl = torch.empty(max(n, 1), dtype=torch.float32, device="cuda")
        ns = torch.zeros(1, dtype=torch.int64, device="cuda")
        wsb = int(_lib.mhr_pruner_sample_workspace(nq, n))
        ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device="cuda")
        _check(_lib.mhr_pruner_sample(nq, _ptr(c.cand_off), _ptr(c.cand_split), n, _ptr(c.q), _ptr(c.v), _ptr(c.r),
                                      _ptr(c.e), _ptr(pos), int(neg_per_hop), int(seed), _ptr(sq), _ptr(sv), _ptr(sr),
                                      _ptr(sl), _ptr(ns), _ptr(ws), ws.numel(), st), "mhr_pruner_sample")
        m = int(ns.item())
        return sq[:m], sv[:m], sr[:m], sl[:m], s, d

    def fit(self, src, dst, K: int = 32, batch_queries: int = 4096, step_samples: int = 65536, epochs: int = 1,
            lr: float = 1e-3, neg_per_hop: int = 64, seed: int = 1, log=None):
        """Trains on the queries (host or device arrays) with the library's
        whole-run call (mhr_pruner_train); returns the loss per step."""
        o = TrainOpts()
        o.k, o.batch_queries, o.step_samples, o.epochs = int(K), int(batch_queries), int(step_samples), int(epochs)
        o.neg_per_hop, o.lr, o.seed = int(neg_per_hop), float(lr), int(seed)
        losses = self.net.train(self.graph, src, dst, o)
        if log and losses:
            log(f"trained {len(losses)} steps: loss {np.mean(losses[:3]):.4f} -> {np.mean(losses[-10:]):.4f}")
        return losses

    # ---- inference ----------------------------------------------------------
    def logits(self, c, chunk: int = 1 << 18):
        """The network's logits of every candidate of c (mhr_pruner_score)."""
        return self.net.score(self.graph, c.src, c.dst, c.q[:c.n], c.v[:c.n], c.r[:c.n], chunk=chunk)

    def search(self, src, dst, K: int, keep_permille: int = 100, tau: float = 0.5, scores=None,
               fallback: bool = True):
        """Pruned search with the exact search as fallback (fallback=False:
        the pruned result alone).  scores: ranking of the candidates (None =
        the network's logits).  Returns (TopK, stats)."""
        torch = _torch()
        g = self.graph
        s, d = _dev_u32(src), _dev_u32(dst)
        nq = s.numel()
        c = candidates(g, s, d)
        sc = self.logits(c) if scores is None else scores
        keep, mass = select(g, c, sc, keep_permille)
        res = g.topk_pruned(s, d, K, keep, c.entry_off)
        fb = torch.empty((4, nq), dtype=torch.int32, device="cuda")
        nfb_t = torch.zeros(1, dtype=torch.int32, device="cuda")
        st = _stream_ptr()
        _check(_lib.mhr_pruner_fallback(nq, _ptr(s), _ptr(d), None, K, _ptr(res.count), _ptr(res.status), _ptr(mass),
                                        float(tau), _ptr(fb[0]), _ptr(fb[1]), _ptr(fb[2]), _ptr(fb[3]), _ptr(nfb_t),
                                        st), "mhr_pruner_fallback")
        nfb = int(nfb_t.item()) if fallback else 0
        if nfb:
            ex = g.topk(fb[0][:nfb], fb[1][:nfb], K)
            _check(_lib.mhr_scatter_results(nfb, _ptr(fb[3]), K, _ptr(ex.paths), _ptr(ex.count), _ptr(ex.total),
                                            _ptr(ex.status), _ptr(res.paths), _ptr(res.count), _ptr(res.total),
                                            _ptr(res.status), st), "mhr_scatter_results")
        kept = int(keep[:c.n_entries].sum().item()) if c.n_entries else 0
        return res, {"queries": nq, "fallback": nfb, "candidates": c.n, "entries": c.n_entries, "entries_kept": kept}

    def baseline_scores(self, c, kind: str, seed: int = 0):
        """Rankings without the network: 'random' (uniform draws) or 'beam'
        (the candidate edge's own weight w(s, r1, a) or w(b, r3, t), as a
        per-level score beam keeps the best partial paths)."""
        torch = _torch()
        if kind == "random":
            rng = np.random.Generator(np.random.PCG64(seed))
            return torch.from_numpy(rng.random(c.n).astype(np.float32)).cuda()
        if kind == "beam":
            w = torch.empty(max(c.n, 1), dtype=torch.float32, device="cuda")
            _check(_lib.mhr_pruner_candidate_weights(self.graph._h, c.n, _ptr(c.src), _ptr(c.dst), _ptr(c.q),
                                                     _ptr(c.v), _ptr(c.r), _ptr(w), _stream_ptr()),
                   "mhr_pruner_candidate_weights")
            return w[:c.n]
        raise ValueError(kind)


def path_sets(paths, count):
    """Per query, the set of its returned paths (a, b, r1, r2, r3)."""
    out = []
    for q in range(len(count)):
        p = paths[q][:count[q]]
        out.append(set(zip(p["a"].tolist(), p["b"].tolist(), p["r1"].tolist(), p["r2"].tolist(), p["r3"].tolist())))
    return out


def topk_recall(exact, approx):
    """Mean over queries with at least one path of |approx ∩ exact| / |exact|
    (exact, approx: to_numpy() results)."""
    es = path_sets(exact[0], exact[1])
    as_ = path_sets(approx[0], approx[1])
    r = [len(a & e) / len(e) for e, a in zip(es, as_) if e]
    return float(np.mean(r)) if r else 1.0
