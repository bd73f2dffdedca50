"""Helpers shared by the GPU parity tests: building inputs from the seeded
generators, running the HIP path through the binding, running the CPU
oracle, and comparing the two result by result."""

from __future__ import annotations

import sys

import numpy as np

import kgsynth
import oracle

REL_TOL = 1e-5          # |S_gpu - S_64| <= 1e-5 |S_64| (FP32 scores)
ORACLE_SLACK = 1e-13    # the FP64 oracle's own rounding, added to err_bound


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def workload(name):
    cfg = kgsynth.CONFIGS[name]
    h, r, t = kgsynth.make_graph(cfg.graph)
    X, Y = kgsynth.embeddings(cfg.graph.n, cfg.graph.R, cfg.emb)
    s, d, k = kgsynth.queries(h, cfg.graph.n, cfg.query)
    return cfg, (h, r, t), (X, Y), (s, d, k)


def gpu_graph(n, R, h, r, t, X, Y, dtype="f32"):
    import torch
    import paper_2406_07727_amd as mhr
    g = mhr.Graph(h, r, t, n, R)
    if dtype == "bf16":
        Xd = torch.from_numpy(np.ascontiguousarray(X).view(np.int16)).cuda()
        Yd = torch.from_numpy(np.ascontiguousarray(Y).view(np.int16)).cuda()
    else:
        Xd = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).cuda()
        Yd = torch.from_numpy(np.ascontiguousarray(Y, dtype=np.float32)).cuda()
    g.set_embeddings(Xd, Yd, dtype=dtype)
    return g


def run_gpu(g, s, d, k, k_max=None, opts=None):
    import torch
    res = g.topk(s, d, k, k_max=k_max, opts=opts)
    torch.cuda.synchronize()
    return res.to_numpy()


def run_oracle(n, R, h, r, t, X, Y, s, d, k, dtype="f32"):
    og = oracle.Graph(n, R, h, r, t)
    return og.topk(oracle.as_f32_table(X, dtype), oracle.as_f32_table(Y, dtype), s, d, k)


def _runs(flags):
    """Split positions into maximal runs joined by the precision-tie flag."""
    runs, cur = [], [0]
    for i in range(1, len(flags)):
        if flags[i - 1] & 2:
            cur.append(i)
        else:
            runs.append(cur)
            cur = [i]
    runs.append(cur)
    return runs


def compare(gpu, orc, queries=None, rel_tol=REL_TOL):
    """Asserts GPU == oracle on every query: counts, totals, the ranked ids
    (permutations allowed only inside runs flagged as precision ties), and
    each score within rel_tol and within its own error bound."""
    gp, gc, gt, gs = gpu
    op, oc, ot = orc
    nq = len(gc) if queries is None else len(queries)
    ties = 0
    for qi in range(nq):
        q = qi if queries is None else queries[qi]
        assert gs[q] in (0, 4), f"query {q}: status {gs[q]}"
        assert int(gc[q]) == int(oc[qi]), f"query {q}: count {gc[q]} vs {oc[qi]}"
        assert int(gt[q]) == int(ot[qi]), f"query {q}: total {gt[q]} vs {ot[qi]}"
        c = int(gc[q])
        if c == 0:
            continue
        g = gp[q][:c]
        o = op[qi][:c]
        gid = list(zip(g["a"].tolist(), g["b"].tolist(), g["r1"].tolist(), g["r2"].tolist(), g["r3"].tolist()))
        oid = list(zip(o["a"].tolist(), o["b"].tolist(), o["r1"].tolist(), o["r2"].tolist(), o["r3"].tolist()))
        if gid != oid:
            runs = _runs(g["flags"])
            for ri, run in enumerate(runs):
                gs_ = set(gid[i] for i in run)
                os_ = set(oid[i] for i in run)
                last_tied = ri == len(runs) - 1 and (g["flags"][run[-1]] & 2)
                if gs_ != os_ and not last_tied:
                    raise AssertionError(f"query {q}: ranked paths differ at {run}: {sorted(gs_)} vs {sorted(os_)}")
                ties += len(run) > 1
        osc = o["s"].astype(np.float64)
        gsc = g["score"].astype(np.float64)
        err = np.abs(gsc - osc)
        assert np.all(err <= rel_tol * np.abs(osc)), f"query {q}: score error {err.max()}"
        assert np.all(err <= g["err_bound"].astype(np.float64) + ORACLE_SLACK), \
            f"query {q}: error {err.max()} above its bound {g['err_bound'].max()}"
    return ties
