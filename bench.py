"""Benchmark: exact three-hop top-K path search on one MI355X.

One step = one batched top-K call over the whole query batch (planning,
gather/score, merge with compensated rescoring, and the exhaustive pass when
needed), with the graph, embeddings and queries already resident in HBM.

Workload (default): Chung-Lu typed KG (exponent 2.1) with 1M vertices,
16 relations and 20M edges, d=128 FP32 embeddings ~N(0, 1/d), 1,024 queries
with degree-proportional sources and uniform targets, K=32.  Synthetic,
seeded; it stands in for WikiKG90Mv2.

Prints one JSON line.  value = scored three-hop paths per second, where a
batch scores sum_q |P(s_q, t_q)| paths (the path counts the GPU reports,
equal to the oracle's on the sampled queries).
"""

from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "scored 3-hop paths/s and queries/s at K=32 (exact top-K vs FP64 oracle)"
HBM_PEAK_GBS = 8000.0

# HBM bytes of one gather launch on the realistic workload, from two
# rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch) of this
# script, each scaled by what the same counter reads for a plain 1 GiB device
# copy (bench.py --calibrate-copy): FETCH_SIZE read 524302 KiB for 1048576 KiB
# fetched (scale 2.0), WRITE_SIZE read 1048576 KiB (scale 1.0).  Valid only
# for the kernel sources they were taken on (sha256 over the query sources).
TRAFFIC = {
    "sources_sha256": "0b9007da003a26f479831b45210ce6cceddd52eb1aa1b814942f2af17b7531d3",
    "fetch_kib": 464367.9,
    "write_kib": 3019.1,
    "fetch_scale": 2.0,
    "write_scale": 1.0,
}
KERNEL_SOURCES = ("paper_2406_07727_amd/csrc/mhr_query.hip", "paper_2406_07727_amd/csrc/mhr_device.h",
                  "paper_2406_07727_amd/csrc/mhr_internal.h")


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(config):
    """HBM bytes per gather launch from the committed counter run, or None
    when the kernel sources changed since (or for another workload)."""
    if config != "realistic" or TRAFFIC["sources_sha256"] != kernel_sources_sha256():
        return None
    return int(TRAFFIC["fetch_kib"] * 1024 * TRAFFIC["fetch_scale"] + TRAFFIC["write_kib"] * 1024 * TRAFFIC["write_scale"])


def log(msg):
    print(msg, file=sys.stderr, flush=True)


class HipEvents:
    """hipEvent_t handles through the HIP runtime (timing on the stream the
    kernels run on)."""

    def __init__(self):
        self.hip = ctypes.CDLL("libamdhip64.so.7")  # the runtime torch already loaded
        self.hip.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
        self.hip.hipEventSynchronize.argtypes = [ctypes.c_void_p]
        self.hip.hipEventDestroy.argtypes = [ctypes.c_void_p]
        self.hip.hipEventRecord.argtypes = [ctypes.c_void_p, ctypes.c_void_p]

    def create(self):
        e = ctypes.c_void_p()
        assert self.hip.hipEventCreate(ctypes.byref(e)) == 0
        return e

    def elapsed_ms(self, a, b):
        assert self.hip.hipEventSynchronize(b) == 0
        ms = ctypes.c_float()
        assert self.hip.hipEventElapsedTime(ctypes.byref(ms), a, b) == 0
        return float(ms.value)


def gather_bytes(csr_out, csr_in, src, dst, d, elem, k=None, totals=None):
    """Algorithmic bytes of one gather launch, two ways, and the matched
    middle pairs: (layout_bytes, model_bytes, matches).

    Both follow the plan the library uses (the cheaper of backward and
    forward meet-in-the-middle) and count one embedding row (d * elem B) per
    distinct list-side and scan-side vertex on some path, plus s and t.

    layout_bytes, this library's pair layout: list row L entries (col +
    mask, 8 B) and the row_ptr pairs of those rows (8 B); probe row P
    entries (8 B); scanned entries C (col, 4 B); matched entries M (mask,
    4 B).

    model_bytes, the per-query model of the hot-path scope's measurement
    plan (one 4-byte entry per triple): 8 (2 + L) of row_ptr pairs, 4 bytes
    per triple of s's out-row, t's in-row and the scanned rows, the
    embedding rows, and 16 bytes per returned path (min(k, |P|), when k and
    the path totals are given)."""
    orp, ocol, omask = csr_out
    irp, icol, imask = csr_in
    odeg = np.diff(orp).astype(np.int64)
    ideg = np.diff(irp).astype(np.int64)
    # triples per row (a pair entry carries one triple per relation bit)
    ocs = np.concatenate([[0], np.cumsum(np.bitwise_count(omask).astype(np.int64))])
    ics = np.concatenate([[0], np.cumsum(np.bitwise_count(imask).astype(np.int64))])
    otrip = ocs[orp[1:].astype(np.int64)] - ocs[orp[:-1].astype(np.int64)]
    itrip = ics[irp[1:].astype(np.int64)] - ics[irp[:-1].astype(np.int64)]
    total = model = 0
    matches = 0
    for qi, (s, t) in enumerate(zip(src.tolist(), dst.tolist())):
        bl = icol[irp[t]:irp[t + 1]]
        cost_b = int(ideg[bl].sum())
        al = ocol[orp[s]:orp[s + 1]]
        cost_f = int(odeg[al].sum())
        fwd = cost_f < cost_b
        if fwd:
            lst, rp, col, probe, trip = al, orp, ocol, icol[irp[t]:irp[t + 1]], otrip
        else:
            lst, rp, col, probe, trip = bl, irp, icol, ocol[orp[s]:orp[s + 1]], itrip
        L, P = len(lst), len(probe)
        out_paths = 0
        if k is not None and totals is not None:
            kq = int(k[qi]) if np.ndim(k) else int(k)
            out_paths = min(kq, int(totals[qi]))
        ends_trip = int(otrip[s]) + int(itrip[t])
        if L == 0 or P == 0:
            total += 16 * L + 8 * P
            model += 8 * (2 + L) + 4 * ends_trip + 16 * out_paths
            continue
        starts, ends = rp[lst].astype(np.int64), rp[lst + 1].astype(np.int64)
        lens = ends - starts
        C = int(lens.sum())
        if C:
            idx = np.repeat(starts - np.concatenate([[0], np.cumsum(lens)[:-1]]), lens) + np.arange(C)
            scanned = col[idx]
            pos = np.searchsorted(probe, scanned)
            pos[pos >= P] = 0
            hit = probe[pos] == scanned
            M = int(hit.sum())
            ystar = len(np.unique(scanned[hit]))
            rowid = np.repeat(np.arange(L), lens)
            xstar = len(np.unique(rowid[hit]))
        else:
            M = ystar = xstar = 0
        matches += M
        emb = d * elem * (xstar + ystar + 2)
        total += 16 * L + 8 * P + 4 * C + 4 * M + emb
        model += 8 * (2 + L) + 4 * (ends_trip + int(trip[lst].sum())) + emb + 16 * out_paths
    return total, model, matches


def gather_byte_parts(csr_out, csr_in, src, dst, d, elem):
    """The terms of gather_bytes separately: list rows (16 B per entry with
    its row bounds), probe rows (8 B), scanned columns (4 B), middle-edge
    masks of matches (4 B) and embedding rows."""
    orp, ocol, _ = csr_out
    irp, icol, _ = csr_in
    odeg = np.diff(orp).astype(np.int64)
    ideg = np.diff(irp).astype(np.int64)
    out = {"list_rows": 0, "probe_rows": 0, "scan": 0, "match_masks": 0, "emb": 0}
    for s, t in zip(src.tolist(), dst.tolist()):
        bl = icol[irp[t]:irp[t + 1]]
        al = ocol[orp[s]:orp[s + 1]]
        fwd = int(odeg[al].sum()) < int(ideg[bl].sum())
        if fwd:
            lst, rp, col, probe = al, orp, ocol, icol[irp[t]:irp[t + 1]]
        else:
            lst, rp, col, probe = bl, irp, icol, ocol[orp[s]:orp[s + 1]]
        L, P = len(lst), len(probe)
        out["list_rows"] += 16 * L
        out["probe_rows"] += 8 * P
        if L == 0 or P == 0:
            continue
        starts, ends = rp[lst].astype(np.int64), rp[lst + 1].astype(np.int64)
        lens = ends - starts
        C = int(lens.sum())
        if not C:
            continue
        idx = np.repeat(starts - np.concatenate([[0], np.cumsum(lens)[:-1]]), lens) + np.arange(C)
        scanned = col[idx]
        pos = np.searchsorted(probe, scanned)
        pos[pos >= P] = 0
        hit = probe[pos] == scanned
        rowid = np.repeat(np.arange(L), lens)
        out["scan"] += 4 * C
        out["match_masks"] += 4 * int(hit.sum())
        out["emb"] += d * elem * (len(np.unique(scanned[hit])) + len(np.unique(rowid[hit])) + 2)
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg, h, r, t, X, Y, s, d, k, nsample, gpu_result=None, per_core_queries=32, scorer="distmult"):
    """The FP64 oracle timed on the host cores (OpenMP over queries, threads
    pinned close to cores), on the first nsample queries; then a
    single-thread run on the first per_core_queries for a per-core rate.
    When gpu_result is given, the GPU's results on the sampled queries are
    compared with the oracle's, path by path."""
    os.environ.setdefault("OMP_PROC_BIND", "close")
    os.environ.setdefault("OMP_PLACES", "cores")
    import oracle
    from tests.parity import parity_summary, run_oracle
    oracle.build(force=False)
    og = oracle.Graph(cfg.graph.n, cfg.graph.R, h, r, t)
    threads = oracle.max_threads()
    t0 = time.perf_counter()
    orc = run_oracle(cfg.graph.n, cfg.graph.R, h, r, t, X, Y, s[:nsample], d[:nsample], k[:nsample],
                     cfg.emb.dtype, og=og, scorer=scorer)
    dt = time.perf_counter() - t0
    npaths = int(orc.total.sum())
    parity = None
    if gpu_result is not None:
        parity = parity_summary(gpu_result, orc, range(nsample))
        if parity["first_mismatch"] is None:
            del parity["first_mismatch"]
    n1 = min(per_core_queries, nsample)
    Xf = oracle.as_f32_table(X, cfg.emb.dtype)
    Yf = oracle.as_f32_table(Y, cfg.emb.dtype)
    t1 = time.perf_counter()
    _, _, tot1 = og.topk(Xf, Yf, s[:n1], d[:n1], k[:n1], nthreads=1, scorer=scorer)
    dt1 = time.perf_counter() - t1
    out = {"value": npaths / dt, "unit": "paths/s", "cores": int(threads), "kind": "oracle",
           "sample": f"first {nsample} of the {len(s)} queries (K={int(k[0])}); FP64 brute-force enumeration, "
                     f"OpenMP over queries (OMP_PROC_BIND={os.environ['OMP_PROC_BIND']}, "
                     f"OMP_PLACES={os.environ['OMP_PLACES']}); {dt:.1f} s; {npaths} paths; "
                     f"queries/s {nsample / dt:.2f}",
           "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
           "queries_per_s": nsample / dt,
           "per_core": {"paths_per_s": float(tot1.sum()) / dt1, "queries_per_s": n1 / dt1, "queries": n1,
                        "seconds": round(dt1, 2)}}
    return out, parity


def calibrate_copy(nbytes=1 << 30, reps=3):
    """A plain device copy of known size (torch's copy kernel, nbytes read and
    nbytes written per launch): the reference that scales the FETCH_SIZE and
    WRITE_SIZE counters of a profiled run into bytes."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "launches": reps}), flush=True)


def run_turing(args):
    """The paper's three-hop award pipeline as a candidate scan (sections
    3.2-3.3): 539,603 persons, 89,689 universities, K = 50, d = 8, over a
    91,230,610-entity synthetic table (the shape of WikiKG90Mv2 as the paper
    ran it).  One step = one pipeline (npipe = 1), and a batched form of
    independent pipelines in one call.  Exactness: the FP64 oracle's
    pipeline is compared bit for bit."""
    import torch
    import kgsynth
    import paper_2406_07727_amd as mhr
    spec = kgsynth.TURING["turing"]
    t0 = time.perf_counter()
    X, Y, persons, univ, award, field, (ra, rw, rf) = kgsynth.turing_workload(spec)
    log(f"turing inputs generated in {time.perf_counter() - t0:.1f} s")
    torch.cuda.set_device(0)
    Xd = torch.from_numpy(X).cuda()
    Yd = torch.from_numpy(Y).cuda()
    ev = HipEvents()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    K = spec.k
    scores_per_pipe = len(persons) + K + K * len(univ)
    results = {}
    for npipe in (1, args.turing_batch):
        rng = np.random.Generator(np.random.PCG64(spec.seed + 7))
        awards = np.concatenate([[award], rng.integers(0, spec.n, npipe - 1)]).astype(np.uint32)
        fields = np.concatenate([[field], rng.integers(0, spec.n, npipe - 1)]).astype(np.uint32)
        pl = mhr.ScanPipeline(Xd, Yd, persons, univ, K, npipe=npipe)
        aw = torch.from_numpy(awards.view(np.int32)).cuda()
        fi = torch.from_numpy(fields.view(np.int32)).cuda()
        for _ in range(max(1, args.warmup)):
            pl.run(aw, fi, ra, rw, rf)
        torch.cuda.synchronize()
        e0, e1 = ev.create(), ev.create()
        assert ev.hip.hipEventRecord(e0, stream) == 0
        for _ in range(args.steps):
            pl.run(aw, fi, ra, rw, rf)
        assert ev.hip.hipEventRecord(e1, stream) == 0
        ms = ev.elapsed_ms(e0, e1) / args.steps
        results[npipe] = {"ms_per_call": ms, "pipelines_per_s": npipe / (ms * 1e-3),
                          "candidate_scores_per_s": npipe * scores_per_pipe / (ms * 1e-3)}
        log(f"turing npipe={npipe}: {results[npipe]}")
        if npipe == 1:
            pl1 = pl
    # distinct HBM bytes of one pipeline: each candidate's id and row once
    # per hop (rows re-read by later queries of a hop are cache hits)
    row = spec.d * 4
    nbytes = len(persons) * (4 + row) + K * (4 + row) + len(univ) * (4 + row) + 3 * K * 12
    ms1 = results[1]["ms_per_call"]
    achieved = nbytes / (ms1 * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": "scan_chunk_kernel (whole pipeline)",
            "bytes_per_launch": int(nbytes), "kernel_ms": round(ms1, 4)}
    parity = cpu = None
    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        t1 = time.perf_counter()
        (h1, s1), (h2, s2), (h3, s3) = oracle.turing_pipeline(X, Y, persons, univ, award, field, ra, rw, rf, K)
        dt = time.perf_counter() - t1
        same = (np.array_equal(pl1.hop1_id[0].cpu().numpy().view(np.uint32), h1) and
                np.array_equal(pl1.hop1_score[0].cpu().numpy(), s1) and
                np.array_equal(pl1.hop2_id[0].cpu().numpy().view(np.uint32), h2) and
                np.array_equal(pl1.hop2_score[0].cpu().numpy(), s2) and
                np.array_equal(pl1.hop3_id[0].cpu().numpy().view(np.uint32), h3) and
                np.array_equal(pl1.hop3_score[0].cpu().numpy(), s3))
        parity = {"checked": 1, "mismatches": 0 if same else 1, "flagged_ties": 0}
        cpu = {"value": 1.0 / dt, "unit": "pipelines/s", "cores": oracle.max_threads(), "kind": "oracle",
               "sample": f"one pipeline, FP64 scan with OpenMP over queries; {dt:.2f} s", "cpu_model": cpu_model()}
    out = {"metric": "award-pipeline candidate scan (three hops, K=50, d=8): pipelines/s", "value":
           results[1]["pipelines_per_s"], "unit": "pipelines/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms1, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"turing: {spec.n} entities, d={spec.d} f32, {len(persons)} persons, "
                                  f"{len(univ)} universities, K={K}", "batched": {str(k): v for k, v in results.items()}},
           "roofline": roof, "cpu_baseline": cpu, "parity": parity}
    print(json.dumps(out), flush=True)


def run_wide(args):
    """Wide-relation knowledge graph at the paper's scale (section 4.1:
    91,230,610 entities, 1,387 relations, 601,062,811 triples, d = 8),
    TransE-L1 scores in FP64.  One step = one mhr_wide_topk_paths call over
    the batch (planning with its one synchronisation, frontier weights, the
    tile kernel, the merge).  Exactness: sampled queries are compared bit for
    bit with the oracle run on the union of their subgraphs (the triples
    their paths can use), which is also the CPU baseline."""
    import torch
    import kgsynth
    import paper_2406_07727_amd as mhr
    sp = kgsynth.WIDE[args.config]
    t0 = time.perf_counter()
    h, r, t = kgsynth.wide_graph(sp)
    log(f"wide graph drawn in {time.perf_counter() - t0:.1f} s ({sp.m} triples)")
    X, Y = kgsynth.wide_embeddings(sp)
    log(f"embeddings drawn ({time.perf_counter() - t0:.1f} s)")
    torch.cuda.set_device(0)
    dev = lambda a: torch.from_numpy(a.view(np.int32)).cuda()
    t1 = time.perf_counter()
    g = mhr.WideGraph(dev(h), dev(r), dev(t), sp.n, sp.R)
    torch.cuda.synchronize()
    ingest_s = time.perf_counter() - t1
    st = g.stats()
    log(f"ingest {ingest_s:.2f} s: {st}")
    g.set_embeddings(torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda(), gamma=1.0)
    K = 32
    src, dst = kgsynth.wide_queries(h, t, args.wide_queries, seed=sp.seed + 3)
    sd, dd = dev(src), dev(dst)
    wsb = g.workspace_size(sd, dd, K)
    ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device="cuda")
    log(f"{len(src)} queries, workspace {wsb / 2**20:.1f} MiB")
    ev = HipEvents()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for _ in range(max(1, args.warmup)):
        res = g.topk(sd, dd, K, workspace=ws)
    torch.cuda.synchronize()
    pe = [mhr.PhaseEvents(*(ev.create() for _ in range(4))) for _ in range(args.steps)]
    e0, e1 = ev.create(), ev.create()
    assert ev.hip.hipEventRecord(e0, stream) == 0
    for i in range(args.steps):
        res = g.topk(sd, dd, K, workspace=ws, events=pe[i])
    assert ev.hip.hipEventRecord(e1, stream) == 0
    ms = ev.elapsed_ms(e0, e1) / args.steps
    gather_ms = sum(ev.elapsed_ms(p.gather_begin, p.gather_end) for p in pe) / args.steps
    log(f"wide: {ms:.3f} ms per step, tile kernel {gather_ms:.3f} ms")
    w = res.work_numpy()
    p_np, cnt, tot, stat = res.to_numpy()
    # algorithmic bytes of the tile kernel, per query: every scanned entry
    # (4-byte id, 2-byte relation); the embedding rows of each matched
    # neighbour and of each distinct list vertex; the probe row's ids once per
    # tile when the kernel copies it to LDS (at most 2,048 entries and at most
    # twice the entries one tile scans), else per scanned entry the
    # neighbour's row bounds and one id of its row (12 bytes)
    d = sp.d
    short = (w["probe_len"] <= 2048) & (w["probe_len"] <= 2 * np.minimum(w["scanned"], 16384))
    nbytes = int(6 * w["scanned"].sum() + 4 * d * (w["matches"].sum() + w["distinct"].sum())
                 + (4 * w["probe_len"] * w["tiles"])[short].sum() + 12 * w["scanned"][~short].sum())
    achieved = nbytes / (gather_ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": "wide_gather_kernel",
            "bytes_per_launch": nbytes, "kernel_ms": round(gather_ms, 4)}
    paths = int(tot.sum())
    parity = cpu = None
    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        ns = min(args.cpu_sample or 32, len(src))
        qi = np.linspace(0, len(src) - 1, ns).astype(np.int64)
        t2 = time.perf_counter()
        first = np.isin(h, src[qi], kind="table")
        mids = np.unique(t[first])
        keep = first | np.isin(h, mids, kind="table") | np.isin(t, dst[qi], kind="table")
        og = oracle.Graph(sp.n, sp.R, h[keep], r[keep], t[keep])
        log(f"oracle subgraph: {int(keep.sum())} triples ({time.perf_counter() - t2:.1f} s)")
        t3 = time.perf_counter()
        op, oc, ot = og.topk(X, Y, src[qi], dst[qi], K, scorer="transe_l1", gamma=1.0)
        dt = time.perf_counter() - t3
        bad = 0
        for j, q in enumerate(qi):
            n = int(cnt[q])
            same = (int(tot[q]) == int(ot[j]) and n == int(oc[j]) and
                    np.array_equal(p_np[q][:n]["score"], op[j][:n]["s"]) and
                    all(np.array_equal(p_np[q][:n][f].astype(np.uint32), op[j][:n][f]) for f in ("a", "b", "r1", "r2", "r3")))
            bad += 0 if same else 1
        parity = {"checked": int(ns), "mismatches": bad, "flagged_ties": 0}
        cpu = {"value": ns / dt, "unit": "queries/s", "cores": oracle.max_threads(), "kind": "oracle",
               "sample": f"{ns} of the batch's queries on the union of their subgraphs, OpenMP over queries; "
                         f"{dt:.2f} s", "cpu_model": cpu_model()}
        log(f"wide parity {parity}, oracle {ns / dt:.1f} queries/s")
    out = {"metric": "exact three-hop top-K (K=32) on a paper-scale knowledge graph: queries/s", "value":
           len(src) / (ms * 1e-3), "unit": "queries/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": f"{args.config}: {sp.n} entities, {sp.R} relations, {sp.m} triples drawn "
                                  f"({st['num_triples']} distinct), d={sp.d} f32, TransE-L1, {len(src)} queries, K={K}",
                      "paths_per_batch": paths, "paths_per_s": paths / (ms * 1e-3), "ingest_s": round(ingest_s, 2),
                      "scanned_entries": int(w["scanned"].sum()), "matches": int(w["matches"].sum())},
           "roofline": roof, "cpu_baseline": cpu, "parity": parity}
    print(json.dumps(out), flush=True)


def run_beam(args, cfg, g, h, r, t, X, Y, s, d):
    """The generic multi-hop search (section 5: level by level, cycle
    exclusion, targets recorded early, the best K children of each parent
    carried to the next level) on the workload's graph and queries, scored
    in FP64; one step = one mhr_beam_search call over the batch.  A sample of
    queries is compared with the FP64 oracle's search (same vertex and
    relation sequences in the same order; DistMult scores to 1e-13, the
    device and host exp / log1p may differ in the last bit)."""
    import torch
    import oracle
    import paper_2406_07727_amd as mhr
    H, K = args.beam_hops, args.beam_k
    sd = torch.from_numpy(s.view(np.int32)).cuda()
    dd = torch.from_numpy(d.view(np.int32)).cuda()
    for _ in range(max(1, args.warmup)):
        res = g.beam(sd, dd, H, K)
    torch.cuda.synchronize()
    ev = HipEvents()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    e0, e1 = ev.create(), ev.create()
    assert ev.hip.hipEventRecord(e0, stream) == 0
    for _ in range(args.steps):
        res = g.beam(sd, dd, H, K)
    assert ev.hip.hipEventRecord(e1, stream) == 0
    ms = ev.elapsed_ms(e0, e1) / args.steps
    gp, gc, gr = mhr.beam_to_numpy(*res)
    log(f"beam H={H} K={K}: {ms:.3f} ms per step, {int(gr.sum())} paths recorded")
    parity = cpu = None
    if not args.no_cpu_baseline:
        oracle.build(force=False)
        ns = min(args.cpu_sample or 64, len(s))
        qi = np.linspace(0, len(s) - 1, ns).astype(np.int64)
        og = oracle.Graph(cfg.graph.n, cfg.graph.R, h, r, t)
        Xf, Yf = oracle.as_f32_table(X, cfg.emb.dtype), oracle.as_f32_table(Y, cfg.emb.dtype)
        t0 = time.perf_counter()
        op, oc, orr = og.beam(Xf, Yf, s[qi], d[qi], H, K, scorer=args.scorer, gamma=1.0)
        dt = time.perf_counter() - t0
        bad = 0
        for j, q in enumerate(qi):
            n = int(gc[q])
            same = n == int(oc[j]) and int(gr[q]) == int(orr[j])
            if same:
                for a, b in zip(gp[q][:n], op[j][:n]):
                    L = int(a["len"])
                    same = same and L == int(b["len"]) and np.array_equal(a["v"][:L], b["v"][:L]) \
                        and np.array_equal(a["r"][:L], b["r"][:L]) \
                        and abs(float(a["score"]) - float(b["s"])) <= 1e-13 * max(1.0, abs(float(b["s"])))
            bad += 0 if same else 1
        parity = {"checked": int(ns), "mismatches": bad}
        cpu = {"value": ns / dt, "unit": "queries/s", "cores": oracle.max_threads(), "kind": "oracle",
               "sample": f"{ns} of the batch's queries, the oracle's level-by-level search in FP64; {dt:.2f} s",
               "cpu_model": cpu_model()}
        log(f"beam parity {parity}; oracle {ns / dt:.1f} queries/s")
    out = {"metric": f"generic {H}-hop beam search (K={K}): queries/s", "value": len(s) / (ms * 1e-3),
           "unit": "queries/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"{args.config} graph: {cfg.graph.n} vertices, {cfg.graph.R} relations, "
                                  f"{cfg.graph.m} edges, d={cfg.emb.d} {cfg.emb.dtype}, {len(s)} queries, "
                                  f"{args.scorer}, H={H}, K={K}",
                      "paths_recorded": int(gr.sum())},
           "roofline": None, "cpu_baseline": cpu, "parity": parity}
    print(json.dumps(out), flush=True)


def run_pruner(args, cfg, g, h, s, d):
    """The learned-pruner form: train the network on exact-search labels,
    then answer the held-out batch with the pruned search (and the exact
    search as fallback) beside the exact search alone."""
    import torch
    import kgsynth
    import paper_2406_07727_amd as mhr
    from paper_2406_07727_amd.learned import LearnedPruner, topk_recall
    K = cfg.query.k
    s_tr, d_tr, _ = kgsynth.queries(h, cfg.graph.n, kgsynth.QuerySpec(args.train_queries, "degree", K, seed=15))
    lp = LearnedPruner(g, cfg.emb.d, args.hidden, seed=3)
    t0 = time.perf_counter()
    losses = lp.fit(s_tr, d_tr, K=K, step_samples=8192, epochs=1, lr=1e-3, seed=4, log=log)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(reps):
            out = fn()
        torch.cuda.synchronize()
        return out, (time.perf_counter() - t1) / reps

    exact, t_exact = timed(lambda: g.topk(s, d, K), args.steps)
    exn = exact.to_numpy()
    out = {"train_queries": args.train_queries, "hidden": args.hidden, "train_seconds": round(train_s, 1),
           "train_steps": len(losses), "loss_first": round(float(np.mean(losses[:5])), 4),
           "loss_last": round(float(np.mean(losses[-20:])), 4), "keep_permille": 100,
           "exact_queries_per_s": len(s) / t_exact}
    c = mhr.candidates(g, s, d)
    # the network over every frontier candidate of the held-out batch
    # (mhr_pruner_score); algorithmic flops: the candidate's share of the
    # first layer, the second layer and the output per candidate, the
    # endpoints' share per query and hop, the relations' share once
    dim, H = cfg.emb.d, args.hidden
    _, t_score = timed(lambda: lp.logits(c), args.steps)
    flops = c.n * 2 * (dim * H + H * H + H) + len(s) * 2 * 2 * (2 * dim) * H + cfg.graph.R * 2 * dim * H
    out["scoring"] = {"candidates": c.n, "ms": round(1e3 * t_score, 3), "candidates_per_s": c.n / t_score,
                      "tflop_per_s": round(flops / t_score / 1e12, 1),
                      "frac_bf16_peak": round(flops / t_score / 1e12 / 2500.0, 4)}
    for kind in ("net", "random", "beam"):
        sc = None if kind == "net" else lp.baseline_scores(c, kind, seed=5)
        res, st = lp.search(s, d, K, keep_permille=100, scores=sc, fallback=False)
        torch.cuda.synchronize()
        out[f"recall_{kind}_no_fallback"] = round(topk_recall(exn, res.to_numpy()), 4)
    # the confidence threshold: the smallest tau on a grid whose recall on a
    # validation split (queries disjoint from training and held-out, same
    # law) reaches 0.95; then the held-out batch at that tau
    s_va, d_va, _ = kgsynth.queries(h, cfg.graph.n, kgsynth.QuerySpec(2048, "degree", K, seed=16))
    ex_va = g.topk(s_va, d_va, K).to_numpy()
    c_va = mhr.candidates(g, s_va, d_va)
    sc_va = lp.logits(c_va)
    sweep = {}
    tau_star = 1.0
    for tau in (0.0, 0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8, 0.9, 0.95, 0.98, 0.99, 1.0):
        res, st = lp.search(s_va, d_va, K, keep_permille=100, tau=tau, scores=sc_va)
        rec = topk_recall(ex_va, res.to_numpy())
        sweep[str(tau)] = {"recall": round(rec, 4), "fallback": st["fallback"]}
        if rec >= 0.95:
            tau_star = tau
            break
    out["tau_sweep_validation"] = sweep
    out["tau_selected"] = tau_star
    for tau in sorted({0.0, tau_star}):
        (res, st), t_pr = timed(lambda: lp.search(s, d, K, keep_permille=100, tau=tau), args.steps)
        out[f"tau_{tau}"] = {"recall": round(topk_recall(exn, res.to_numpy()), 4), "fallback": st["fallback"],
                             "queries_per_s": len(s) / t_pr}
    log(f"pruner: {out}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="realistic")
    ap.add_argument("--cpu-sample", type=int, default=None,
                    help="queries the oracle baseline runs (default: 1024 realistic, 256 precision, 512 batched)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-bytes", action="store_true")
    ap.add_argument("--train-queries", type=int, default=200000, help="learned-pruner form: training queries")
    ap.add_argument("--hidden", type=int, default=512, help="learned-pruner form: hidden width")
    ap.add_argument("--scorer", default="distmult", choices=["distmult", "transe_l1"],
                    help="edge scorer (transe_l1: gamma = 1 minus the L1 distance, the paper's score)")
    ap.add_argument("--band-abs", type=float, default=0.0,
                    help="absolute rescoring band below the K-th score (0: the rigorous band alone)")
    ap.add_argument("--turing-batch", type=int, default=64, help="turing: pipelines per batched call")
    ap.add_argument("--wide-queries", type=int, default=16384, help="paper_kg / paper_kg_16th: queries per batch")
    ap.add_argument("--beam-hops", type=int, default=0,
                    help="run the generic multi-hop beam search with this many hops instead of the exact search")
    ap.add_argument("--beam-k", type=int, default=32, help="beam search: children kept per parent and paths returned")
    ap.add_argument("--phase-clocks", action="store_true",
                    help="load the phase-clock build (libmhr_phase.so) and report the gather kernel's time and "
                         "bytes per phase (timings include the clock reads; not a benchmark line)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain 1 GiB device copy (for scaling HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(queries are independent and would be dealt out across GPUs by planning cost).", file=sys.stderr)
        sys.exit(2)

    if args.calibrate_copy:
        calibrate_copy()
        return

    if args.config in ("paper_kg", "paper_kg_16th"):
        run_wide(args)
        return
    if args.config == "turing":
        run_turing(args)
        return
    if args.phase_clocks:
        os.environ["MHR_LIBRARY"] = os.path.join(ROOT, "paper_2406_07727_amd", "libmhr_phase.so")

    import torch
    import kgsynth
    import paper_2406_07727_amd as mhr

    cfg = kgsynth.CONFIGS[args.config]
    t0 = time.perf_counter()
    h, r, t = kgsynth.make_graph(cfg.graph)
    X, Y = kgsynth.embeddings(cfg.graph.n, cfg.graph.R, cfg.emb)
    s, d, k = kgsynth.queries(h, cfg.graph.n, cfg.query)
    log(f"inputs generated in {time.perf_counter() - t0:.1f} s")

    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    g = mhr.Graph(h, r, t, cfg.graph.n, cfg.graph.R)
    if args.scorer != "distmult":
        g.set_scorer(args.scorer, 1.0)
    if cfg.emb.dtype == "bf16":
        Xd = torch.from_numpy(X.view(np.int16)).cuda()
        Yd = torch.from_numpy(Y.view(np.int16)).cuda()
    else:
        Xd = torch.from_numpy(X).cuda()
        Yd = torch.from_numpy(Y).cuda()
    g.set_embeddings(Xd, Yd, dtype=cfg.emb.dtype)
    torch.cuda.synchronize()
    log(f"graph built on the GPU in {time.perf_counter() - t0:.2f} s: {g.stats()}")

    sd = torch.from_numpy(s.view(np.int32)).cuda()
    dd = torch.from_numpy(d.view(np.int32)).cuda()
    kd = torch.from_numpy(k.view(np.int32)).cuda()
    k_max = int(k.max())
    per_query_k = cfg.query.k_choices is not None
    kk = kd if per_query_k else int(k[0])

    if args.beam_hops:
        run_beam(args, cfg, g, h, r, t, X, Y, s, d)
        return
    ev = HipEvents()
    if args.config == "pruner":
        pr = run_pruner(args, cfg, g, h, s, d)
        print(json.dumps({"metric": "pruned top-K recall and queries/s at K=32 (learned pruner vs exact search)",
                          "value": pr["tau_0.0"]["queries_per_s"], "unit": "queries/s", "n_gpus": 1,
                          "steps": args.steps, "warmup": args.warmup, "higher_is_better": True,
                          "dtype": cfg.emb.dtype, "data": "synthetic",
                          "config": {"workload": "pruner: Chung-Lu 4M vertices, 32 relations, 64M edges, d=256 bf16, "
                                                 f"{len(s)} held-out queries, K={cfg.query.k}"},
                          "pruner": pr}), flush=True)
        return
    batched = {}
    if args.config == "batched":
        # the batched form: autotuned settings, one captured plan per batch
        t1 = time.perf_counter()
        tuned, tuned_ms = g.autotune(sd, dd, kk, k_max=k_max, reps=2)
        batched["autotune"] = {"tile_edges": tuned.tile_edges, "hash_log2": tuned.hash_log2,
                               "ms_per_call": round(tuned_ms, 4), "seconds": round(time.perf_counter() - t1, 1)}
        log(f"autotuned: {batched['autotune']}")
        plan = g.plan(sd, dd, kk, k_max=k_max, opts=tuned)
        for _ in range(max(1, args.warmup)):
            plan.launch()
        torch.cuda.synchronize()
        e0, e1 = ev.create(), ev.create()
        stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        w0 = time.perf_counter()
        assert ev.hip.hipEventRecord(e0, stream) == 0
        for _ in range(args.steps):
            plan.launch()
        assert ev.hip.hipEventRecord(e1, stream) == 0
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        step_ms = ev.elapsed_ms(e0, e1) / args.steps
        res = plan.out
        # the same batch as one non-captured call per query (bounded sample)
        nper = min(512, len(s))
        out1 = g.topk(sd[:1], dd[:1], kd[:1], k_max=k_max)
        torch.cuda.synchronize()
        p0 = time.perf_counter()
        for q in range(nper):
            g.topk(sd[q:q + 1], dd[q:q + 1], kd[q:q + 1], k_max=k_max, out=out1)
        torch.cuda.synchronize()
        per_query_s = (time.perf_counter() - p0) / nper
        batched["per_query_launch_queries_per_s"] = 1.0 / per_query_s
        batched["per_query_launch_sample"] = nper
        gather_avg = None
    else:
        qo = mhr.QueryOpts(0, 0, 0, 0, args.band_abs) if args.band_abs > 0 else None
        res = g.topk(sd, dd, kk, k_max=k_max, opts=qo)
        torch.cuda.synchronize()
        for _ in range(args.warmup):
            g.topk(sd, dd, kk, k_max=k_max, out=res, opts=qo)
        torch.cuda.synchronize()

        evs = [mhr.PhaseEvents(ev.create().value, ev.create().value, ev.create().value, ev.create().value)
               for _ in range(args.steps)]
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        for i in range(args.steps):
            g.topk(sd, dd, kk, k_max=k_max, out=res, events=evs[i], opts=qo)
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        step_ms = ev.elapsed_ms(ctypes.c_void_p(evs[0].begin), ctypes.c_void_p(evs[-1].end)) / args.steps
        gather_ms = [ev.elapsed_ms(ctypes.c_void_p(e.gather_begin), ctypes.c_void_p(e.gather_end)) for e in evs]
        gather_avg = float(np.mean(gather_ms))

    phases = None
    if args.phase_clocks:
        # the timed steps again, with the phase clocks reset before them
        mhr.phase_ticks(reset=True)
        for i in range(args.steps):
            g.topk(sd, dd, kk, k_max=k_max, out=res, opts=qo)
        (tab, dirk), rate = mhr.phase_ticks(by_kind=True)
        ticks = {p: tab[p] + dirk[p] for p in mhr.GATHER_PHASES}
        phases = {"ticks": ticks, "rate_hz": rate, "kinds": (tab, dirk)}
    p, cnt, tot, st = res.to_numpy()
    paths = int(tot.sum())
    exact_pass = int(np.sum((st & mhr.Q_EXACT_PASS) != 0))
    bad = int(np.sum((st & ~np.uint32(mhr.Q_EXACT_PASS)) != 0))
    log(f"step {step_ms:.3f} ms (host wall {1e3 * wall / args.steps:.3f} ms/step), gather {gather_avg} ms, "
        f"paths/batch {paths}, exact-pass queries {exact_pass}, bad statuses {bad}")

    roof = None
    if not args.no_bytes and gather_avg is not None:
        t1 = time.perf_counter()
        csr_out = tuple(x.cpu().numpy().view(np.uint32) for x in g.export_csr(reverse=False))
        csr_in = tuple(x.cpu().numpy().view(np.uint32) for x in g.export_csr(reverse=True))
        elem = 2 if cfg.emb.dtype == "bf16" else 4
        layout_b, nbytes, matches = gather_bytes(csr_out, csr_in, s, d, cfg.emb.d, elem, k=k, totals=tot)
        rel_table = cfg.graph.R * cfg.emb.d * elem   # once per launch
        nbytes += rel_table
        layout_b += rel_table
        achieved = nbytes / (gather_avg * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(args.config),
                "kernel": "gather_kernel", "bytes_per_launch": int(nbytes), "bytes_per_launch_pair_layout":
                int(layout_b), "kernel_ms": round(gather_avg, 4)}
        log(f"gather algorithmic bytes {nbytes / 1e6:.1f} MB per the per-query model, {layout_b / 1e6:.1f} MB in the "
            f"pair layout ({matches} matched middle pairs) in {time.perf_counter() - t1:.1f} s")

    if phases is not None:
        # per phase: the average workgroup's wall time per launch, and the
        # algorithmic bytes the phase moves (scanned columns for the probe
        # phase; embedding rows and middle-edge masks for formation and scoring)
        ticks, rate = phases["ticks"], phases["rate_hz"]
        tot_ticks = sum(ticks.values())
        # the persistent grid holds one workgroup per CU (the LDS of one fills a CU)
        nblocks = torch.cuda.get_device_properties(0).multi_processor_count
        per_launch_s = {k: v / rate / nblocks / args.steps for k, v in ticks.items()}
        out_ph = {k: {"share": round(v / tot_ticks, 4), "ms_per_launch": round(1e3 * per_launch_s[k], 4)}
                  for k, v in ticks.items()}
        if roof is not None:
            csr_out = tuple(x.cpu().numpy().view(np.uint32) for x in g.export_csr(reverse=False))
            csr_in = tuple(x.cpu().numpy().view(np.uint32) for x in g.export_csr(reverse=True))
            elem = 2 if cfg.emb.dtype == "bf16" else 4
            parts = gather_byte_parts(csr_out, csr_in, s, d, cfg.emb.d, elem)
            ph_bytes = {"probe": parts["scan"], "form": parts["match_masks"], "score": parts["emb"],
                        "setup": parts["probe_rows"], "rows": parts["list_rows"]}
            for k, b in ph_bytes.items():
                out_ph[k]["bytes"] = int(b)
                if per_launch_s[k] > 0:
                    out_ph[k]["GB_s"] = round(b / per_launch_s[k] / 1e9, 1)
        # per tile kind (probe side in the LDS table, or probing through the
        # row directory): phase times and the work counts per launch
        kinds = {}
        for name, kd in zip(("table", "directory"), phases["kinds"]):
            kinds[name] = {"ms_per_launch": {p: round(1e3 * kd[p] / rate / nblocks / args.steps, 4)
                                             for p in mhr.GATHER_PHASES},
                           "counts_per_launch": {c: kd[c] // args.steps for c in mhr.GATHER_COUNTS}}
        log(f"gather phases: {json.dumps(out_ph)}")
        log(f"per tile kind: {json.dumps(kinds)}")
        print(json.dumps({"phases": out_ph, "tile_kinds": kinds, "config": args.config, "steps": args.steps,
                          "note": "phase-clock build; wall time of the average workgroup per launch"}), flush=True)
        return

    cpu = parity = None
    if not args.no_cpu_baseline:
        nsample = args.cpu_sample or {"realistic": 1024, "precision": 256, "batched": 512}.get(args.config, 256)
        cpu, parity = cpu_baseline(cfg, h, r, t, X, Y, s, d, k, min(nsample, len(s)),
                                   gpu_result=(p, cnt, tot, st), scorer=args.scorer)
        log(f"cpu baseline: {cpu}")
        log(f"parity against the oracle: {parity}")

    value = paths / (step_ms * 1e-3)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "paths/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if cfg.emb.dtype == "f32" else "bf16",
        "data": "synthetic",
        "queries_per_s": len(s) / (step_ms * 1e-3),
        "paths_per_batch": paths,
        "config": {"workload": f"{args.config}: Chung-Lu typed KG {cfg.graph.n} vertices, {cfg.graph.R} relations, "
                               f"{cfg.graph.m} edges, d={cfg.emb.d} {cfg.emb.dtype}, {len(s)} queries, "
                               f"K={'/'.join(map(str, cfg.query.k_choices)) if per_query_k else cfg.query.k}",
                   "queries": len(s), "k": k_max, "dim": cfg.emb.d,
                   "band_abs": args.band_abs, "scorer": args.scorer},
        "roofline": roof,
        "cpu_baseline": cpu,
        "parity": parity,
    }
    if batched:
        out["batched"] = batched
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
