"""The allocation-free query entry point (mhr_topk_paths_noalloc) against
mhr_topk_paths with a caller workspace: byte-identical results on two calls
in a row, the second with a smaller batch and K; batches whose workspace
exceeds the fixed scratch array are rejected before anything runs."""

import numpy as np
import pytest

from tests.parity import compare, gpu_graph, run_oracle, say, workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2406_07727_amd  # noqa: F401


def test_noalloc_matches_workspace_entry_point():
    import torch
    import paper_2406_07727_amd as mhr
    cfg, (h, r, t), (X, Y), (s, d, kk) = workload("hub_tiny")
    n, R = cfg.graph.n, cfg.graph.R
    say("case no-alloc entry point")
    g = gpu_graph(n, R, h, r, t, X, Y)
    kq = (np.arange(len(s)) % 3 * 7 + 1).astype(np.uint32)   # K in {1, 8, 15}
    calls = [(s, d, kq, 16), (s[:20].copy(), d[:20].copy(), np.full(20, 4, np.uint32), 4)]
    for ci, (ss, dd, kc, kmax) in enumerate(calls):
        say(f"call {ci}: nq={len(ss)} k_max={kmax}")
        ref = g.topk(ss, dd, kc, k_max=kmax)
        got = g.topk_noalloc(ss, dd, kc, k_max=kmax)
        torch.cuda.synchronize()
        ref, got = ref.to_numpy(), got.to_numpy()
        for a, b in zip(ref, got):
            assert np.array_equal(a, b), f"call {ci}"
        compare(got, run_oracle(n, R, h, r, t, X, Y, ss, dd, kc))


def test_noalloc_rejects_oversized_batch():
    import paper_2406_07727_amd as mhr
    cfg, (h, r, t), (X, Y), (s, d, kk) = workload("tiny")
    g = gpu_graph(cfg.graph.n, cfg.graph.R, h, r, t, X, Y)
    nq = 8192
    assert g.workspace_bytes(nq, 224) > mhr.NOALLOC_SCRATCH_BYTES
    ss = np.resize(s, nq).astype(np.uint32)
    dd = np.resize(d, nq).astype(np.uint32)
    with pytest.raises(mhr.MhrError) as e:
        g.topk_noalloc(ss, dd, 8, k_max=224)
    assert e.value.status == 2     # MHR_ERR_WORKSPACE_TOO_SMALL
