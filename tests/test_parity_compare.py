"""The GPU-vs-oracle comparison itself, on the CPU: a result copied from the
oracle passes, and each planted mistake (a swapped pair, a dishonest
precision-tie flag, a path from beyond the oracle's ranking, a score off by
more than its bound, a wrong count) fails.  The mistakes are planted in
copies of the oracle's output; no GPU is involved."""

import numpy as np
import pytest

import kgsynth
import oracle
from tests.parity import OracleResult, compare, parity_summary, run_oracle

GPU_DTYPE = np.dtype([("a", np.uint32), ("b", np.uint32), ("r1", np.uint16), ("r2", np.uint16),
                      ("r3", np.uint16), ("flags", np.uint16), ("score", np.float32),
                      ("err_bound", np.float32)])


@pytest.fixture(scope="module")
def case(oracle_lib):
    cfg = kgsynth.CONFIGS["dense_tiny"]
    h, r, t = kgsynth.make_graph(cfg.graph)
    X, Y = kgsynth.embeddings(cfg.graph.n, cfg.graph.R, cfg.emb)
    s, d, _ = kgsynth.queries(h, cfg.graph.n, cfg.query)
    K = 10
    orc = run_oracle(cfg.graph.n, cfg.graph.R, h, r, t, X, Y, s, d, K)
    assert np.all(orc.count == K) and np.all(orc.full == K + 8)
    return orc, K


def as_gpu(orc, K):
    """A GPU-shaped result equal to the oracle's: FP32 scores with bounds of
    1 ulp of 4, no flags."""
    nq = len(orc.count)
    p = np.zeros((nq, K), GPU_DTYPE)
    for f in ("a", "b", "r1", "r2", "r3"):
        p[f] = orc.paths[f][:, :K]
    p["score"] = orc.paths["s"][:, :K].astype(np.float32)
    p["err_bound"] = np.float32(2.0 ** -21)
    return p, orc.count.copy(), orc.total.copy(), np.zeros(nq, np.uint32)


def test_copy_of_oracle_passes(case):
    orc, K = case
    assert compare(as_gpu(orc, K), orc) == 0
    s = parity_summary(as_gpu(orc, K), orc, range(len(orc.count)))
    assert s["mismatches"] == 0 and s["checked"] == len(orc.count)


def _planted(case, plant):
    orc, K = case
    gpu = as_gpu(orc, K)
    plant(gpu, orc)
    return gpu, orc


def test_swap_without_flag_fails(case):
    def plant(gpu, orc):
        p = gpu[0]
        p[0, [3, 4]] = p[0, [4, 3]]
    gpu, orc = _planted(case, plant)
    with pytest.raises(AssertionError, match="differ"):
        compare(gpu, orc)


def test_dishonest_tie_flag_fails(case):
    """A swapped pair flagged as a precision tie, although the oracle's
    scores lie far apart compared with the bounds: the flag is rejected."""
    orc, K = case
    gap = orc.paths["s"][:, 3] - orc.paths["s"][:, 4]
    q = int(np.argmax(gap))
    assert gap[q] > 1e-4

    def plant(gpu, orc):
        p = gpu[0]
        p[q, [3, 4]] = p[q, [4, 3]]
        p["flags"][q, 3] = 2
    gpu, orc = _planted(case, plant)
    with pytest.raises(AssertionError, match="flagged as a precision tie"):
        compare(gpu, orc, max_ties=5)


def test_honest_tie_flag_is_counted(case):
    """A flag whose scores lie within the bounds is accepted, but counted:
    compare fails when more flags appear than allowed."""
    orc, K = case
    gap = orc.paths["s"][:, 3] - orc.paths["s"][:, 4]
    q = int(np.argmin(np.where(gap > 0, gap, np.inf)))

    def plant(gpu, orc):
        p = gpu[0]
        p[q, [3, 4]] = p[q, [4, 3]]
        p["flags"][q, 3] = 2
        p["err_bound"][q, 3:5] = np.float32(gap[q] + 2.0 ** -20)
    gpu, orc = _planted(case, plant)
    assert compare(gpu, orc, max_ties=1) == 1
    with pytest.raises(AssertionError, match="precision-tie flags"):
        compare(gpu, orc)


def test_foreign_path_at_kth_place(case):
    """A flagged last place may hold the oracle's (K+1)-th path only when
    its score is within the bounds of the K-th; a path from further down
    fails."""
    orc, K = case
    gap = orc.paths["s"][:, K - 1] - orc.paths["s"][:, K]

    def plant_near(gpu, orc):
        p = gpu[0]
        q = int(np.argmin(gap))
        for f in ("a", "b", "r1", "r2", "r3"):
            p[f][q, K - 1] = orc.paths[f][q, K]
        p["score"][q, K - 1] = np.float32(orc.paths["s"][q, K])
        p["flags"][q, K - 1] = 2
        p["err_bound"][q, K - 1] = np.float32(gap[q] + 2.0 ** -20)
    gpu, o = _planted(case, plant_near)
    assert compare(gpu, o, max_ties=1) == 1

    def plant_far(gpu, orc):
        p = gpu[0]
        q = int(np.argmax(orc.paths["s"][:, K - 1] - orc.paths["s"][:, K + 7]))
        for f in ("a", "b", "r1", "r2", "r3"):
            p[f][q, K - 1] = orc.paths[f][q, K + 7]
        p["score"][q, K - 1] = np.float32(orc.paths["s"][q, K + 7])
        p["flags"][q, K - 1] = 2
    gpu, o = _planted(case, plant_far)
    with pytest.raises(AssertionError):
        compare(gpu, o, max_ties=1)


def test_score_outside_bound_fails(case):
    def plant(gpu, orc):
        gpu[0]["score"][2, 5] += np.float32(1e-5)
    gpu, orc = _planted(case, plant)
    with pytest.raises(AssertionError, match="bound"):
        compare(gpu, orc)


def test_count_and_total_mismatch_fail(case):
    def plant_c(gpu, orc):
        gpu[1][4] -= 1
    gpu, orc = _planted(case, plant_c)
    with pytest.raises(AssertionError, match="count"):
        compare(gpu, orc)

    def plant_t(gpu, orc):
        gpu[2][4] += 1
    gpu, orc = _planted(case, plant_t)
    with pytest.raises(AssertionError, match="total"):
        compare(gpu, orc)
    s = parity_summary(gpu, orc, range(len(orc.count)))
    assert s["mismatches"] == 1 and "total" in s["first_mismatch"]


def test_three_field_oracle_tuple_still_accepted(case):
    orc, K = case
    op = orc.paths[:, :K]
    assert compare(as_gpu(orc, K), (op, orc.count, orc.total)) == 0
    assert isinstance(OracleResult(op, orc.count, orc.total, orc.count), tuple)
