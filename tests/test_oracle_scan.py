"""Pins for the oracle's candidate scan (the paper's Turing-award pipeline,
section 3.2, with the TransE-L1 scores of section 3.3):

* a hand-worked example with integer embeddings (exact scores, a tie
  broken by the candidate id, K larger than the list);
* on embeddings from a dyadic grid (every sum exact in FP64), the scan
  equals numpy's independent evaluation (vectorised L1 distance, lexsort);
* the order of the candidate list does not matter;
* the pipeline's second hop re-ranks exactly the first hop's persons, and
  its third hop equals one scan per ranked person.
"""

import numpy as np
import pytest

import oracle


def test_handworked_scan(oracle_lib):
    X = np.array([[0, 0], [1, 1], [2, 1], [0, 1], [3, 3], [1, 0]], np.float32)
    Y = np.array([[1, 1]], np.float32)
    # anchor X[0] + Y[0] = (1, 1); distances: 1 -> 0, 2 -> 1, 3 -> 1, 4 -> 4, 5 -> 1
    ids, sc = oracle_lib.scan_topk(X, Y, [0], [0], [4, 3, 2, 1, 5], 3, gamma=1.0)
    assert ids[0].tolist() == [1, 2, 3] and sc[0].tolist() == [1.0, 0.0, 0.0]
    ids, sc = oracle_lib.scan_topk(X, Y, [0], [0], [4, 3, 2, 1, 5], 7, gamma=2.0)
    assert ids[0].tolist() == [1, 2, 3, 5, 4, 0xFFFFFFFF, 0xFFFFFFFF]
    assert sc[0][:5].tolist() == [2.0, 1.0, 1.0, 1.0, -2.0] and np.all(np.isneginf(sc[0][5:]))


def _grid(seed, n, R, d):
    rng = np.random.Generator(np.random.PCG64(seed))
    X = (rng.integers(-256, 257, (n, d)) / 128.0).astype(np.float32)
    Y = (rng.integers(-256, 257, (R, d)) / 128.0).astype(np.float32)
    return rng, X, Y


def test_scan_equals_numpy_on_dyadic_grid(oracle_lib):
    rng, X, Y = _grid(3, 5000, 3, 8)
    cand = rng.choice(5000, 3000, replace=False).astype(np.uint32)
    head = rng.integers(0, 5000, 6).astype(np.uint32)
    rel = rng.integers(0, 3, 6).astype(np.uint32)
    K = 50
    ids, sc = oracle_lib.scan_topk(X, Y, head, rel, cand, K, gamma=1.0)
    for q in range(len(head)):
        s = 1.0 - np.abs((X[head[q]].astype(np.float64) + Y[rel[q]]) - X[cand]).sum(1)
        order = np.lexsort((cand, -s))[:K]
        assert ids[q].tolist() == cand[order].tolist()
        assert np.array_equal(sc[q], s[order])
    # the grid makes ties common: some are broken by the id
    assert any(len(np.unique(sc[q])) < K for q in range(len(head)))


def test_candidate_order_irrelevant(oracle_lib):
    rng, X, Y = _grid(4, 2000, 2, 8)
    cand = rng.choice(2000, 1500, replace=False).astype(np.uint32)
    a = oracle_lib.scan_topk(X, Y, [7, 9], [0, 1], cand, 40)
    b = oracle_lib.scan_topk(X, Y, [7, 9], [0, 1], cand[rng.permutation(len(cand))], 40)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_pipeline_composition(oracle_lib):
    rng, X, Y = _grid(5, 3000, 3, 8)
    perm = rng.permutation(3000).astype(np.uint32)
    persons, unis = perm[2:1500], perm[1500:2600]
    K = 16
    (h1, s1), (h2, s2), (h3, s3) = oracle_lib.turing_pipeline(X, Y, persons, unis, perm[0], perm[1], 0, 1, 2, K)
    assert sorted(h1.tolist()) == sorted(h2.tolist())
    assert np.all(np.diff(s2) <= 0)
    for k in range(K):
        ids, sc = oracle_lib.scan_topk(X, Y, [h2[k]], [2], unis, K)
        assert np.array_equal(h3[k], ids[0]) and np.array_equal(s3[k], sc[0])
