"""Pure-Python oracle (tiny graphs only).  TEST INFRASTRUCTURE ONLY.

The same definition as the C oracle, written independently: a dict-of-lists
adjacency over the distinct triples, a literal triple loop over the edges
s->a, a->b and b->t, math.log1p / math.exp for the log-sigmoid, and one full
sort by the key tuple (-S, a, b, r1, r2, r3).  S is the correctly rounded
sum of the three weights (math.fsum), so it depends only on their multiset.  See ``oracle/__init__.py``
for the definition; edge weights follow the DistMult + log-sigmoid reading
or the paper's TransE-L1 score (gamma minus the L1 distance between head
plus relation and tail, section 3.3), path scores the sum of the three
weights of a three-hop walk (section 3.1).
"""

from __future__ import annotations

import math
from collections import defaultdict


def logsigmoid(x: float) -> float:
    return min(x, 0.0) - math.log1p(math.exp(-abs(x)))


def edge_weight(X, Y, u, r, v, scorer="distmult", gamma=1.0) -> float:
    acc = 0.0
    if scorer == "transe_l1":
        for i in range(len(X[u])):
            acc += abs((float(X[u][i]) + float(Y[r][i])) - float(X[v][i]))
        return gamma - acc
    if scorer != "distmult":
        raise ValueError(scorer)
    for i in range(len(X[u])):
        acc += (float(X[u][i]) * float(Y[r][i])) * float(X[v][i])
    return logsigmoid(acc)


def topk_paths(edges, X, Y, s, t, K, keep_first=None, keep_last=None, scorer="distmult", gamma=1.0):
    """edges: iterable of (h, r, t) triples (duplicates allowed; they are
    merged).  X, Y: nested sequences of floats.  Returns (paths, total) with
    paths a list of (S, a, b, r1, r2, r3), best first.

    keep_first / keep_last (sets of vertices, or None for all) restrict the
    paths to those whose first intermediate vertex a, resp. second
    intermediate vertex b, is kept: the pruned search, where a pruner drops
    the pair (s, a) as a first edge or the pair (b, t) as a last edge."""
    out = defaultdict(list)
    for (h, r, v) in sorted(set((int(h), int(r), int(v)) for (h, r, v) in edges)):
        out[h].append((r, v))
    paths = []
    for (r1, a) in out[s]:
        if keep_first is not None and a not in keep_first:
            continue
        w1 = edge_weight(X, Y, s, r1, a, scorer, gamma)
        for (r2, b) in out[a]:
            w2 = edge_weight(X, Y, a, r2, b, scorer, gamma)
            if keep_last is not None and b not in keep_last:
                continue
            for (r3, tt) in out[b]:
                if tt != t:
                    continue
                w3 = edge_weight(X, Y, b, r3, t, scorer, gamma)
                paths.append((math.fsum((w1, w2, w3)), a, b, r1, r2, r3))
    paths.sort(key=lambda p: (-p[0], p[1], p[2], p[3], p[4], p[5]))
    return paths[:K], len(paths)


def beam_paths(edges, X, Y, s, t, H, K, scorer="distmult", gamma=1.0):
    """The generic multi-hop search of section 5 in plain Python: level by
    level, every current path grows by each out-edge whose head is not on
    it; extensions reaching t are recorded, the others keep the best K per
    parent (score descending, then the vertex sequence, then the relation
    sequence).  Returns (best K recorded paths as (S, vertices, relations),
    number recorded)."""
    out = defaultdict(list)
    for (h, r, v) in sorted(set((int(h), int(r), int(v)) for (h, r, v) in edges)):
        out[h].append((v, r))

    def key(p):
        return (-p[0], list(p[1]), list(p[2]))

    curr = [(0.0, (), ())]
    results = []
    for _ in range(H):
        nxt = []
        for score, vs, rs in curr:
            h = vs[-1] if vs else s
            kids = []
            for (nb, r) in out[h]:
                if nb == s or nb in vs:
                    continue
                x = (score + edge_weight(X, Y, h, r, nb, scorer, gamma), vs + (nb,), rs + (r,))
                (results if nb == t else kids).append(x)
            kids.sort(key=key)
            nxt.extend(kids[:K])
        curr = nxt
    results.sort(key=key)
    return results[:K], len(results)
