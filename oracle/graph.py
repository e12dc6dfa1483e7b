"""Flat proximity graph in float64, from the definitions.  Test
infrastructure only.

The paper applies FINGER to a given graph (Section 3.3 and Algorithm 2 take
G = (D, E) as input; its experiments use HNSW graphs).  The graph here is
this project's stand-in for HNSW's layer 0, defined by four steps:

1. k nearest neighbours of every point among the others, by the key
   (squared distance, id);
2. symmetrization: the union of every edge and its reverse, each row sorted
   by (squared distance, id), no duplicates;
3. for rows longer than ``max_degree``, HNSW's neighbour-selection
   heuristic: scan the row in order and keep a candidate iff fewer than
   ``max_degree`` are kept and it is strictly closer to the base point than
   to every neighbour kept so far;
4. reachability repair from ``entry``: while some node is unreached, the
   smallest-id unreached node u gets an edge from the reached node v with a
   free slot that minimises (squared distance to u, id), appended to v's
   row; u gets the reverse edge if it has a free slot and does not list v
   yet; then everything reachable from u is marked reached.

Squared distances use |x|^2 + |y|^2 - 2 x.y in float64, which is exact for
the integer-valued workloads.
"""
from __future__ import annotations

import numpy as np


def _sq(X: np.ndarray) -> np.ndarray:
    return (X * X).sum(1)


def knn(data: np.ndarray, k: int, chunk: int = 4096):
    """Step 1 (k < n).  Returns (ids int64 [n, k], d2 float64 [n, k]) sorted
    by (d2, id), the point itself excluded."""
    X = np.asarray(data, dtype=np.float64)
    n = X.shape[0]
    sq = _sq(X)
    ids = np.empty((n, k), dtype=np.int64)
    d2 = np.empty((n, k), dtype=np.float64)
    cols = np.arange(n)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        D = sq[s:e, None] + sq[None, :] - 2.0 * (X[s:e] @ X.T)
        np.maximum(D, 0.0, out=D)
        for r in range(e - s):
            i = s + r
            row = D[r].copy()
            row[i] = np.inf
            # the k smallest keys (d2, id): every point at or below the k-th
            # smallest distance, ordered by (d2, id)
            kth = np.partition(row, k - 1)[k - 1]
            pool = cols[row <= kth]
            order = np.lexsort((pool, row[pool]))[:k]
            ids[i] = pool[order]
            d2[i] = row[pool[order]]
    return ids, d2


def symmetrize(ids: np.ndarray, d2: np.ndarray):
    """Step 2.  Returns a list of rows, each a list of (d2, id) sorted."""
    n = ids.shape[0]
    rows = [dict() for _ in range(n)]
    for i in range(n):
        for j, d in zip(ids[i].tolist(), d2[i].tolist()):
            rows[i][j] = d
            rows[j][i] = d
    return [sorted((d, j) for j, d in r.items()) for r in rows]


def prune(data: np.ndarray, rows, max_degree: int) -> np.ndarray:
    """Step 3.  Returns int32 [n, max_degree], -1 padded."""
    X = np.asarray(data, dtype=np.float64)
    sq = _sq(X)
    n = len(rows)
    G = np.full((n, max_degree), -1, dtype=np.int32)
    for i, row in enumerate(rows):
        if len(row) <= max_degree:
            G[i, :len(row)] = [j for _, j in row]
            continue
        kept = []
        for d, j in row:
            if len(kept) >= max_degree:
                break
            if all(d < max(float(sq[j] + sq[t] - 2.0 * (X[j] @ X[t])), 0.0) for t in kept):
                kept.append(j)
        G[i, :len(kept)] = kept
    return G


def _mark_from(G: np.ndarray, reached: np.ndarray, start: int) -> None:
    stack = [start]
    reached[start] = True
    while stack:
        v = stack.pop()
        for u in G[v]:
            if u >= 0 and not reached[u]:
                reached[u] = True
                stack.append(int(u))


def repair(data: np.ndarray, G: np.ndarray, entry: int):
    """Step 4.  Returns (graph, components before repair, edges added)."""
    X = np.asarray(data, dtype=np.float64)
    G = G.copy()
    n, W = G.shape
    deg = (G >= 0).sum(1)
    reached = np.zeros(n, dtype=bool)
    _mark_from(G, reached, entry)
    sq = _sq(X)
    repairs = added = 0
    u = 0
    while True:
        while u < n and reached[u]:
            u += 1
        if u == n:
            break
        repairs += 1
        d = np.maximum(sq + sq[u] - 2.0 * (X @ X[u]), 0.0)
        ok = np.flatnonzero(reached & (deg < W))
        if ok.size == 0:
            raise RuntimeError("no reached node has a free slot")
        v = int(ok[np.lexsort((ok, d[ok]))[0]])
        G[v, deg[v]] = u
        deg[v] += 1
        added += 1
        if deg[u] < W and v not in G[u, :deg[u]].tolist():
            G[u, deg[u]] = v
            deg[u] += 1
            added += 1
        _mark_from(G, reached, u)
    return G, repairs + 1, added


def build(data: np.ndarray, k: int, max_degree: int, entry: int):
    """Steps 1-4.  Returns (graph int32 [n, max_degree], stats)."""
    ids, d2 = knn(data, k)
    rows = symmetrize(ids, d2)
    G = prune(data, rows, max_degree)
    G, comps, added = repair(data, G, entry)
    return G, {"sym_degree_max": max(len(r) for r in rows),
               "sym_edges": sum(len(r) for r in rows),
               "components_before_repair": comps, "edges_added": added}
