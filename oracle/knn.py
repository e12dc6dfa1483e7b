"""Exact distances and brute-force k-nearest neighbours (Section 1: the KNNS
problem and recall@K).  Test infrastructure only."""
from __future__ import annotations

import numpy as np


def sqdist(x: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """Squared L2 distance between x [m] and each row of Y [.., m], by direct
    differences in float64 (never by norm expansion)."""
    diff = np.asarray(Y, dtype=np.float64) - np.asarray(x, dtype=np.float64)
    return (diff * diff).sum(axis=-1)


def ipdist(x: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """Inner-product "distance" -q.y for maximum inner-product search
    (Supplementary A): smaller is better, so the search's ordering and
    admission rule apply unchanged."""
    return -(np.asarray(Y, dtype=np.float64) @ np.asarray(x, dtype=np.float64))


def dist(x: np.ndarray, Y: np.ndarray, metric: str = "l2") -> np.ndarray:
    """Squared L2 (``"l2"``) or negated inner product (``"ip"``)."""
    if metric == "l2":
        return sqdist(x, Y)
    if metric == "ip":
        return ipdist(x, Y)
    raise ValueError(metric)


def normalize_rows(X: np.ndarray) -> np.ndarray:
    """Unit-normalize rows in float64 (angular distance is L2 on unit vectors,
    Supplementary A); zero rows stay zero."""
    X = np.asarray(X, dtype=np.float64)
    nrm = np.sqrt((X * X).sum(axis=-1, keepdims=True))
    return np.where(nrm > 0, X / np.where(nrm > 0, nrm, 1.0), 0.0)


def brute_force_knn(data: np.ndarray, queries: np.ndarray, k: int, metric: str = "l2"):
    """The K closest points of ``data`` to each query, ordered by (d2, id)
    (for ``metric="ip"``: by (-q.x, id), the K largest inner products).

    Returns (ids int64 [nq, k], d2 float64 [nq, k]); if k > n the tail is
    padded with id -1 and d2 +inf."""
    data = np.asarray(data, dtype=np.float64)
    queries = np.atleast_2d(np.asarray(queries, dtype=np.float64))
    n = data.shape[0]
    nq = queries.shape[0]
    ids = np.full((nq, k), -1, dtype=np.int64)
    d2 = np.full((nq, k), np.inf, dtype=np.float64)
    idx = np.arange(n)
    for i in range(nq):
        d = dist(queries[i], data, metric)
        order = np.lexsort((idx, d))[:k]
        ids[i, :order.size] = order
        d2[i, :order.size] = d[order]
    return ids, d2


def recall_at_k(found: np.ndarray, gt_ids: np.ndarray, k: int,
                found_d2: np.ndarray | None = None,
                gt_d2: np.ndarray | None = None) -> float:
    """Mean over queries of |T intersect A| / K (Section 1).

    With ``found_d2`` and ``gt_d2`` a returned id also counts when its
    distance is <= the K-th true distance (tie-tolerant recall, exact on
    integer data where equal distances are real ties)."""
    found = np.atleast_2d(found)[:, :k]
    gt_ids = np.atleast_2d(gt_ids)[:, :k]
    hits = 0
    for i in range(found.shape[0]):
        A = set(int(x) for x in gt_ids[i] if x >= 0)
        if found_d2 is not None and gt_d2 is not None:
            kth = gt_d2[i, k - 1]
            hits += sum(1 for j, x in enumerate(found[i])
                        if x >= 0 and (int(x) in A or found_d2[i, j] <= kth))
        else:
            hits += sum(1 for x in found[i] if int(x) in A)
    return hits / float(k * found.shape[0])
