"""Greedy graph search (Algorithm 1) and approximate greedy search
(Algorithm 4, Supplementary C) in float64.  Test infrastructure only.

State: T, the best entries found so far (at most ef_eff = max(ef, K) of them,
ordered by the key (d2, id)), each flagged expanded or not; V, the visited
set.  Readings of the pseudo-code:

* Admission size test.  "|T| <= efs" is read as |T| < ef_eff: T grows to
  ef_eff and then stays there (add, then evict the furthest).  Taken
  literally every neighbour would be admitted and the screen of
  Algorithm 4 could never skip anything.
* Ties.  Keys are (d2, id), compared lexicographically.  A neighbour is
  admitted iff T is not full or its key is below the worst key in T.
* Candidate queue.  C is the set of unexpanded entries of T.  An admitted
  entry that is later evicted from T has a key above the worst of T from
  then on, so Algorithm 1 would stop as soon as it became the nearest of C;
  hence "pop the nearest of C; stop if it is beyond ub" is the same as
  "expand the best unexpanded entry of T; stop when there is none".
* Screening (Algorithm 4).  Its warm-up condition is read as: screening
  starts once the number of expansions so far, counting the current one,
  exceeds W (default 5).
  The screen is applied only when T is full at the start of the expansion
  (otherwise every neighbour would be admitted anyway).  A screened-out
  neighbour stays in V.  Survivors get their exact distance and the normal
  admission rule (Supplementary G: candidates always carry exact distances).
* ub inside one expansion.  ``ub_mode="batched"`` (default) screens every
  neighbour of an expansion against ub at the start of the expansion and
  then admits the survivors together; for plain search this equals the
  sequential order exactly (the final T of an expansion is the best ef_eff
  keys of T plus the admitted ones, whatever the order).
  ``ub_mode="sequential"`` follows Algorithm 4 literally: neighbours in
  stored order, ub refreshed after each admission.
* Estimates and ub are compared as squared distances.

Start points: the nearest of a set of pivot nodes (``pivot_entries``) or the
greedy descent through the upper layers of an HNSW-style hierarchy
(``descend``), with the same (d, id) keys.
"""
from __future__ import annotations

import bisect
import math

import numpy as np

from .estimate import estimate as finger_estimate
from .estimate import estimate_ip as finger_estimate_ip
from .knn import dist

COUNTER_NAMES = ("expansions", "exact", "screened", "skipped", "visited", "preps")


class _TopList:
    """T: sorted keys (d2, id) with an expanded flag per id."""

    def __init__(self, cap: int):
        self.cap = cap
        self.keys: list[tuple[float, int]] = []
        self.expanded: set[int] = set()

    def full(self) -> bool:
        return len(self.keys) >= self.cap

    def worst(self):
        return self.keys[-1]

    def admit(self, d2: float, i: int) -> bool:
        key = (float(d2), int(i))
        if len(self.keys) >= self.cap and not key < self.keys[-1]:
            return False
        bisect.insort(self.keys, key)
        if len(self.keys) > self.cap:
            self.keys.pop()
        return True

    def best_unexpanded(self):
        for key in self.keys:
            if key[1] not in self.expanded:
                return key
        return None


def search(data: np.ndarray, graph: np.ndarray, q: np.ndarray, entry: int,
           ef: int, k: int, mode: str = "plain", tables: dict | None = None,
           warmup: int = 5, ub_mode: str = "batched", estimator=None,
           record: list | None = None, metric: str = "l2"):
    """One query.  Returns (ids int64 [k], d2 float64 [k], counters dict,
    margin) where ids/d2 are the first k keys of T (padded with -1/+inf)
    and margin is the smallest |est - ub^2| / ub^2 over all screening
    decisions (inf if none were taken).

    ``estimator(q, c_id, nbr_ids, ub2) -> est`` overrides Algorithm 3 (used
    for quantized codes and the learned gate).  ``record``, if a list,
    receives one tuple (cur, nbr_ids, est, ub2) per screened expansion.
    ``metric="ip"`` searches by -q.d (maximum inner product, Supplementary
    A) with the inner-product estimate; the margin is then relative to |ub|."""
    assert mode in ("plain", "finger")
    ef_eff = max(int(ef), int(k))
    q = np.asarray(q, dtype=np.float64)
    T = _TopList(ef_eff)
    V = {int(entry)}
    T.admit(float(dist(q, data[entry], metric)), int(entry))
    cnt = dict.fromkeys(COUNTER_NAMES, 0)
    cnt["exact"] = 1
    margin = math.inf

    def est_of(cur, ids, ub2):
        if estimator is not None:
            return np.asarray(estimator(q, cur, ids, ub2), dtype=np.float64)
        if metric == "ip":
            return finger_estimate_ip(q, data[cur], data[ids], tables)
        return finger_estimate(q, data[cur], data[ids], tables)

    while True:
        key = T.best_unexpanded()
        if key is None:
            break
        cur = key[1]
        T.expanded.add(cur)
        cnt["expansions"] += 1
        new = []
        for nb in graph[cur]:
            nb = int(nb)
            if nb < 0 or nb in V:
                continue
            V.add(nb)
            new.append(nb)
        if not new:
            continue
        screen_phase = mode == "finger" and cnt["expansions"] > warmup
        if ub_mode == "batched":
            survivors = new
            if screen_phase and T.full():
                ub2 = T.worst()[0]
                est = est_of(cur, new, ub2)
                cnt["screened"] += len(new)
                cnt["preps"] += 1
                keep = est <= ub2
                cnt["skipped"] += int((~keep).sum())
                if ub2 != 0:
                    margin = min(margin, float(np.min(np.abs(est - ub2)) / abs(ub2)))
                if record is not None:
                    record.append((cur, np.array(new), est, ub2))
                survivors = [nb for nb, kp in zip(new, keep) if kp]
            if survivors:
                d2 = dist(q, data[survivors], metric)
                cnt["exact"] += len(survivors)
                for nb, dd in zip(survivors, d2):
                    T.admit(dd, nb)
        elif ub_mode == "sequential":
            for nb in new:
                if screen_phase and T.full():
                    ub2 = T.worst()[0]
                    est = float(est_of(cur, [nb], ub2)[0])
                    cnt["screened"] += 1
                    if ub2 != 0:
                        margin = min(margin, abs(est - ub2) / abs(ub2))
                    if est > ub2:
                        cnt["skipped"] += 1
                        continue
                dd = float(dist(q, data[nb], metric)[()])
                cnt["exact"] += 1
                T.admit(dd, nb)
        else:
            raise ValueError(ub_mode)
    cnt["visited"] = len(V)
    ids = np.full(k, -1, dtype=np.int64)
    d2 = np.full(k, np.inf)
    for j, (dd, i) in enumerate(T.keys[:k]):
        ids[j] = i
        d2[j] = dd
    return ids, d2, cnt, margin


def pivot_entries(queries: np.ndarray, data: np.ndarray, pivots: np.ndarray,
                  metric: str = "l2") -> np.ndarray:
    """Start point p of each query (Algorithm 1's input) when it is chosen
    among pivot nodes: the pivot at the smallest exact distance (squared L2,
    or -q.p), ties to the earlier pivot in the list.  (A flat stand-in for
    the upper layers of the HNSW graph the paper searches.)"""
    P = np.asarray(data[pivots], dtype=np.float64)
    out = np.empty(np.atleast_2d(queries).shape[0], dtype=np.int64)
    for i, q in enumerate(np.atleast_2d(queries)):
        out[i] = pivots[int(np.argmin(dist(q, P, metric)))]
    return out


def descend(q: np.ndarray, data: np.ndarray, levels: np.ndarray, upper: np.ndarray,
            metric: str = "l2") -> tuple[int, int]:
    """Start point p of Algorithm 1 as an HNSW graph supplies it: the greedy
    descent through the upper layers (HNSW's layer search with a result
    list of one).  From the smallest id among the nodes of the highest
    level, in each layer from the top down to 1, move to the neighbour of
    smallest (d, id) key while that key is below the current node's, then
    keep the node for the layer below.  ``upper`` holds one row per (node,
    layer), node-major with ascending layers; a node's rows start at the sum
    of the levels of the nodes before it.

    Neighbours evaluated before are evaluated again: every one of them has a
    key above the current node's (the current node is the best seen), so
    this changes only the count, not the node reached.  Returns (node,
    distance evaluations including the top entry's)."""
    levels = np.asarray(levels, dtype=np.int64)
    first_row = np.concatenate([[0], np.cumsum(levels)[:-1]])
    top_level = int(levels.max())
    cur = int(np.flatnonzero(levels == top_level)[0])
    key = (float(dist(q, data[cur], metric)[()]), cur)
    calls = 1
    for layer in range(top_level, 0, -1):
        while True:
            nb = upper[first_row[cur] + layer - 1]
            nb = nb[nb >= 0]
            if nb.size == 0:
                break
            d = dist(q, data[nb], metric)
            calls += nb.size
            best = min((float(dv), int(i)) for dv, i in zip(d, nb))
            if not best < key:
                break
            key = best
            cur = best[1]
    return cur, calls


def hierarchy_entries(queries, data, levels, upper, metric: str = "l2"):
    """``descend`` for each query: (entries int64 [nq], calls int64 [nq])."""
    qs = np.atleast_2d(queries)
    out = np.array([descend(q, data, levels, upper, metric) for q in qs], dtype=np.int64)
    return out[:, 0], out[:, 1]


def search_batch(data, graph, queries, entries, ef, k, **kw):
    """``search`` over many queries.  ``entries`` is one id or one per query;
    ``ef``/``k`` are scalars or per-query sequences.  Returns (ids [nq, kmax],
    d2 [nq, kmax], counters int64 [nq, 6] in COUNTER_NAMES order, margins [nq])."""
    queries = np.atleast_2d(queries)
    nq = queries.shape[0]
    ks = np.broadcast_to(np.asarray(k), (nq,))
    efs = np.broadcast_to(np.asarray(ef), (nq,))
    ents = np.broadcast_to(np.asarray(entries), (nq,))
    kmax = int(ks.max())
    ids = np.full((nq, kmax), -1, dtype=np.int64)
    d2 = np.full((nq, kmax), np.inf)
    cnts = np.zeros((nq, len(COUNTER_NAMES)), dtype=np.int64)
    margins = np.full(nq, np.inf)
    for i in range(nq):
        a, b, c, mg = search(data, graph, queries[i], int(ents[i]), int(efs[i]),
                             int(ks[i]), **kw)
        ids[i, :a.size] = a
        d2[i, :b.size] = b
        cnts[i] = [c[nm] for nm in COUNTER_NAMES]
        margins[i] = mg
    return ids, d2, cnts, margins
