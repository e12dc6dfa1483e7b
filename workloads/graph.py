"""Proximity-graph construction for the synthetic workloads.

The paper applies FINGER to any given graph G = (D, E) (Section 3.3 and
Algorithm 2 take G as input); its experiments use HNSW.  The flat stand-in
built here is:

1. exact k-NN of every point (self excluded, ties broken by smaller id);
2. symmetrization (an edge in either direction becomes an edge both ways);
3. for rows longer than ``max_degree``: the neighbour-selection heuristic of
   HNSW (scan candidates by ascending distance to the base point; keep a
   candidate only if it is closer to the base than to every kept neighbour;
   stop at ``max_degree``; no fill-back);
4. reachability repair from the entry, in the spirit of NSG's spanning step
   (mixture data splits into one component per cluster): while a node is
   unreached, the smallest-id unreached node u gets an in-edge from its
   nearest reached node v that still has a free slot (and u -> v if u has one).

Rows are int32, sorted by (distance to base, id), padded with -1 at the end.
Heavy pairwise work runs through torch matmuls on the chosen device; integer
data (values 0..255, m <= 128) is exact in float32 so any device gives the
same graph.
"""
from __future__ import annotations

import numpy as np
import torch


def _as_dev(x: np.ndarray, device, dtype) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(x)).to(device=device, dtype=dtype)


def _work_dtype(data: np.ndarray, device) -> torch.dtype:
    integral = bool(np.all(data == np.rint(data))) and float(np.abs(data).max()) <= 255 \
        and data.shape[1] <= 128
    if integral:
        return torch.float32          # exact: every partial sum is an integer < 2^24
    return torch.float64 if torch.device(device).type == "cpu" else torch.float32


def knn_lists(data: np.ndarray, k: int, device="cpu", chunk: int = 2048):
    """Exact k nearest neighbours of every point of ``data`` among ``data``.

    Returns (ids int64 [n, k], d2 float64 [n, k]) sorted by (d2, id).
    Selection uses |x|^2 + |y|^2 - 2 x.y; the k+8 best are re-sorted by
    (d2, id) so equal distances resolve to the smaller id.
    """
    n = data.shape[0]
    dt = _work_dtype(data, device)
    X = _as_dev(data, device, dt)
    sq = (X * X).sum(1)
    kk = min(k + 8, n - 1)
    out_i = np.empty((n, k), dtype=np.int64)
    out_d = np.empty((n, k), dtype=np.float64)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        d2 = sq[s:e, None] + sq[None, :] - 2.0 * (X[s:e] @ X.T)
        d2.clamp_(min=0)
        rows = torch.arange(s, e, device=X.device)
        d2[rows - s, rows] = float("inf")
        vals, idx = torch.topk(d2, kk, dim=1, largest=False, sorted=True)
        vals = vals.double().cpu().numpy()
        idx = idx.cpu().numpy()
        order = np.lexsort((idx, vals), axis=1)
        out_i[s:e] = np.take_along_axis(idx, order, 1)[:, :k]
        out_d[s:e] = np.take_along_axis(vals, order, 1)[:, :k]
    return out_i, out_d


def symmetrize(ids: np.ndarray, d2: np.ndarray):
    """Union of out- and in-edges.  Returns CSR (indptr, nbr, dist) with each
    row sorted by (dist, id)."""
    n, k = ids.shape
    src = np.repeat(np.arange(n, dtype=np.int64), k)
    dst = ids.reshape(-1)
    dd = d2.reshape(-1)
    s2 = np.concatenate([src, dst])
    t2 = np.concatenate([dst, src])
    d2c = np.concatenate([dd, dd])
    order = np.lexsort((t2, d2c, s2))
    s2, t2, d2c = s2[order], t2[order], d2c[order]
    # drop duplicate (src, dst) pairs: same pair always has the same distance
    key = s2 * n + t2
    _, first = np.unique(key, return_index=True)
    first.sort()
    s2, t2, d2c = s2[first], t2[first], d2c[first]
    # rows are still sorted by (src, dist, dst) after removing duplicates
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(indptr, s2 + 1, 1)
    indptr = np.cumsum(indptr)
    return indptr, t2, d2c


def prune_heuristic(data: np.ndarray, indptr, nbr, dist, max_degree: int,
                    device="cpu"):
    """Apply the HNSW neighbour-selection heuristic to rows longer than
    ``max_degree``; shorter rows are kept whole.  Returns int32 [n, max_degree]."""
    n = indptr.shape[0] - 1
    deg = np.diff(indptr)
    G = np.full((n, max_degree), -1, dtype=np.int32)
    short = np.nonzero(deg <= max_degree)[0]
    if short.size:
        for j in range(int(deg[short].max())):
            sel = short[deg[short] > j]
            G[sel, j] = nbr[indptr[sel] + j]
    long_rows = np.nonzero(deg > max_degree)[0]
    if long_rows.size == 0:
        return G
    dt = _work_dtype(data, device)
    X = _as_dev(data, device, dt)
    # batch rows of similar length
    order = long_rows[np.argsort(deg[long_rows], kind="stable")]
    B = 1024
    for s in range(0, order.size, B):
        rows = order[s:s + B]
        D = int(deg[rows].max())
        cand = np.full((rows.size, D), -1, dtype=np.int64)
        dbase = np.full((rows.size, D), np.inf, dtype=np.float64)
        for j in range(D):
            ok = deg[rows] > j
            cand[ok, j] = nbr[indptr[rows[ok]] + j]
            dbase[ok, j] = dist[indptr[rows[ok]] + j]
        valid = torch.from_numpy(cand >= 0).to(X.device)
        ci = torch.from_numpy(np.where(cand >= 0, cand, 0)).to(X.device)
        V = X[ci]                                   # [b, D, m]
        sq = (V * V).sum(-1)
        pair = sq[:, :, None] + sq[:, None, :] - 2.0 * torch.bmm(V, V.transpose(1, 2).contiguous())
        pair.clamp_(min=0)
        db = torch.from_numpy(dbase).to(X.device, dtype=pair.dtype)
        kept = torch.zeros_like(valid)
        count = torch.zeros(rows.size, dtype=torch.int64, device=X.device)
        for j in range(D):
            # candidate j survives iff closer to base than to every kept one
            closer = db[:, j:j + 1] < pair[:, j, :j]
            ok = torch.all(closer | ~kept[:, :j], dim=1) & valid[:, j] & (count < max_degree)
            kept[:, j] = ok
            count += ok.long()
        kept_np = kept.cpu().numpy()
        for bi, r in enumerate(rows):
            sel = cand[bi][kept_np[bi]]
            G[r, :sel.size] = sel
    return G


def _bfs(G: np.ndarray, reached: np.ndarray, seeds: np.ndarray) -> None:
    frontier = np.unique(seeds)
    reached[frontier] = True
    while frontier.size:
        nb = G[frontier].reshape(-1)
        nb = nb[nb >= 0]
        nb = nb[~reached[nb]]
        if nb.size == 0:
            break
        nb = np.unique(nb)
        reached[nb] = True
        frontier = nb


def repair_reachability(data: np.ndarray, G: np.ndarray, entry: int,
                        device="cpu") -> tuple[np.ndarray, int, int]:
    """Make every node reachable from ``entry`` (see module doc, step 4).

    Returns (graph, components_before, edges_added)."""
    G = G.copy()
    n, W = G.shape
    deg = (G >= 0).sum(1)
    reached = np.zeros(n, dtype=bool)
    _bfs(G, reached, np.array([entry]))
    dt = _work_dtype(data, device)
    X = _as_dev(data, device, dt)
    sq = (X * X).sum(1)
    added = 0
    repairs = 0
    cursor = 0
    while True:
        un = np.flatnonzero(~reached[cursor:])
        if un.size == 0:
            break
        u = int(cursor + un[0])
        cursor = u
        repairs += 1
        d2 = sq + sq[u] - 2.0 * (X @ X[u])
        mask = torch.from_numpy(reached & (deg < W)).to(X.device)
        d2 = torch.where(mask, d2, torch.full_like(d2, float("inf")))
        v = int(torch.argmin(d2).item())      # argmin returns the first (smallest id) minimum
        if not np.isfinite(float(d2[v].item())):
            raise RuntimeError("no reached node has a free slot")
        G[v, deg[v]] = u
        deg[v] += 1
        added += 1
        if deg[u] < W and not np.any(G[u, :deg[u]] == v):
            G[u, deg[u]] = v
            deg[u] += 1
            added += 1
        _bfs(G, reached, np.array([u]))
    return G, repairs + 1, added


def medoid(data: np.ndarray) -> int:
    """Index of the point nearest the FP64 mean (direct differences; ties go
    to the smaller index)."""
    mu = data.astype(np.float64).mean(0)
    best, best_i = np.inf, -1
    for s in range(0, data.shape[0], 1 << 16):
        blk = data[s:s + (1 << 16)].astype(np.float64) - mu
        d = (blk * blk).sum(1)
        i = int(np.argmin(d))
        if d[i] < best:
            best, best_i = d[i], s + i
    return best_i


def pick_pivots(n: int, count: int, seed: int) -> np.ndarray:
    """``count`` distinct node ids drawn with a seeded generator, ascending."""
    rng = np.random.default_rng(seed ^ 0x5EED)
    return np.sort(rng.choice(n, size=min(count, n), replace=False)).astype(np.int32)


def build_graph(data: np.ndarray, knn_k: int = 16, max_degree: int = 32,
                device="cpu", entry: int | None = None):
    """Full recipe (module doc).  Returns (graph int32 [n, max_degree], entry,
    stats dict)."""
    ids, d2 = knn_lists(data, knn_k, device=device)
    indptr, nbr, dist = symmetrize(ids, d2)
    sym_deg = np.diff(indptr)
    G = prune_heuristic(data, indptr, nbr, dist, max_degree, device=device)
    if entry is None:
        entry = medoid(data)
    G, comps, added = repair_reachability(data, G, entry, device=device)
    stats = {
        "sym_degree_mean": float(sym_deg.mean()),
        "sym_degree_max": int(sym_deg.max()),
        "degree_mean": float((G >= 0).sum(1).mean()),
        "components_before_repair": int(comps),
        "edges_added": int(added),
        "entry": int(entry),
    }
    return G, int(entry), stats


def draw_levels(n: int, M: int, seed: int) -> np.ndarray:
    """Top layer of each node as HNSW draws it: floor(-ln(U) / ln(M)) with U
    uniform on (0, 1] from a seeded generator (int32 [n])."""
    rng = np.random.default_rng(seed ^ 0x1E7E15)
    u = 1.0 - rng.random(n)                       # (0, 1]
    return np.floor(-np.log(u) / np.log(M)).astype(np.int32)


def build_hierarchy(data: np.ndarray, levels: np.ndarray, M: int = 16, candidates: int = 128,
                    device="cpu"):
    """Upper layers of an HNSW-style hierarchy over ``data`` (layer 0 is the
    flat graph built elsewhere).

    Layer l >= 1 holds the nodes with levels >= l.  HNSW builds its layers by
    inserting nodes one at a time, linking each to M of the ``candidates``
    nearest it finds in the layer (its construction beam) through the
    neighbour-selection heuristic, and adding the reverse links (re-pruned by
    the heuristic when a row overflows).  This stand-in takes the end state
    directly: exact kNN with k = ``candidates`` inside the layer,
    symmetrization, the heuristic down to M, and reachability repair from the
    layer's copy of the top entry.  A wide candidate pool matters on
    clustered data: with only the few nearest, the heuristic has no
    neighbour outside the node's own cluster to keep.  The top entry is the
    smallest id among the nodes of the highest level.

    Returns (upper int32 [rows][M], top entry): node-major rows, one per
    (node, layer) with 1 <= layer <= levels[node], ascending node id then
    ascending layer, each holding global neighbour ids padded with -1."""
    levels = np.asarray(levels, dtype=np.int64)
    n = data.shape[0]
    top_level = int(levels.max()) if n else 0
    top = int(np.flatnonzero(levels == top_level)[0]) if n else -1
    row0 = np.concatenate([[0], np.cumsum(levels)[:-1]]).astype(np.int64)
    upper = np.full((int(levels.sum()), M), -1, dtype=np.int32)
    for layer in range(1, top_level + 1):
        S = np.flatnonzero(levels >= layer)
        if S.size < 2:
            continue
        sub = np.ascontiguousarray(data[S])
        k = max(1, min(candidates, S.size - 1))
        ids, d2 = knn_lists(sub, k, device=device)
        indptr, nbr, dist = symmetrize(ids, d2)
        G = prune_heuristic(sub, indptr, nbr, dist, M, device=device)
        G, _, _ = repair_reachability(sub, G, int(np.searchsorted(S, top)), device=device)
        rows = row0[S] + layer - 1
        upper[rows] = np.where(G >= 0, S[np.maximum(G, 0)], -1)
    return upper, top
