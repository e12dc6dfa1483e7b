"""Shared seeded workloads for the tests (inputs only; no method arithmetic)."""
from __future__ import annotations

import functools

import numpy as np

from workloads import SPECS, build_graph, make_points, pick_pivots


@functools.lru_cache(maxsize=None)
def c1(nq: int = 1000):
    """The parity workload: 10,000 points from 100 Gaussians in 32-d,
    exact 16-NN symmetrized and pruned to 32, medoid entry."""
    spec = SPECS["c1"].scaled(nq=nq)
    data, qs = make_points(spec)
    G, entry, stats = build_graph(data, knn_k=16, max_degree=32)
    return data, qs, G, entry, stats


@functools.lru_cache(maxsize=None)
def c2_small(n: int = 20_000, clusters: int = 20, nq: int = 200, pivots: int = 80):
    """The integer-valued 128-d workload at reduced n (same points per
    cluster as the 1M-point configuration), with nearest-pivot entries."""
    spec = SPECS["c2"].scaled(n=n, n_centers=clusters, nq=nq)
    data, qs = make_points(spec)
    G, entry, stats = build_graph(data, knn_k=16, max_degree=32)
    piv = pick_pivots(n, pivots, spec.seed)
    return data, qs, G, entry, piv
