"""The paper's ablation variants and rank rule on the library's kernels.

Section 4.4 compares FINGER (learned basis plus distribution matching) with
its low-rank part alone and with random-projection angle estimates (RPLSH:
a Gaussian r x m matrix P, Section 3.3) with and without distribution
matching, by the approximation error |t - t_hat| / |t| of the residual
cosine and by recall against the effective number of distance calls
a + b r / m (a full-length, b r-dimensional calls).  Supplementary E picks r
by growing it in steps of 8 until the correlation of Algorithm 2's X and Y
reaches 0.7.

Every variant is the same search kernel with different tables: the basis
comes from the build (or the build's ``basis`` option), and "no distribution
matching" is the override mu = mu_hat = 0, sigma = sigma_hat = 1, eps = 0.
"""
from __future__ import annotations

import numpy as np
import torch

from . import api, gate

VARIANTS = ("finger", "lowrank", "rplsh+dm", "rplsh")
NO_DM = (0.0, 1.0, 0.0, 1.0, 0.0)   # mu, sigma, mu_hat, sigma_hat, eps


def select_rank(data: torch.Tensor, graph: torch.Tensor, target: float = 0.7, start: int = 8,
                step: int = 8, max_rank: int | None = None, **build_kw):
    """Supplementary E's rule on the library's own X, Y statistics (the
    build's corr_xy).  Returns (rank, tables, [(rank, corr), ...])."""
    m = data.shape[1]
    top = min(m, 256 if max_rank is None else max_rank)
    r = min(start, top)
    hist = []
    while True:
        t = api.finger_build_tables(data, graph, rank=r, **build_kw)
        c = t.info()["corr_xy"]
        hist.append((r, c))
        if c >= target or r >= top:
            return r, t, hist
        t.close()
        r = min(r + step, top)


def variant_tables(data: torch.Tensor, graph: torch.Tensor, rank: int, variant: str,
                   projection: np.ndarray | None = None, **build_kw) -> api.Tables:
    """Tables for one ablation variant; ``projection`` is the r x m Gaussian
    matrix for the RPLSH variants."""
    if variant == "finger":
        return api.finger_build_tables(data, graph, rank=rank, **build_kw)
    if variant == "lowrank":
        return api.finger_build_tables(data, graph, rank=rank, dm_override=NO_DM, **build_kw)
    if projection is None:
        raise ValueError("the RPLSH variants need a projection matrix")
    if variant == "rplsh+dm":
        return api.finger_build_tables(data, graph, rank=rank, basis=projection, **build_kw)
    if variant == "rplsh":
        return api.finger_build_tables(data, graph, rank=rank, basis=projection,
                                       dm_override=NO_DM, **build_kw)
    raise ValueError(f"unknown variant {variant}")


def approximation_error(tables: api.Tables, queries: torch.Tensor, ef: int,
                        capacity: int = 1 << 22) -> dict:
    """|t - t_used| / |t| over every edge that FINGER searches of ``queries``
    screen at ``ef``: t is the true residual cosine (from the logged exact
    distance, finger_gate_targets), t_used the estimate the screen compares,
    i.e. t_hat mapped by the tables' distribution matching (without the
    error-correction offset eps, which is a deliberate bias, not part of the
    estimate).  Edges with t = 0 are left out."""
    feats, targs, total = gate.collect_log(tables, queries, ef, capacity=capacity)
    inf = tables.info()
    r = inf["rank"]
    t = api.finger_gate_targets(feats, targs, feats.shape[0], r).double()
    t_hat = feats[:, 2 * r].double()
    scale = inf["sigma"] / inf["sigma_hat"] if inf["sigma_hat"] > 0 else 1.0
    t_used = (t_hat - inf["mu_hat"]) * scale + inf["mu"]
    keep = t.abs() > 0
    err = ((t - t_used).abs()[keep] / t.abs()[keep]).cpu().numpy()
    return dict(median=float(np.median(err)), mean=float(err.mean()),
                p90=float(np.quantile(err, 0.9)), edges=int(err.size), screened=int(total))


def effective_calls(counters: np.ndarray, rank: int, m: int) -> float:
    """Mean effective distance calls per query: exact + screened r / m."""
    return float(counters[:, 1].mean() + counters[:, 2].mean() * rank / m)
