"""FINGER's approximate distance (Algorithm 3) in float64, straight from the
definitions of Section 3.2 and 3.3.  Test infrastructure only.

For a query q, centre c and neighbours d of c:
  q = q_proj + q_res, d = d_proj + d_res                          (Eq. 1)
  ||q - d||^2 = ||q_proj - d_proj||^2 + ||q_res||^2 + ||d_res||^2
                - 2 q_res . d_res                                 (Eq. 2)
and the one unknown term q_res . d_res is replaced by
||q_res|| ||d_res|| t, where t_hat = cos(P q_res, P d_res) and
t = (t_hat - mu_hat) sigma / sigma_hat + mu + eps (Algorithm 3).

Readings: t is not clipped to [-1, 1], so an estimate may be negative; a
cosine with a zero vector is 0; when d_res = 0 or q_res = 0 (a point on the
line through c) the last term of Eq. 2 vanishes and the estimate is exact;
sigma_hat = 0 makes the scale 1.  This module never uses the law-of-cosines shortcut for
q.c or the stored projections P c and P d_res: those are the library's
factorization, checked against this direct form by the tests.
"""
from __future__ import annotations

import numpy as np

from .build import split


def dm_map(t_hat: np.ndarray, tables: dict) -> np.ndarray:
    """Distribution matching plus the error correction (Algorithm 3)."""
    sh = tables["sigma_hat"]
    scale = tables["sigma"] / sh if sh > 0 else 1.0
    return (t_hat - tables["mu_hat"]) * scale + tables["mu"] + tables["eps"]


def parts(q: np.ndarray, c: np.ndarray, D: np.ndarray, P: np.ndarray,
          codes: np.ndarray | None = None) -> dict:
    """The pieces of Eq. 2 for every row of D, plus the low-rank cosine.

    With ``codes`` (rows = unit vectors standing in for P d_res/||P d_res||,
    e.g. after BF16/FP8 rounding) t_hat is cos(P q_res, .) against them."""
    q = np.asarray(q, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    D = np.atleast_2d(np.asarray(D, dtype=np.float64))
    aq, qp, qr = split(q, c)
    ad, dp, dr = split(D, c)
    Pq = P @ qr
    nq = np.sqrt(Pq @ Pq)
    if codes is None:
        Pd = dr @ P.T
        nd = np.sqrt((Pd * Pd).sum(-1))
        den = nq * nd
        t_hat = np.where(den > 0, (Pd @ Pq) / np.where(den > 0, den, 1.0), 0.0)
    else:
        U = np.atleast_2d(np.asarray(codes, dtype=np.float64))
        t_hat = (U @ Pq) / nq if nq > 0 else np.zeros(U.shape[0])
    return dict(
        proj=((qp - dp) ** 2).sum(-1),
        rq=float(np.sqrt(qr @ qr)),
        rd=np.sqrt((dr * dr).sum(-1)),
        t_hat=t_hat,
        alpha_q=float(aq),
        alpha_d=ad,
        cc=float(c @ c),
    )


def combine(p: dict, t: np.ndarray) -> np.ndarray:
    """Eq. 2 with q_res . d_res replaced by ||q_res|| ||d_res|| t."""
    return p["proj"] + p["rq"] ** 2 + p["rd"] ** 2 - 2.0 * p["rq"] * p["rd"] * t


def estimate(q, c, D, tables: dict, codes=None) -> np.ndarray:
    """Algorithm 3 for each row of D (squared distance estimate)."""
    p = parts(q, c, D, tables["P"], codes)
    return combine(p, dm_map(p["t_hat"], tables))


def estimate_ip(q, c, D, tables: dict, codes=None) -> np.ndarray:
    """Supplementary A for inner products: q.d = q_proj.d_proj + q_res.d_res
    with q_proj.d_proj = alpha_q alpha_d (c.c) and q_res.d_res replaced by
    ||q_res|| ||d_res|| t as in Algorithm 3.  Returned negated (the search
    minimises -q.d), so adding eps to t again lowers the estimate."""
    p = parts(q, c, D, tables["P"], codes)
    t = dm_map(p["t_hat"], tables)
    return -(p["alpha_q"] * p["alpha_d"] * p["cc"] + p["rq"] * p["rd"] * t)


def true_cosine(q, c, D) -> np.ndarray:
    """cos(q_res, d_res), the quantity Algorithm 3 estimates (0 if either
    residual is zero)."""
    _, _, qr = split(np.asarray(q, dtype=np.float64), np.asarray(c, dtype=np.float64))
    _, _, dr = split(np.atleast_2d(np.asarray(D, dtype=np.float64)), np.asarray(c, dtype=np.float64))
    num = dr @ qr
    den = np.sqrt(qr @ qr) * np.sqrt((dr * dr).sum(-1))
    return np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0)
