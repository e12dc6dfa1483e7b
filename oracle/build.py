"""FINGER construction (Algorithm 2) in float64.  Test infrastructure only.

Follows Section 3.3 ("Low-rank Estimation", Eq. 3, Proposition 3.1,
"Distribution Matching", "Overall Algorithm") and Algorithm 2, with these
readings of the text:

* Residuals.  Algorithm 2 writes cos(d, d') and cos(Pd, Pd') but the
  quantities being modelled are angles between residuals w.r.t. the centre
  node c (Section 3.2, Fig. 3/4 captions, Algorithm 3), so X and Y are taken
  on d_res = d - (c.d / c.c) c and d'_res.
* Sigma.  Algorithm 2 names the mean squared deviation sigma while
  distribution matching scales by sigma / sigma_hat and speaks of matching
  mean and variance; sigma is read as the population standard deviation
  (the square root of Algorithm 2's quantity).  ``sigma_mode="variance"``
  keeps the literal reading.
* Basis.  P = U_{1:r}^T from the SVD of D_res (m x N), uncentred
  (Proposition 3.1).  Algorithm 3's estimate depends only on P's row space
  (cosines of P-projections are unchanged by signs or rotations of P's
  rows); each row's sign is fixed so that its largest-magnitude entry is
  positive, which the learned gate's per-coordinate features need.
* Degenerate vectors.  c.c = 0 gives no projection (alpha = 0); a cosine
  with a zero vector is 0; sigma_hat = 0 makes the scale factor 1.
* Samples.  One pair per sampled node; N_s = min(n, n_samples) nodes drawn
  by ``oracle.rng.sample_pairs``; only d_res enters D_res.
"""
from __future__ import annotations

import numpy as np

from .rng import sample_pairs


def split(x: np.ndarray, c: np.ndarray):
    """Eq. 1: x = x_proj + x_res with x_proj = (c.x / c.c) c.  Rows of x
    (.., m) share one centre c (m,).  Returns (alpha, x_proj, x_res)."""
    x = np.asarray(x, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    cc = float(c @ c)
    alpha = (x @ c) / cc if cc > 0 else np.zeros(x.shape[:-1])
    proj = np.multiply.outer(alpha, c)
    return alpha, proj, x - proj


def cosine_rows(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Row-wise cosine; 0 where either row is the zero vector."""
    num = (A * B).sum(-1)
    den = np.sqrt((A * A).sum(-1) * (B * B).sum(-1))
    return np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0)


def residual_pairs(data: np.ndarray, c: np.ndarray, d: np.ndarray,
                   dp: np.ndarray):
    """d_res and d'_res of each sample w.r.t. its own centre (Eq. 1)."""
    C = np.asarray(data[c], dtype=np.float64)
    D = np.asarray(data[d], dtype=np.float64)
    Dp = np.asarray(data[dp], dtype=np.float64)
    cc = (C * C).sum(1)
    safe = np.where(cc > 0, cc, 1.0)
    a = np.where(cc > 0, (D * C).sum(1) / safe, 0.0)
    ap = np.where(cc > 0, (Dp * C).sum(1) / safe, 0.0)
    return D - a[:, None] * C, Dp - ap[:, None] * C


def canonical_signs(P: np.ndarray) -> np.ndarray:
    """Flip each row so that its entry of largest magnitude (the first one on
    ties) is positive.  Singular vectors are defined up to sign; fixing it
    makes per-coordinate features of P-projections comparable across
    implementations."""
    P = P.copy()
    for i in range(P.shape[0]):
        j = int(np.argmax(np.abs(P[i])))
        if P[i, j] < 0:
            P[i] = -P[i]
    return P


def basis_from_residuals(Dres_rows: np.ndarray, rank: int) -> tuple[np.ndarray, np.ndarray]:
    """Proposition 3.1: the first r left singular vectors of D_res (m x N)
    as the rows of P (signs canonical).  Returns (P [r, m], singular values)."""
    U, S, _ = np.linalg.svd(Dres_rows.T, full_matrices=False)
    return canonical_signs(U[:, :rank].T), S


def dm_stats(X: np.ndarray, Y: np.ndarray, sigma_mode: str = "std"):
    """Distribution matching statistics of Algorithm 2: means, spreads and
    the mean absolute error after matching (the correction term epsilon)."""
    N = X.shape[0]
    mu = X.sum() / N
    mu_hat = Y.sum() / N
    var = ((X - mu) ** 2).sum() / N
    var_hat = ((Y - mu_hat) ** 2).sum() / N
    if sigma_mode == "std":
        sigma, sigma_hat = np.sqrt(var), np.sqrt(var_hat)
    elif sigma_mode == "variance":
        sigma, sigma_hat = var, var_hat
    else:
        raise ValueError(sigma_mode)
    scale = sigma / sigma_hat if sigma_hat > 0 else 1.0
    eps = np.abs((Y - mu_hat) * scale + mu - X).sum() / N
    return dict(mu=float(mu), sigma=float(sigma), mu_hat=float(mu_hat),
                sigma_hat=float(sigma_hat), eps=float(eps))


def build(data: np.ndarray, graph: np.ndarray, rank: int,
          n_samples: int = 100_000, seed: int = 0,
          sigma_mode: str = "std", basis: np.ndarray | None = None) -> dict:
    """Algorithm 2.  Returns P (r x m, float64), the five distribution
    parameters, the Pearson correlation of X and Y (Supplementary E) and
    the intermediate samples for inspection.

    ``basis`` (r x m) replaces Proposition 3.1's P, e.g. with the random
    Gaussian projections of RPLSH that the ablation study compares against
    (Section 4.4); the distribution-matching statistics are then taken with
    that P."""
    c, d, dp, idx = sample_pairs(graph, n_samples, seed)
    Dres, Dres2 = residual_pairs(data, c, d, dp)
    if basis is None:
        P, S = basis_from_residuals(Dres, rank)
    else:
        P, S = np.asarray(basis, dtype=np.float64), None
        assert P.shape == (rank, data.shape[1])
    X = cosine_rows(Dres, Dres2)
    Y = cosine_rows(Dres @ P.T, Dres2 @ P.T)
    out = dm_stats(X, Y, sigma_mode)
    out.update(P=P, singular_values=S, X=X, Y=Y, corr=pearson(X, Y),
               samples=(c, d, dp, idx), rank=rank)
    return out


def pearson(X: np.ndarray, Y: np.ndarray) -> float:
    """Correlation coefficient of two samples (0 if either is constant)."""
    dx, dy = X - X.mean(), Y - Y.mean()
    den = np.sqrt((dx * dx).sum() * (dy * dy).sum())
    return float((dx * dy).sum() / den) if den > 0 else 0.0


def select_rank(data: np.ndarray, graph: np.ndarray, target: float = 0.7, start: int = 8,
                step: int = 8, max_rank: int | None = None, **build_kw) -> tuple[int, dict]:
    """Supplementary E's rule of thumb: start at r = 8 and grow r by 8 until
    the correlation of X and Y from Algorithm 2 reaches 0.7 (or r reaches
    min(m, max_rank)).  Returns (r, tables of that r)."""
    m = data.shape[1]
    top = m if max_rank is None else min(m, max_rank)
    r = min(start, top)
    while True:
        t = build(data, graph, r, **build_kw)
        if t["corr"] >= target or r >= top:
            return r, t
        r = min(r + step, top)


def identity_dm(tables: dict) -> dict:
    """Copy of ``tables`` with distribution matching switched off
    (mu = mu_hat = 0, sigma = sigma_hat = 1, eps = 0): the low-rank-only
    estimate of the ablation study (Section 4.3)."""
    t = dict(tables)
    t.update(mu=0.0, sigma=1.0, mu_hat=0.0, sigma_hat=1.0, eps=0.0)
    return t
