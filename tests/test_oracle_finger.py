"""Pins for the oracle's FINGER construction (Algorithm 2), estimate
(Algorithm 3) and approximate search (Algorithm 4).  CPU only."""
import json
import os

import numpy as np
import pytest

from oracle.build import basis_from_residuals, build, dm_stats, identity_dm, residual_pairs
from oracle.estimate import estimate, parts, true_cosine
from oracle.knn import sqdist
from oracle.rng import sample_pairs, splitmix64
from oracle.search import search_batch
from workloads import SPECS, build_graph, make_points

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_published_outputs():
    # first outputs of SplitMix64 seeded with 0 (Steele, Lea, Flood 2014;
    # the same sequence Java's SplittableRandom and Vigna's reference give)
    assert [splitmix64(0, j) for j in range(4)] == [
        0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F, 0xF88BB8A8724C81EC]


def test_sample_pairs_recipe():
    G = np.array([[1, 2, 3, -1], [0, -1, -1, -1], [0, 3, -1, -1], [0, 2, 1, -1]], dtype=np.int32)
    c, d, dp, idx = sample_pairs(G, 100, 7)
    assert 1 not in c.tolist()              # degree-1 node is dropped
    assert idx.tolist() == [0, 2, 3]
    for ci, di, dpi in zip(c, d, dp):
        row = G[ci][G[ci] >= 0].tolist()
        assert di in row and dpi in row and di != dpi
    # subsampling path: ids drawn with replacement from the counter stream
    c2, _, _, idx2 = sample_pairs(G, 2, 7)
    assert all(ci == splitmix64(7, 3 * i) % 4 for ci, i in zip(c2, idx2))


@pytest.fixture(scope="module")
def c1_small():
    spec = SPECS["c1"].scaled(n=2000, n_centers=10, nq=40)
    data, qs = make_points(spec)
    G, entry, _ = build_graph(data, knn_k=12, max_degree=16)
    return data.astype(np.float64), qs.astype(np.float64), G, entry


def test_prop31_svd_basis_is_top_eigvecs_and_optimal(c1_small):
    """Proposition 3.1: the top-r left singular vectors of D_res minimise
    Eq. 3.  Checked two ways: (i) the SVD projector equals the projector on
    the top-r eigenvectors of D_res D_res^T (a different LAPACK route);
    (ii) on sampled residual pairs the SVD basis has a smaller Eq. 3
    objective than random orthonormal bases of the same rank."""
    data, _, G, _ = c1_small
    c, d, dp, _ = sample_pairs(G, 10_000, 0)
    Dres, _ = residual_pairs(data, c, d, dp)
    r = 8
    P, S = basis_from_residuals(Dres, r)
    w, V = np.linalg.eigh(Dres.T @ Dres)
    Ve = V[:, np.argsort(w)[::-1][:r]]
    assert S[r - 1] > S[r] * 1.0001
    np.testing.assert_allclose(P.T @ P, Ve @ Ve.T, atol=1e-10)
    rng = np.random.default_rng(0)
    i = rng.integers(0, Dres.shape[0], 4000)
    j = rng.integers(0, Dres.shape[0], 4000)
    Z = Dres[i] - Dres[j]

    def obj(B):
        return abs(((Z @ B.T) ** 2).sum() - (Z ** 2).sum())

    best = obj(P)
    for _ in range(5):
        Q, _ = np.linalg.qr(rng.standard_normal((data.shape[1], r)))
        assert obj(Q.T) > best


def test_canonical_signs():
    from oracle.build import canonical_signs
    rng = np.random.default_rng(8)
    Q, _ = np.linalg.qr(rng.normal(size=(9, 4)))
    P = canonical_signs(-Q.T)
    for row in P:
        assert row[np.argmax(np.abs(row))] > 0
    np.testing.assert_allclose(P.T @ P, Q @ Q.T, atol=1e-12)


def test_dm_matches_moments_exactly():
    rng = np.random.default_rng(0)
    X = rng.normal(0.3, 0.1, 5000)
    Y = 1.7 * X + 0.2 + rng.normal(0, 0.05, 5000)
    s = dm_stats(X, Y)
    t = (Y - s["mu_hat"]) * s["sigma"] / s["sigma_hat"] + s["mu"]
    assert abs(t.mean() - s["mu"]) < 1e-12
    assert abs(t.std() - s["sigma"]) < 1e-12
    assert s["eps"] == pytest.approx(np.abs(t - X).mean(), rel=1e-12)
    # literal reading keeps the variances as the scales
    v = dm_stats(X, Y, "variance")
    assert v["sigma"] == pytest.approx(s["sigma"] ** 2, rel=1e-12)


def test_full_rank_basis_makes_dm_trivial(c1_small):
    """r = m with an orthonormal P preserves every cosine, so Y = X,
    mu_hat = mu, sigma_hat = sigma and eps = 0."""
    data, _, G, _ = c1_small
    t = build(data, G, data.shape[1], n_samples=3000, seed=1)
    np.testing.assert_allclose(t["Y"], t["X"], atol=1e-12)
    assert t["mu_hat"] == pytest.approx(t["mu"], abs=1e-12)
    assert t["sigma_hat"] == pytest.approx(t["sigma"], abs=1e-12)
    assert t["eps"] < 1e-12


def _random_case(seed, m=12):
    rng = np.random.default_rng(seed)
    q = rng.normal(size=m) * 3
    c = rng.normal(size=m) * 3
    D = c + rng.normal(size=(9, m))
    return q, c, D


def test_full_rank_identity_dm_estimate_is_exact():
    """Eq. 2 is an identity: with P orthonormal of rank m and distribution
    matching switched off, t_hat = cos(q_res, d_res) and the estimate is the
    exact squared distance."""
    for seed in range(5):
        q, c, D = _random_case(seed)
        Q, _ = np.linalg.qr(np.random.default_rng(seed + 100).normal(size=(12, 12)))
        tab = identity_dm({"P": Q.T})
        np.testing.assert_allclose(estimate(q, c, D, tab), sqdist(q, D), rtol=1e-12)


def test_point_on_centre_line_is_exact():
    """d = a c has d_res = 0, so the estimate is exact for any P and any
    distribution-matching constants."""
    q, c, _ = _random_case(1)
    D = np.stack([c, 0.5 * c, -2.0 * c])
    rng = np.random.default_rng(5)
    tab = {"P": rng.normal(size=(3, 12)), "mu": 0.4, "sigma": 0.1,
           "mu_hat": 0.2, "sigma_hat": 0.3, "eps": 0.05}
    np.testing.assert_allclose(estimate(q, c, D, tab), sqdist(q, D), rtol=1e-12)


def test_factorized_form_equals_direct_form():
    """Supplementary G's factorization: q.c from ||q||^2, ||c||^2 and the
    exact ||q - c||^2 (Section 3.2), ||q_res||^2 = ||q||^2 - ||q_proj||^2,
    P q_res = Pq - (c.q / c.c) Pc, and stored per-edge alpha_d, ||d_res||,
    u_d = P d_res / ||P d_res||.  Written here independently of the oracle's
    direct form and compared with it."""
    rng = np.random.default_rng(9)
    P = rng.normal(size=(5, 12))
    tab = {"P": P, "mu": 0.1, "sigma": 0.2, "mu_hat": 0.05, "sigma_hat": 0.3, "eps": 0.02}
    for seed in range(4):
        q, c, D = _random_case(seed)
        qq, cc = q @ q, c @ c
        delta = ((q - c) ** 2).sum()
        qc = (qq + cc - delta) / 2
        aq = qc / cc
        rq2 = qq - aq * qc
        w = P @ q - aq * (P @ c)
        ad = (D @ c) / cc
        Dres = D - ad[:, None] * c
        rd = np.sqrt((Dres ** 2).sum(1))
        Pd = Dres @ P.T
        u = Pd / np.sqrt((Pd ** 2).sum(1))[:, None]
        that = (u @ w) / np.sqrt(w @ w)
        t = (that - 0.05) * (0.2 / 0.3) + 0.1 + 0.02
        est = (aq - ad) ** 2 * cc + rq2 + rd ** 2 - 2 * np.sqrt(rq2) * rd * t
        np.testing.assert_allclose(est, estimate(q, c, D, tab), rtol=1e-10)


def test_estimate_invariant_to_basis_rotation():
    """Only P's row space matters: cos(R P x, R P y) = cos(P x, P y) for any
    orthogonal R, including sign flips of single rows."""
    q, c, D = _random_case(3)
    rng = np.random.default_rng(4)
    P = rng.normal(size=(6, 12))
    R, _ = np.linalg.qr(rng.normal(size=(6, 6)))
    tab = {"P": P, "mu": 0.1, "sigma": 0.2, "mu_hat": 0.05, "sigma_hat": 0.3, "eps": 0.02}
    tab2 = dict(tab, P=R @ P)
    np.testing.assert_allclose(estimate(q, c, D, tab), estimate(q, c, D, tab2), rtol=1e-12)


def test_estimate_parts_and_true_cosine():
    q, c, D = _random_case(7)
    p = parts(q, c, D, np.eye(12))
    # with P = I the low-rank cosine is the true residual cosine
    np.testing.assert_allclose(p["t_hat"], true_cosine(q, c, D), rtol=1e-12)
    assert p["cc"] == pytest.approx(c @ c)


def test_warmup_infinite_equals_plain(c1_small):
    data, qs, G, entry = c1_small
    tab = build(data, G, 8, n_samples=2000)
    a = search_batch(data, G, qs, entry, 24, 10)
    b = search_batch(data, G, qs, entry, 24, 10, mode="finger", tables=tab, warmup=10**9)
    for x, y in zip(a[:3], b[:3]):
        np.testing.assert_array_equal(x, y)


def test_full_rank_identity_finger_returns_plain_ids(c1_small):
    """With an exact estimate every skipped neighbour would have been
    rejected by the admission rule anyway, so ids and distances match plain
    search; only the exact-distance count drops."""
    data, qs, G, entry = c1_small
    m = data.shape[1]
    Q, _ = np.linalg.qr(np.random.default_rng(2).normal(size=(m, m)))
    tab = identity_dm({"P": Q.T})
    a = search_batch(data, G, qs, entry, 24, 10)
    b = search_batch(data, G, qs, entry, 24, 10, mode="finger", tables=tab)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    assert (b[2][:, 1] <= a[2][:, 1]).all() and b[2][:, 3].sum() > 0


def test_finger_soundness_and_counters(c1_small):
    data, qs, G, entry = c1_small
    tab = build(data, G, 8, n_samples=2000)
    for ub_mode in ("batched", "sequential"):
        ids, d2, cnt, margins = search_batch(data, G, qs, entry, 24, 10, mode="finger",
                                             tables=tab, ub_mode=ub_mode)
        for i in range(qs.shape[0]):
            np.testing.assert_array_equal(d2[i], sqdist(qs[i], data[ids[i]]))
        # exact distances = entry + (visited - 1 - skipped)
        np.testing.assert_array_equal(cnt[:, 1], cnt[:, 4] - cnt[:, 3])
        assert (cnt[:, 3] <= cnt[:, 2]).all()
        assert np.isfinite(margins).any()


def test_table1_extra_memory_formula():
    """Supplementary F: FINGER's extra memory is (r+2)|E| floats.  With
    HNSW's bottom-layer cap of 2M out-edges per node, (r+2) n 2M 4 bytes
    comes within 10% of every difference Table 1 prints."""
    with open(os.path.join(GOLD, "table1_sizes.json")) as f:
        rows = json.load(f)["rows"]
    for r in rows:
        formula = (r["r"] + 2) * r["n"] * 2 * r["M"] * 4 / 1e9
        printed = r["finger_gb"] - r["hnsw_gb"]
        assert abs(formula - printed) / printed < 0.10, r


def test_any_full_rank_orthonormal_basis_reproduces_x(c1_small):
    """Cosines are invariant under rotations, so any orthonormal basis of
    full rank gives Y = X: correlation 1 and no correction (Algorithm 2 with
    a supplied basis, the hook the RPLSH comparison uses)."""
    data, _, G, _ = c1_small
    m = data.shape[1]
    Q, _ = np.linalg.qr(np.random.default_rng(21).normal(size=(m, m)))
    t = build(data, G, m, n_samples=3000, seed=2, basis=Q.T)
    np.testing.assert_allclose(t["Y"], t["X"], atol=1e-12)
    assert t["corr"] == pytest.approx(1.0, abs=1e-12)
    assert t["eps"] < 1e-12


def test_pearson_matches_numpy():
    from oracle.build import pearson
    rng = np.random.default_rng(3)
    X = rng.normal(size=500)
    Y = 0.3 * X + rng.normal(size=500)
    assert pearson(X, Y) == pytest.approx(np.corrcoef(X, Y)[0, 1], rel=1e-12)
    assert pearson(X, np.full(500, 2.0)) == 0.0


def test_rank_rule_of_thumb(c1_small):
    """Supplementary E: the chosen r is a multiple of 8, reaches the target
    correlation, and r - 8 does not; unreachable targets stop at m."""
    from oracle.build import select_rank
    data, _, G, _ = c1_small
    m = data.shape[1]
    kw = dict(n_samples=4000, seed=3)
    for target in (0.5, 0.7, 0.9):
        r, t = select_rank(data, G, target=target, **kw)
        assert r % 8 == 0 and 8 <= r <= m
        assert t["corr"] >= target or r == m
        if r > 8:
            assert build(data, G, r - 8, **kw)["corr"] < target
    r, t = select_rank(data, G, target=1.5, **kw)
    assert r == m
    r, _ = select_rank(data, G, target=-1.0, **kw)
    assert r == 8


def test_learned_basis_beats_random_projection(c1_small):
    """Section 3.3 / the ablation: at equal rank the SVD basis tracks the
    true residual angles better than random Gaussian projections."""
    from workloads import gaussian_projection
    data, _, G, _ = c1_small
    svd = build(data, G, 8, n_samples=4000, seed=4)
    rp = build(data, G, 8, n_samples=4000, seed=4,
               basis=gaussian_projection(8, data.shape[1], 7))
    assert svd["corr"] > rp["corr"]
    assert svd["eps"] < rp["eps"]
