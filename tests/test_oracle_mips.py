"""Pins for the oracle's inner-product (maximum inner-product search)
variant of Supplementary A.  CPU only."""
import numpy as np
import pytest

from oracle.build import build, identity_dm
from oracle.estimate import estimate, estimate_ip
from oracle.knn import brute_force_knn, ipdist
from oracle.search import pivot_entries, search_batch
from workloads import SPECS, build_graph, make_points


def _case(seed, m=12):
    rng = np.random.default_rng(seed)
    q = rng.normal(size=m) * 2
    c = rng.normal(size=m) * 2
    D = c + rng.normal(size=(7, m))
    return q, c, D


def test_full_rank_identity_ip_estimate_is_exact():
    """q.d = q_proj.d_proj + q_res.d_res is an identity: with an orthonormal
    P of full rank and no distribution matching the estimate is -q.d."""
    for seed in range(4):
        q, c, D = _case(seed)
        Q, _ = np.linalg.qr(np.random.default_rng(seed + 50).normal(size=(12, 12)))
        tab = identity_dm({"P": Q.T})
        np.testing.assert_allclose(estimate_ip(q, c, D, tab), -(D @ q), rtol=1e-12, atol=1e-12)


def test_ip_and_l2_estimates_are_one_decomposition():
    """With the same t, |q - d|^2 = |q|^2 + |d|^2 - 2 q.d holds between the
    two estimates for any basis and distribution-matching constants."""
    rng = np.random.default_rng(2)
    tab = {"P": rng.normal(size=(4, 12)), "mu": 0.2, "sigma": 0.15, "mu_hat": 0.1,
           "sigma_hat": 0.25, "eps": 0.03}
    for seed in range(4):
        q, c, D = _case(seed)
        l2 = estimate(q, c, D, tab)
        ip = estimate_ip(q, c, D, tab)
        np.testing.assert_allclose(l2, q @ q + (D * D).sum(1) + 2 * ip, rtol=1e-10)


def test_point_on_centre_line_ip_is_exact():
    q, c, _ = _case(5)
    D = np.stack([c, -1.5 * c, 0.25 * c])
    rng = np.random.default_rng(1)
    tab = {"P": rng.normal(size=(3, 12)), "mu": 0.4, "sigma": 0.1, "mu_hat": 0.2,
           "sigma_hat": 0.3, "eps": 0.05}
    np.testing.assert_allclose(estimate_ip(q, c, D, tab), -(D @ q), rtol=1e-12)


def test_brute_force_ip_orders_by_largest_inner_product():
    rng = np.random.default_rng(4)
    X = rng.integers(-3, 4, size=(200, 6)).astype(np.float64)   # many ties
    q = rng.integers(-3, 4, size=6).astype(np.float64)
    ids, d = brute_force_knn(X, q, 15, metric="ip")
    s = X @ q
    want = sorted(range(200), key=lambda i: (-s[i], i))[:15]
    assert ids[0].tolist() == want
    np.testing.assert_array_equal(d[0], -s[want])
    np.testing.assert_array_equal(ipdist(q, X), -s)


@pytest.fixture(scope="module")
def small():
    spec = SPECS["c1"].scaled(n=1500, n_centers=8, nq=12)
    data, qs = make_points(spec)
    G, entry, _ = build_graph(data, knn_k=12, max_degree=16)
    return data.astype(np.float64), qs.astype(np.float64), G, entry


def test_exhaustive_ip_search_is_exact(small):
    """With ef = n the search expands every reachable node, so its top K are
    the brute-force K largest inner products."""
    data, qs, G, entry = small
    n = data.shape[0]
    ids, d, _, _ = search_batch(data, G, qs, entry, n, 10, metric="ip")
    bi, bd = brute_force_knn(data, qs, 10, metric="ip")
    np.testing.assert_array_equal(ids, bi)
    np.testing.assert_allclose(d, bd, rtol=1e-12)


def test_ip_finger_search_soundness(small):
    data, qs, G, entry = small
    tab = build(data, G, 8, n_samples=1500)
    ids, d, cnt, margin = search_batch(data, G, qs, entry, 24, 10, mode="finger", tables=tab,
                                       metric="ip")
    for i in range(qs.shape[0]):
        np.testing.assert_allclose(d[i], -(data[ids[i]] @ qs[i]), rtol=1e-12)
        assert (np.diff(d[i]) >= 0).all()
    np.testing.assert_array_equal(cnt[:, 1], cnt[:, 4] - cnt[:, 3])
    assert cnt[:, 3].sum() > 0
    # full rank and no matching: FINGER returns plain's ids
    m = data.shape[1]
    Q, _ = np.linalg.qr(np.random.default_rng(9).normal(size=(m, m)))
    exact = identity_dm({"P": Q.T})
    a = search_batch(data, G, qs, entry, 24, 10, metric="ip")
    b = search_batch(data, G, qs, entry, 24, 10, mode="finger", tables=exact, metric="ip")
    np.testing.assert_array_equal(a[0], b[0])


def test_ip_pivot_entries():
    rng = np.random.default_rng(6)
    X = rng.normal(size=(50, 5))
    qs = rng.normal(size=(7, 5))
    piv = np.array([3, 9, 14, 27, 41])
    ent = pivot_entries(qs, X, piv, metric="ip")
    for q, e in zip(qs, ent):
        assert e == piv[int(np.argmax(X[piv] @ q))]
