"""Pins for the oracle's distances, brute-force kNN and greedy search
(Algorithm 1).  CPU only."""
import json
import os

import numpy as np
import pytest
from scipy.spatial.distance import cdist

from oracle.knn import brute_force_knn, recall_at_k, sqdist
from oracle.search import search, search_batch
from workloads import SPECS, build_graph, make_points

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _traces():
    with open(os.path.join(GOLD, "search_traces.json")) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _traces(), ids=lambda c: c["name"])
def test_hand_traced_search(case):
    data = np.array(case["points"], dtype=np.float64)
    G = np.array(case["graph"], dtype=np.int32)
    ids, d2, cnt, _ = search(data, G, np.array(case["query"]), case["entry"],
                             case["ef"], case["k"])
    assert ids.tolist() == case["expect_ids"]
    np.testing.assert_allclose(d2, case["expect_d2"], rtol=1e-12, atol=1e-12)
    for kname, v in case["expect_counters"].items():
        assert cnt[kname] == v, kname


def test_sqdist_closed_form():
    # 3-4-5 triangle and an integer lattice point
    assert sqdist(np.array([0.0, 0.0]), np.array([[3.0, 4.0]]))[0] == 25.0
    x = np.arange(8.0)
    y = x[::-1].copy()
    assert sqdist(x, y[None])[0] == sum((2 * i - 7) ** 2 for i in range(8))


def test_bruteforce_matches_scipy_and_tie_order():
    rng = np.random.default_rng(3)
    data = rng.integers(0, 4, size=(60, 3)).astype(np.float64)   # many exact ties
    qs = rng.integers(0, 4, size=(7, 3)).astype(np.float64)
    ids, d2 = brute_force_knn(data, qs, 9)
    D = cdist(qs, data, "sqeuclidean")
    for i in range(qs.shape[0]):
        order = np.argsort(D[i], kind="stable")[:9]     # stable: equal d2 keep id order
        assert ids[i].tolist() == order.tolist()
        np.testing.assert_array_equal(d2[i], D[i][order])


def test_bruteforce_pads_when_k_exceeds_n():
    ids, d2 = brute_force_knn(np.eye(3), np.zeros((1, 3)), 5)
    assert ids[0].tolist() == [0, 1, 2, -1, -1]
    assert np.isinf(d2[0, 3:]).all()


def test_recall_definition():
    gt = np.array([[1, 2, 3, 4]])
    assert recall_at_k(np.array([[4, 3, 9, 8]]), gt, 4) == 0.5
    # tie-tolerant: id 9 sits at the same distance as the 4th true neighbour
    assert recall_at_k(np.array([[1, 2, 3, 9]]), gt, 4,
                       np.array([[0.0, 1.0, 1.0, 2.0]]),
                       np.array([[0.0, 1.0, 1.0, 2.0]])) == 1.0


@pytest.fixture(scope="module")
def small_c1():
    spec = SPECS["c1"].scaled(n=600, n_centers=6, nq=25)
    data, qs = make_points(spec)
    G, entry, _ = build_graph(data, knn_k=8, max_degree=12)
    return data, qs, G, entry


def test_exhaustive_search_is_exact_knn(small_c1):
    """ef >= n on a graph where every node is reachable: every node is
    admitted and expanded, so T is the exact top-ef, i.e. brute force."""
    data, qs, G, entry = small_c1
    n = data.shape[0]
    ids, d2, cnt, _ = search_batch(data, G, qs, entry, n, 10)
    gi, gd = brute_force_knn(data, qs, 10)
    np.testing.assert_array_equal(ids, gi)
    np.testing.assert_array_equal(d2, gd)
    assert (cnt[:, 4] == n).all()          # visited everything


def test_row_order_invariance(small_c1):
    """Within one expansion the final T is the top-ef of T plus the admitted
    keys whatever the order, so shuffling every adjacency row changes
    nothing (results and counters)."""
    data, qs, G, entry = small_c1
    rng = np.random.default_rng(1)
    G2 = G.copy()
    for i in range(G.shape[0]):
        deg = int((G[i] >= 0).sum())
        G2[i, :deg] = rng.permutation(G[i, :deg])
    a = search_batch(data, G, qs, entry, 12, 10)
    b = search_batch(data, G2, qs, entry, 12, 10)
    for x, y in zip(a[:3], b[:3]):
        np.testing.assert_array_equal(x, y)


def test_sequential_equals_batched_for_plain(small_c1):
    data, qs, G, entry = small_c1
    a = search_batch(data, G, qs, entry, 16, 10, ub_mode="batched")
    b = search_batch(data, G, qs, entry, 16, 10, ub_mode="sequential")
    for x, y in zip(a[:3], b[:3]):
        np.testing.assert_array_equal(x, y)


def test_returned_distances_are_exact(small_c1):
    data, qs, G, entry = small_c1
    ids, d2, _, _ = search_batch(data, G, qs, entry, 8, 5)
    for i in range(qs.shape[0]):
        np.testing.assert_array_equal(d2[i], sqdist(qs[i], data[ids[i]]))
        assert list(zip(d2[i], ids[i])) == sorted(zip(d2[i], ids[i]))


def test_k_larger_than_ef_uses_k(small_c1):
    data, qs, G, entry = small_c1
    a = search_batch(data, G, qs[:5], entry, 3, 10)
    b = search_batch(data, G, qs[:5], entry, 10, 10)
    np.testing.assert_array_equal(a[0], b[0])
