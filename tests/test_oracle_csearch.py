"""Pins for the compiled float64 search (oracle/csearch.c): the hand-traced
runs of Algorithm 1, the exhaustive-search and exact-estimate special
cases, W = infinity, and agreement with the NumPy oracle's search on the
same inputs (two independent renderings of Algorithms 1 and 4).  CPU only."""
import json
import os

import numpy as np
import pytest

from oracle import csearch
from oracle.build import build, identity_dm
from oracle.knn import brute_force_knn
from oracle.search import search_batch
from workloads import SPECS, build_graph, make_points

GOLD = os.path.join(os.path.dirname(__file__), "golden")
COUNTERS = ("expansions", "exact", "screened", "skipped", "visited", "preps")


@pytest.fixture(scope="module")
def small():
    spec = SPECS["c1"].scaled(n=2000, n_centers=10, nq=40)
    data, qs = make_points(spec)
    G, entry, _ = build_graph(data, knn_k=12, max_degree=16)
    return data.astype(np.float64), qs.astype(np.float64), G, entry


def _traces():
    with open(os.path.join(GOLD, "search_traces.json")) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _traces(), ids=lambda c: c["name"])
def test_hand_traced_search(case):
    data = np.array(case["points"], dtype=np.float64)
    G = np.array(case["graph"], dtype=np.int32)
    ids, d2, cnt, _ = csearch.search_batch(data, G, np.array([case["query"]], dtype=np.float64),
                                           case["entry"], case["ef"], case["k"])
    assert ids[0].tolist() == case["expect_ids"]
    np.testing.assert_allclose(d2[0], case["expect_d2"], rtol=1e-12, atol=1e-12)
    for kname, v in case["expect_counters"].items():
        assert cnt[0, COUNTERS.index(kname)] == v, kname


@pytest.mark.parametrize("metric", ["l2", "ip"])
def test_exhaustive_search_is_brute_force(small, metric):
    """ef = n: every reachable node is admitted and expanded (the graph is
    connected by construction), so the top K are the brute-force top K."""
    data, qs, G, entry = small
    ids, d, cnt, _ = csearch.search_batch(data, G, qs, entry, data.shape[0], 10, metric=metric)
    bi, bd = brute_force_knn(data, qs, 10, metric=metric)
    np.testing.assert_array_equal(ids, bi)
    np.testing.assert_allclose(d, bd, rtol=1e-12)
    assert (cnt[:, 4] == data.shape[0]).all()


def test_warmup_infinite_equals_plain(small):
    data, qs, G, entry = small
    tab = build(data, G, 8, n_samples=2000)
    a = csearch.search_batch(data, G, qs, entry, 24, 10)
    b = csearch.search_batch(data, G, qs, entry, 24, 10, mode="finger", tables=tab, warmup=10**9)
    for x, y in zip(a[:3], b[:3]):
        np.testing.assert_array_equal(x, y)


@pytest.mark.parametrize("metric", ["l2", "ip"])
def test_exact_estimate_returns_plain_ids(small, metric):
    """Full-rank orthonormal P with identity matching makes Eq. 2 exact, so
    a skipped neighbour is one the admission rule would have rejected: ids
    and distances equal plain search, with fewer exact distances."""
    data, qs, G, entry = small
    m = data.shape[1]
    Q, _ = np.linalg.qr(np.random.default_rng(2).normal(size=(m, m)))
    tab = identity_dm({"P": Q.T})
    a = csearch.search_batch(data, G, qs, entry, 24, 10, metric=metric)
    b = csearch.search_batch(data, G, qs, entry, 24, 10, mode="finger", tables=tab, metric=metric)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    assert (b[2][:, 1] <= a[2][:, 1]).all() and b[2][:, 3].sum() > 0


@pytest.mark.parametrize("metric", ["l2", "ip"])
def test_agrees_with_numpy_oracle(small, metric):
    """Same ids, distances, counters and screening margins as the NumPy
    oracle (the float64 sums run in a different order, so distances and
    margins agree to rounding; every margin here is far above it)."""
    data, qs, G, entry = small
    tab = build(data, G, 8, n_samples=2000)
    for mode, ef in (("plain", 24), ("finger", 24), ("finger", 40)):
        kw = dict(mode=mode, tables=tab, metric=metric) if mode == "finger" else dict(metric=metric)
        a = search_batch(data, G, qs, entry, ef, 10, **kw)
        b = csearch.search_batch(data, G, qs, entry, ef, 10, **kw)
        assert np.min(a[3]) > 1e-9
        np.testing.assert_array_equal(a[0], b[0])
        np.testing.assert_allclose(a[1], b[1], rtol=1e-12)
        np.testing.assert_array_equal(a[2], b[2])
        fin = np.isfinite(a[3])
        np.testing.assert_array_equal(fin, np.isfinite(b[3]))
        np.testing.assert_allclose(a[3][fin], b[3][fin], rtol=1e-6)
        if mode == "finger":
            assert b[2][:, 3].sum() > 0


def test_thread_count_does_not_change_results(small):
    data, qs, G, entry = small
    tab = build(data, G, 8, n_samples=2000)
    a = csearch.search_batch(data, G, qs, entry, 32, 10, mode="finger", tables=tab, threads=1)
    b = csearch.search_batch(data, G, qs, entry, 32, 10, mode="finger", tables=tab, threads=7)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


def test_k_above_ef_and_padding():
    """ef_eff = max(ef, K); a graph with fewer reachable nodes than K pads
    with -1 / +inf."""
    data = np.arange(5, dtype=np.float64)[:, None]
    G = np.array([[1, -1], [0, 2], [1, -1], [4, -1], [3, -1]], dtype=np.int32)
    ids, d2, cnt, _ = csearch.search_batch(data, G, np.array([[0.4]]), 0, 1, 4)
    assert ids[0].tolist() == [0, 1, 2, -1]
    np.testing.assert_allclose(d2[0, :3], [0.16, 0.36, 2.56])
    assert np.isinf(d2[0, 3])
    assert cnt[0].tolist() == [3, 3, 0, 0, 3, 0]


def test_invalid_entry_is_an_error(small):
    data, qs, G, _ = small
    with pytest.raises(RuntimeError):
        csearch.search_batch(data, G, qs[:2], data.shape[0], 24, 10)


def test_agrees_on_the_timed_configuration():
    """The CPU baseline's configuration at reduced n: integer 128-d points,
    per-query nearest-pivot entries, r = 64, FINGER at ef = 56."""
    from oracle.search import pivot_entries
    from tests import helpers
    data, qs, G, _, piv = helpers.c2_small()
    X, Q = data.astype(np.float64), qs.astype(np.float64)
    tab = build(X, G, 64, n_samples=100_000, seed=0)
    ent = pivot_entries(Q, X, piv)
    a = search_batch(X, G, Q, ent, 56, 10, mode="finger", tables=tab)
    b = csearch.search_batch(X, G, Q, ent, 56, 10, mode="finger", tables=tab, threads=4)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])    # integer data: exact squared distances
    np.testing.assert_array_equal(a[2], b[2])
    assert b[2][:, 3].sum() > 0


def test_neighbour_id_out_of_range_is_an_error():
    data = np.arange(3, dtype=np.float64)[:, None]
    G = np.array([[1], [7], [1]], dtype=np.int32)
    with pytest.raises(RuntimeError):
        csearch.search_batch(data, G, np.array([[0.0]]), 0, 4, 2)


def _finger_traces():
    with open(os.path.join(GOLD, "finger_traces.json")) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _finger_traces(), ids=lambda c: c["name"])
@pytest.mark.parametrize("which", ["numpy", "compiled"])
def test_hand_traced_finger_search(case, which):
    data = np.array(case["points"], dtype=np.float64)
    G = np.array(case["graph"], dtype=np.int32)
    q = np.array([case["query"]], dtype=np.float64)
    tab = identity_dm({"P": np.eye(data.shape[1])})
    if "dm" in case:
        tab.update(zip(("mu", "sigma", "mu_hat", "sigma_hat", "eps"), map(float, case["dm"])))
    run = search_batch if which == "numpy" else csearch.search_batch
    ids, d2, cnt, _ = run(data, G, q, case["entry"], case["ef"], case["k"], mode="finger",
                          tables=tab, warmup=case["warmup"])
    assert ids[0].tolist() == case["expect_ids"]
    np.testing.assert_allclose(d2[0], case["expect_d2"], rtol=1e-12, atol=1e-12)
    for kname, v in case["expect_counters"].items():
        assert cnt[0, COUNTERS.index(kname)] == v, kname
