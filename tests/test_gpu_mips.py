"""The inner-product metric (maximum inner-product search, Supplementary A)
on the library against the oracle: exact kNN, plain and FINGER search,
and the estimate, on seeded Gaussian-mixture and integer workloads."""
import sys

import numpy as np
import pytest

from oracle.build import build as oracle_build
from oracle.estimate import estimate_ip
from oracle.knn import brute_force_knn
from oracle.search import pivot_entries, search_batch
from tests import helpers

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def api():
    import torch
    from paper_2206_11408_amd import api as A
    torch.cuda.init()
    return A


def _t(x, dtype=None):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def test_exact_knn_ip(api):
    from paper_2206_11408_amd import _lib as L
    data, qs, _, _, _ = helpers.c1(nq=300)
    ids, dist = (x.cpu().numpy() for x in api.finger_exact_knn(_t(data), _t(qs), 10, metric=L.IP))
    bi, bd = brute_force_knn(data, qs, 10, metric="ip")
    same = (ids == bi).all(1)
    _say(f"exact kNN (inner product): identical on {same.mean():.4f} of queries")
    assert same.mean() >= 0.999
    scale = np.abs(qs).sum(1, keepdims=True) * np.abs(data).max()
    err = np.abs(dist.astype(np.float64) - bd)
    np.testing.assert_array_less(err, np.broadcast_to(1e-5 * scale, err.shape))


def test_plain_search_ip(api):
    from paper_2206_11408_amd import _lib as L
    data, qs, G, entry, _ = helpers.c1(nq=300)
    tab = api.finger_build_tables(_t(data), _t(G), rank=0, metric=L.IP)
    ids, dist, ctr = (x.cpu().numpy() for x in api.finger_search(tab, _t(qs), mode=0, k=10, ef=48,
                                                                  entry=entry))
    oi, od, oc, _ = search_batch(data, G, qs, entry, 48, 10, metric="ip")
    same = (ids == oi).all(1)
    _say(f"plain inner-product search: identical ids on {same.mean():.4f} of queries")
    assert same.mean() >= 0.99
    np.testing.assert_array_equal(ctr[same][:, :6], oc[same])
    scale = np.abs(qs).sum(1, keepdims=True) * np.abs(data).max()
    err = np.abs(dist[same].astype(np.float64) - od[same])
    np.testing.assert_array_less(err, np.broadcast_to(1e-5 * scale[same], err.shape))


def test_finger_search_ip_margin_aware(api):
    from paper_2206_11408_amd import _lib as L
    data, qs, G, _, piv = helpers.c2_small()
    tab = api.finger_build_tables(_t(data), _t(G), rank=32, metric=L.IP, pivots=piv, seed=0)
    orc = oracle_build(data, G, 32, n_samples=100_000, seed=0)
    ids, dist, ctr = (x.cpu().numpy() for x in api.finger_search(tab, _t(qs), mode=1, k=10, ef=32,
                                                                  entry=-1))
    ent = pivot_entries(qs, data, piv, metric="ip")
    oi, od, oc, margin = search_batch(data, G, qs, ent, 32, 10, mode="finger", tables=orc,
                                      metric="ip")
    # the margin is relative to |ub| = |q.x| of the worst kept point; on
    # this non-negative integer data |q||x| <= 2 |q.x| for the points near
    # the bound, so the float32 rounding of the estimate's terms stays below
    # ~1e-6 |ub|, and 1e-5 leaves a factor of ten (all inner products here sit
    # within a few percent of each other, so relative gaps are small)
    safe = margin > 1e-5
    same = (ids == oi).all(1)
    _say(f"FINGER inner-product search: {safe.mean():.3f} of queries with margin > 1e-5, identical "
         f"on {same[safe].mean() if safe.any() else float('nan'):.4f} of them, {same.mean():.4f} overall; "
         f"skipped {ctr[:, 3].sum() / max(ctr[:, 2].sum(), 1):.3f} of screened")
    assert safe.mean() > 0.5
    assert same[safe].all()
    np.testing.assert_array_equal(ctr[safe][:, :6], oc[safe])
    # integer data: inner products are exact in float32
    np.testing.assert_array_equal(dist.astype(np.float64),
                                  np.stack([-(data[i] @ q) for i, q in zip(ids, qs)]))


def test_estimate_ip_against_oracle(api):
    from paper_2206_11408_amd import _lib as L
    data, qs, G, _, piv = helpers.c2_small()
    tab = api.finger_build_tables(_t(data), _t(G), rank=32, metric=L.IP, seed=0)
    orc = oracle_build(data, G, 32, n_samples=100_000, seed=0)
    rng = np.random.default_rng(2)
    deg = (G >= 0).sum(1)
    qi = rng.integers(0, qs.shape[0], 200)
    ci = rng.choice(np.nonzero(deg > 0)[0], 200)
    si = np.array([rng.integers(0, deg[c]) for c in ci])
    est, _ = api.finger_estimate_edges(tab, _t(qs), qi, ci, si)
    est = est.cpu().numpy().astype(np.float64)
    want = np.array([estimate_ip(qs[q], data[c], data[G[c, s]][None], orc)[0]
                     for q, c, s in zip(qi, ci, si)])
    dots = np.array([qs[q] @ data[G[c, s]] for q, c, s in zip(qi, ci, si)])
    rel = np.abs(est - want) / np.maximum(np.abs(want), np.abs(dots))
    _say(f"inner-product estimate: max relative error {rel.max():.2e}")
    assert rel.max() < 1e-4


def test_gate_is_refused_for_inner_product(api):
    from paper_2206_11408_amd import _lib as L
    data, qs, G, entry, _ = helpers.c1(nq=20)
    tab = api.finger_build_tables(_t(data), _t(G), rank=8, metric=L.IP)
    with pytest.raises(L.FingerError, match="L2 and angular only"):
        api.finger_search(tab, _t(qs), mode=2, k=10, ef=32, entry=entry)
    with pytest.raises(L.FingerError, match="L2 and angular only"):
        api.finger_gate_attach(tab, np.zeros(api.finger_gate_param_count(20, 8), np.float32), 20, 8,
                               0.0)
