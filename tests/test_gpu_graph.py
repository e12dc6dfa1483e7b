"""On-device construction of the flat proximity graph against the oracle's
float64 construction from the definitions: integer data (every distance
exact, graphs identical), continuous and angular data (rows identical up to
float32 near-ties), the repair's failure case, and the argument checks."""
import sys

import numpy as np
import pytest

from oracle import graph as og
from oracle.knn import normalize_rows
from tests import helpers
from workloads import SPECS, make_points, medoid

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


def _compare(G, st, O, ost, label, exact):
    same = (G == O).all(1)
    _say(f"{label}: identical rows {same.mean():.5f}; library {st}; oracle {ost}")
    if exact:
        np.testing.assert_array_equal(G, O)
        assert st["sym_edges"] == ost["sym_edges"]
        assert st["sym_degree_max"] == ost["sym_degree_max"]
        assert st["components_before_repair"] == ost["components_before_repair"]
        assert st["edges_added"] == ost["edges_added"]
    else:
        assert same.mean() >= 0.99
        assert st["components_before_repair"] == ost["components_before_repair"]


@pytest.mark.parametrize("k,W", [(16, 32), (10, 12)])
def test_integer_data_matches_oracle_exactly(api, k, W):
    spec = SPECS["c2"].scaled(n=6000, n_centers=6, nq=1)
    data, _ = make_points(spec)
    e = medoid(data)
    G, st = api.finger_build_graph(_t(data), knn_k=k, max_degree=W, entry=e)
    O, ost = og.build(data, k, W, e)
    _compare(G.cpu().numpy(), st, O, ost, f"integer 6000 x 128, k={k} W={W}", exact=True)


def test_continuous_data_matches_oracle(api):
    data, _, _, entry, _ = helpers.c1(nq=10)
    G, st = api.finger_build_graph(_t(data), knn_k=16, max_degree=32, entry=entry)
    O, ost = og.build(data, 16, 32, entry)
    _compare(G.cpu().numpy(), st, O, ost, "continuous 10000 x 32", exact=False)


def test_angular_graph_is_the_graph_of_unit_vectors(api):
    from paper_2206_11408_amd import _lib as L
    rng = np.random.default_rng(4)
    data = (rng.normal(size=(3000, 20)) + 3 * rng.integers(0, 4, size=(3000, 1))).astype(np.float32)
    data *= rng.uniform(0.5, 3.0, size=(3000, 1)).astype(np.float32)
    G, st = api.finger_build_graph(_t(data), knn_k=12, max_degree=16, entry=0, metric=L.ANGULAR)
    O, ost = og.build(normalize_rows(data), 12, 16, 0)
    _compare(G.cpu().numpy(), st, O, ost, "angular 3000 x 20", exact=False)


def test_repair_without_free_slots_fails(api):
    from paper_2206_11408_amd import _lib as L
    # two far triangles, 2-NN rows already full at degree 2: nothing can link them
    x = np.array([0.0, 1.0, 2.0, 100.0, 101.0, 103.0], np.float32)
    data = np.zeros((6, 4), np.float32)
    data[:, 0] = x
    with pytest.raises(L.FingerError, match="no reached node has a free slot"):
        api.finger_build_graph(_t(data), knn_k=2, max_degree=2, entry=0)
    # with a free slot the repair links them
    G, st = api.finger_build_graph(_t(data), knn_k=2, max_degree=3, entry=0)
    O, ost = og.build(data, 2, 3, 0)
    _compare(G.cpu().numpy(), st, O, ost, "two triangles", exact=True)


def test_argument_errors(api):
    from paper_2206_11408_amd import _lib as L
    data = _t(np.zeros((10, 8), np.float32))
    for kw in (dict(knn_k=10), dict(max_degree=0), dict(entry=10), dict(metric=L.IP)):
        args = dict(knn_k=3, max_degree=4, entry=0) | kw
        with pytest.raises(L.FingerError):
            api.finger_build_graph(data, **args)


def test_exact_duplicates_match_oracle(api):
    """Every point three times: distance-0 ties decide the kNN (the point
    itself excluded, its copies kept, ordered by id), the symmetrized rows
    and the heuristic's strict comparison (a candidate at distance 0 from a
    kept copy is dropped)."""
    rng = np.random.default_rng(9)
    base = rng.integers(0, 16, size=(400, 8)).astype(np.float32)
    data = np.ascontiguousarray(np.repeat(base, 3, axis=0)[rng.permutation(1200)])
    G, st = api.finger_build_graph(_t(data), knn_k=6, max_degree=8, entry=0)
    O, ost = og.build(data, 6, 8, 0)
    _compare(G.cpu().numpy(), st, O, ost, "exact duplicates 1200 x 8", exact=True)


def test_grouped_build_equals_full_build_on_separated_clusters():
    """finger_build_graph_grouped with the mixture's components as groups
    (points sorted by component) returns the graph of the full exact build
    when every point's nearest neighbours lie in its own component: the
    96-d, sigma 0.5 mixture of the batching workload at 100,000 points."""
    import torch
    from paper_2206_11408_amd import api
    from workloads import SPECS, make_points
    print("grouped graph build vs full build (96-d mixture, 100k points)", flush=True)
    spec = SPECS["c4"].scaled(n=100_000, n_centers=100, nq=1)
    data, _, lab = make_points(spec, labels=True)
    order = np.argsort(lab, kind="stable")
    data = np.ascontiguousarray(data[order])
    offs = np.concatenate([[0], np.cumsum(np.bincount(lab, minlength=spec.n_centers))])
    d = torch.as_tensor(data, device="cuda")
    Gf, sf = api.finger_build_graph(d, knn_k=16, max_degree=32, entry=0)
    Gg, sg = api.finger_build_graph_grouped(d, offs, knn_k=16, max_degree=32, entry=0)
    np.testing.assert_array_equal(Gf.cpu().numpy(), Gg.cpu().numpy())
    for key in ("sym_edges", "sym_degree_max", "components_before_repair", "edges_added"):
        assert sf[key] == sg[key], key
    print(f"identical graphs; {sg['components_before_repair']} components, knn {sg['ms_knn']:.1f} ms "
          f"grouped vs {sf['ms_knn']:.1f} ms full", flush=True)
    # a group smaller than knn_k + 1 is refused
    from paper_2206_11408_amd import _lib as L
    with pytest.raises(L.FingerError):
        api.finger_build_graph_grouped(d, [0, 10, spec.n], knn_k=16, max_degree=32, entry=0)
