"""Pins for the oracle's flat-graph construction (kNN, symmetrization,
HNSW's neighbour-selection heuristic, reachability repair).  CPU only."""
import numpy as np
import pytest

from oracle import graph as og
from workloads import SPECS, build_graph, make_points, medoid


def test_knn_brute_force_with_ties():
    rng = np.random.default_rng(1)
    X = rng.integers(0, 4, size=(80, 3)).astype(np.float64)    # many equal distances
    ids, d2 = og.knn(X, 7, chunk=16)
    for i in range(80):
        keys = sorted((float(((X[i] - X[j]) ** 2).sum()), j) for j in range(80) if j != i)[:7]
        assert ids[i].tolist() == [j for _, j in keys]
        assert d2[i].tolist() == [d for d, _ in keys]


def test_symmetrize_is_the_union():
    ids = np.array([[1, 2], [0, 2], [0, 1], [0, 1]])
    d2 = np.array([[1.0, 4.0], [1.0, 9.0], [4.0, 9.0], [25.0, 36.0]])
    rows = og.symmetrize(ids, d2)
    assert rows[0] == [(1.0, 1), (4.0, 2), (25.0, 3)]
    assert rows[1] == [(1.0, 0), (9.0, 2), (36.0, 3)]
    assert rows[3] == [(25.0, 0), (36.0, 1)]


def test_heuristic_keeps_one_point_per_direction():
    # base 0 on a line; candidates at 1, 2, 3 and -1, -2
    X = np.array([[0.0], [1.0], [2.0], [3.0], [-1.0], [-2.0]])
    row = sorted((float(X[j, 0] ** 2), j) for j in range(1, 6))
    rows = [row] + [[] for _ in range(5)]
    G = og.prune(X, rows, max_degree=3)
    # 1 kept; -1 kept (closer to 0 than to 1); 2, -2, 3 each closer to a kept point
    assert sorted(G[0][G[0] >= 0].tolist()) == [1, 4]
    assert G[0].tolist()[:2] == [1, 4]


def test_heuristic_keeps_mutually_far_points_up_to_the_cap():
    # orthogonal directions: every pair is farther apart than either is from 0
    m = 8
    X = np.vstack([np.zeros(m), np.diag(1.0 + 0.1 * np.arange(m))])
    rows = [sorted((float((X[j] ** 2).sum()), j) for j in range(1, m + 1))] + [[] for _ in range(m)]
    G = og.prune(X, rows, max_degree=5)
    assert G[0].tolist() == [1, 2, 3, 4, 5]


def test_short_rows_are_kept_whole():
    X = np.random.default_rng(2).normal(size=(5, 2))
    rows = [[(0.1, 3), (0.2, 1)], [], [], [], []]
    G = og.prune(X, rows, max_degree=2)
    assert G[0].tolist() == [3, 1]


def test_repair_links_components_by_the_nearest_free_reached_node():
    # two triangles far apart on a line: {0,1,2} near 0, {3,4,5} near 100
    X = np.array([[0.0], [1.0], [2.0], [100.0], [101.0], [103.0]])
    G = np.array([[1, 2, -1], [0, 2, -1], [0, 1, -1], [4, 5, -1], [3, 5, -1], [3, 4, -1]], np.int32)
    R, comps, added = og.repair(X, G, entry=0)
    # node 3 is the smallest unreached; the nearest reached with a free slot is 2
    assert comps == 2 and added == 2
    assert R[2].tolist() == [0, 1, 3] and R[3].tolist() == [4, 5, 2]
    # a full row cannot take the link: the next nearest reached node with a free slot does
    X2 = np.vstack([X, [[1.5]]])
    G2 = np.array([[1, 2, -1], [0, 2, -1], [0, 1, 6], [4, 5, -1], [3, 5, -1], [3, 4, -1], [2, -1, -1]],
                  np.int32)
    R2, comps2, added2 = og.repair(X2, G2, entry=0)
    assert comps2 == 2 and added2 == 2
    assert R2[6].tolist() == [2, 3, -1] and R2[3].tolist() == [4, 5, 6]
    # no reached node with a free slot: an error, not a silent partial graph
    G3 = np.array([[1, 2], [0, 2], [0, 1], [4, 5], [3, 5], [3, 4]], np.int32)
    with pytest.raises(RuntimeError):
        og.repair(X, G3, entry=0)


@pytest.fixture(scope="module")
def small():
    spec = SPECS["c2"].scaled(n=2000, n_centers=4, nq=1)
    data, _ = make_points(spec)
    return data


def test_matches_the_workload_builder_on_integer_data(small):
    """A second, separately written implementation of the same recipe
    (torch matmuls, vectorised heuristic) builds the same graph."""
    data = small
    e = medoid(data)
    G, st = og.build(data, 16, 32, e)
    W, e2, wst = build_graph(data, knn_k=16, max_degree=32, entry=e)
    np.testing.assert_array_equal(G, W)
    assert st["components_before_repair"] == wst["components_before_repair"]
    assert st["edges_added"] == wst["edges_added"]
    assert st["sym_degree_max"] == wst["sym_degree_max"]


def test_graph_properties(small):
    data = small
    G, st = og.build(data, 12, 16, 0)
    n = G.shape[0]
    # every node reachable from the entry; no self loops; no duplicate ids in a row
    reached = np.zeros(n, bool)
    og._mark_from(G, reached, 0)
    assert reached.all()
    for i in range(n):
        row = G[i][G[i] >= 0]
        assert i not in row and len(set(row.tolist())) == row.size
        assert (G[i][row.size:] == -1).all()
