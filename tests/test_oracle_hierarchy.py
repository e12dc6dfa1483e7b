"""Pins for the oracle's descent through the upper layers of an HNSW-style
hierarchy (the start point of Algorithm 1 on an HNSW graph), and layout
checks of the seeded hierarchy builder.  CPU only."""
import numpy as np
import pytest

from oracle.knn import dist
from oracle.search import descend, hierarchy_entries
from workloads import build_hierarchy, draw_levels


def _line_case():
    """Ten points on a line at x = 0..9; layer 1 is the path 0-2-4-6-8 and
    node 0 alone reaches layer 2."""
    data = np.arange(10, dtype=np.float64)[:, None]
    levels = np.zeros(10, dtype=np.int32)
    levels[[2, 4, 6, 8]] = 1
    levels[0] = 2
    # rows: node 0 (layers 1, 2), then nodes 2, 4, 6, 8 (layer 1)
    upper = np.array([[2, -1], [-1, -1], [0, 4], [2, 6], [4, 8], [6, -1]], dtype=np.int32)
    return data, levels, upper


def test_hand_worked_path():
    data, levels, upper = _line_case()
    # 0 -> 2 -> 4 -> 6 -> 8, then 8's only neighbour 6 is worse
    node, calls = descend(np.array([7.2]), data, levels, upper)
    assert node == 8
    assert calls == 1 + 1 + 2 + 2 + 2 + 1
    # a query past the last layer-1 node ends there too
    assert descend(np.array([100.0]), data, levels, upper)[0] == 8
    # the top entry itself when nothing in layer 1 is closer
    assert descend(np.array([-3.0]), data, levels, upper) == (0, 2)


def test_ties_go_to_the_smaller_id():
    data, levels, upper = _line_case()
    # at 4, neighbour 6 is as close as 4 itself: the key (1, 6) is not below (1, 4)
    assert descend(np.array([5.0]), data, levels, upper)[0] == 4


def test_flat_hierarchy_returns_node_zero():
    data = np.random.default_rng(0).normal(size=(30, 4))
    levels = np.zeros(30, dtype=np.int32)
    upper = np.zeros((0, 8), dtype=np.int32)
    assert descend(data[7], data, levels, upper) == (0, 1)


@pytest.mark.parametrize("metric", ["l2", "ip"])
def test_complete_layer_reaches_its_nearest_node(metric):
    """Layer 1 a complete graph: one hop from the top entry reaches the
    brute-force nearest of the layer by (d, id); a second round over its
    neighbours finds nothing better."""
    rng = np.random.default_rng(3)
    n, m = 60, 5
    data = rng.integers(-4, 5, size=(n, m)).astype(np.float64)   # ties happen
    S = np.sort(rng.choice(n, 12, replace=False))
    levels = np.zeros(n, dtype=np.int32)
    levels[S] = 1
    levels[S[5]] = 2
    first = np.concatenate([[0], np.cumsum(levels)[:-1]])
    upper = np.full((levels.sum(), len(S) - 1), -1, dtype=np.int32)
    for v in S:
        upper[first[v]] = [u for u in S if u != v]
    for q in rng.integers(-4, 5, size=(20, m)).astype(np.float64):
        d = dist(q, data[S], metric)
        want = min(zip(d.tolist(), S.tolist()))[1]
        node, calls = descend(q, data, levels, upper, metric)
        assert node == want
        assert calls == 1 + (len(S) - 1) * (1 if want == S[5] else 2)


@pytest.fixture(scope="module")
def hier():
    rng = np.random.default_rng(5)
    data = rng.normal(size=(3000, 8)) + rng.integers(0, 6, size=(3000, 1))
    levels = draw_levels(3000, 8, 11)
    upper, top = build_hierarchy(data, levels, M=8)
    return data, levels, upper, top


def test_levels_are_geometric():
    lv = draw_levels(200_000, 16, 1)
    frac = np.array([(lv >= l).mean() for l in (1, 2)])
    # P(level >= l) = M^-l; 200,000 draws put the standard error near 1% and 4%
    np.testing.assert_allclose(frac, [16.0 ** -1, 16.0 ** -2], rtol=0.15)


def test_hierarchy_layout(hier):
    data, levels, upper, top = hier
    assert upper.shape[0] == levels.sum()
    assert levels[top] == levels.max() and top == np.flatnonzero(levels == levels.max())[0]
    first = np.concatenate([[0], np.cumsum(levels)[:-1]])
    for v in np.flatnonzero(levels > 0):
        for layer in range(1, levels[v] + 1):
            row = upper[first[v] + layer - 1]
            nb = row[row >= 0]
            assert (row[nb.size:] == -1).all()
            assert v not in nb
            assert (levels[nb] >= layer).all()
    # every layer is reachable from the top entry through its own rows
    for layer in range(1, levels.max() + 1):
        seen, todo = {top}, [top]
        while todo:
            v = todo.pop()
            for u in upper[first[v] + layer - 1]:
                if u >= 0 and u not in seen:
                    seen.add(int(u))
                    todo.append(int(u))
        assert seen == set(np.flatnonzero(levels >= layer).tolist())


@pytest.mark.parametrize("metric", ["l2", "ip"])
def test_descent_ends_in_a_layer_one_local_minimum(hier, metric):
    data, levels, upper, top = hier
    qs = np.random.default_rng(8).normal(size=(40, 8)) * 2 + 2
    ents, calls = hierarchy_entries(qs, data, levels, upper, metric)
    first = np.concatenate([[0], np.cumsum(levels)[:-1]])
    for q, e, c in zip(qs, ents, calls):
        assert levels[e] >= 1
        key = (float(dist(q, data[e], metric)[()]), int(e))
        row = upper[first[e]]
        nb = row[row >= 0]
        assert all(not (float(dv), int(u)) < key for dv, u in zip(dist(q, data[nb], metric), nb))
        assert c >= 1 + levels.max()
    # the descent beats the top entry itself
    dt = np.array([dist(q, data[top], metric) for q in qs])
    de = np.array([dist(q, data[e], metric) for q, e in zip(qs, ents)])
    assert (de <= dt).all() and (de < dt).mean() > 0.9
