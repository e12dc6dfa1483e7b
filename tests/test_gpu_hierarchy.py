"""Start points from the upper layers of an HNSW-style hierarchy, on the
library against the oracle: the descent's entries and evaluation counts,
searches started from them (plain bit-exact, FINGER margin-aware), and the
argument checks of the attach call."""
import sys

import numpy as np
import pytest

from oracle.build import build as oracle_build
from oracle.knn import normalize_rows
from oracle.search import hierarchy_entries, search_batch
from tests import helpers
from workloads import build_hierarchy, draw_levels

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


_H = {}


def _hier(name, M=16):
    if name not in _H:
        if name == "c1":
            data, qs, G, entry, _ = helpers.c1(nq=400)
        else:
            data, qs, G, entry, _ = helpers.c2_small()
        levels = draw_levels(data.shape[0], M, 3)
        upper, top = build_hierarchy(data, levels, M=M)
        _H[name] = (data, qs, G, levels, upper, top)
    return _H[name]


@pytest.mark.parametrize("name,metric", [("c2", "l2"), ("c2", "ip"), ("c1", "l2"), ("c1", "angular")])
def test_descent_matches_oracle(api, name, metric):
    from paper_2206_11408_amd import _lib as L
    data, qs, G, levels, upper, top = _hier(name)
    code = {"l2": L.L2, "ip": L.IP, "angular": L.ANGULAR}[metric]
    tab = api.finger_build_tables(_t(data), _t(G), rank=0, metric=code)
    api.finger_hierarchy_attach(tab, levels, upper)
    inf = tab.info()
    assert inf["hierarchy_top"] == top and inf["hierarchy_top_level"] == levels.max()
    assert inf["hierarchy_rows"] == upper.shape[0]
    ent, calls = (x.cpu().numpy() for x in api.finger_descend(tab, _t(qs)))
    if metric == "angular":
        sd, sq, om = normalize_rows(data), normalize_rows(qs), "l2"
    else:
        sd, sq, om = data.astype(np.float64), qs.astype(np.float64), metric
    oe, oc = hierarchy_entries(sq, sd, levels, upper, om)
    same = (ent == oe) & (calls == oc)
    _say(f"descent {name} {metric}: top level {levels.max()}, {upper.shape[0]} upper rows; "
         f"identical entry and count on {same.mean():.4f} of {len(qs)} queries; "
         f"mean evaluations {calls.mean():.1f}")
    if name == "c2":
        assert same.all()          # integer data: every distance is exact in float32
    else:
        assert same.mean() >= 0.99


@pytest.mark.parametrize("mode", ["plain", "finger"])
def test_search_from_descent_matches_oracle(api, mode):
    from paper_2206_11408_amd import _lib as L
    data, qs, G, levels, upper, top = _hier("c2")
    r = 0 if mode == "plain" else 32
    tab = api.finger_build_tables(_t(data), _t(G), rank=r, seed=0)
    api.finger_hierarchy_attach(tab, levels, upper)
    ef = 32
    ids, dist, ctr = (x.cpu().numpy() for x in api.finger_search(
        tab, _t(qs), mode=0 if mode == "plain" else 1, k=10, ef=ef, entry=L.ENTRY_DESCENT))
    oe, _ = hierarchy_entries(qs.astype(np.float64), data.astype(np.float64), levels, upper)
    if mode == "plain":
        oi, od, oc, _ = search_batch(data, G, qs, oe, ef, 10)
        np.testing.assert_array_equal(ids, oi)
        np.testing.assert_array_equal(dist.astype(np.float64), od)
        np.testing.assert_array_equal(ctr[:, :6], oc)
        _say("plain search from descent entries: bit-exact on every query")
        return
    orc = oracle_build(data, G, r, n_samples=100_000, seed=0)
    oi, od, oc, margin = search_batch(data, G, qs, oe, ef, 10, mode="finger", tables=orc)
    safe = margin > 1e-4
    same = (ids == oi).all(1)
    _say(f"FINGER search from descent entries: {safe.mean():.3f} of queries with margin > 1e-4, "
         f"identical on {same[safe].mean() if safe.any() else float('nan'):.4f} of them, "
         f"{same.mean():.4f} overall")
    assert safe.mean() > 0.5
    assert same[safe].all()
    np.testing.assert_array_equal(ctr[safe][:, :6], oc[safe])


def test_flat_hierarchy_starts_at_node_zero(api):
    data, qs, G, _, _ = helpers.c1(nq=20)
    tab = api.finger_build_tables(_t(data), _t(G), rank=0)
    api.finger_hierarchy_attach(tab, np.zeros(data.shape[0], np.int32), np.zeros((0, 16), np.int32))
    ent, calls = (x.cpu().numpy() for x in api.finger_descend(tab, _t(qs)))
    assert (ent == 0).all() and (calls == 1).all()


def test_attach_and_entry_errors(api):
    from paper_2206_11408_amd import _lib as L
    data, qs, G, levels, upper, top = _hier("c2")
    tab = api.finger_build_tables(_t(data), _t(G), rank=0)
    with pytest.raises(L.FingerError, match="upper layers"):
        api.finger_search(tab, _t(qs[:4]), mode=0, k=10, ef=32, entry=L.ENTRY_DESCENT)
    with pytest.raises(L.FingerError, match="no upper layers"):
        api.finger_descend(tab, _t(qs[:4]))
    with pytest.raises(L.FingerError, match="sum to"):
        api.finger_hierarchy_attach(tab, levels, upper[:-1])
    bad = upper.copy()
    v = int(np.flatnonzero(levels == 1)[0])
    first = int(levels[:v].sum())
    bad[first, 0] = v                         # the node itself
    with pytest.raises(L.FingerError, match="not in the layer"):
        api.finger_hierarchy_attach(tab, levels, bad)
    bad = upper.copy()
    bad[first, 0] = int(np.flatnonzero(levels == 0)[0])   # a node below layer 1
    with pytest.raises(L.FingerError, match="not in the layer"):
        api.finger_hierarchy_attach(tab, levels, bad)
    lv = levels.copy()
    lv[0] = 65
    with pytest.raises(L.FingerError, match="out of range"):
        api.finger_hierarchy_attach(tab, lv, upper)
    # a failed attach leaves the handle without layers; a good one then works
    api.finger_hierarchy_attach(tab, levels, upper)
    ent, _ = api.finger_descend(tab, _t(qs[:4]))
    assert (ent.cpu().numpy() >= 0).all()


def test_angular_search_from_descent_matches_oracle(api):
    """Angular tables: the library normalizes the queries before the descent
    and the search; the oracle runs both on the unit vectors."""
    from paper_2206_11408_amd import _lib as L
    data, qs, G, levels, upper, top = _hier("c1")
    tab = api.finger_build_tables(_t(data), _t(G), rank=0, metric=L.ANGULAR)
    api.finger_hierarchy_attach(tab, levels, upper)
    ids, dist, ctr = (x.cpu().numpy() for x in api.finger_search(tab, _t(qs), mode=0, k=10, ef=32,
                                                                  entry=L.ENTRY_DESCENT))
    sd, sq = normalize_rows(data), normalize_rows(qs)
    oe, _ = hierarchy_entries(sq, sd, levels, upper)
    oi, od, oc, _ = search_batch(sd, G, sq, oe, 32, 10)
    same = (ids == oi).all(1)
    _say(f"angular plain search from descent entries: identical on {same.mean():.4f}")
    assert same.mean() >= 0.99
    np.testing.assert_array_equal(ctr[same][:, :6], oc[same])


def test_persistent_mixed_batch_from_descent(api):
    """One persistent launch, per-query K and ef, descent entries: equal to
    per-group launches and to the oracle on integer data."""
    import torch
    from paper_2206_11408_amd import _lib as L
    data, qs, G, levels, upper, top = _hier("c2")
    tab = api.finger_build_tables(_t(data), _t(G), rank=32, seed=0)
    api.finger_hierarchy_attach(tab, levels, upper)
    rng = np.random.default_rng(6)
    nq = qs.shape[0]
    K = rng.choice([1, 10, 20], size=nq).astype(np.int32)
    EF = rng.choice([16, 32, 64], size=nq).astype(np.int32)
    p = api.search_params(mode=0, k=20, k_max=20, ef=16, entry=L.ENTRY_DESCENT,
                          k_per_query=torch.as_tensor(K, device="cuda"),
                          ef_per_query=torch.as_tensor(EF, device="cuda"), ef_max=64, persistent=1)
    ids, dist, ctr = (x.cpu().numpy() for x in api.finger_search(tab, _t(qs), p))
    oe, _ = hierarchy_entries(qs.astype(np.float64), data.astype(np.float64), levels, upper)
    oi, od, oc, _ = search_batch(data, G, qs, oe, EF, K)
    for i in range(nq):
        np.testing.assert_array_equal(ids[i, :K[i]], oi[i, :K[i]])
        assert (ids[i, K[i]:] == -1).all()
    np.testing.assert_array_equal(ctr[:, :6], oc)
    _say("persistent mixed batch from descent entries: bit-exact on every query")
