"""Parity at the full size of the bandwidth workload (n = 1,000,000 integer
points in 128-d from 1,000 clusters, degree-32 graph, 4,096 pivots, r = 64
fp32 codes, 10,000 queries, K = 10), in the launch configuration the
benchmark times (default geometry, nearest-pivot entries, plain at ef = 48 and
FINGER at ef = 64).

Every query is searched on the GPU in one launch.  A seeded sample of queries
is re-searched by the FP64 oracle one by one and compared id by id; the whole
batch is checked by properties that hold at any size (returned distances are
the exact squared distances of the returned ids, sorted by (d2, id); counter
identities; recall against the exact kNN)."""
import sys
import time

import numpy as np
import pytest

from oracle.build import build as oracle_build
from oracle.search import pivot_entries, search_batch
from workloads import SPECS, build_graph, make_points, pick_pivots

pytestmark = pytest.mark.gpu

N_SAMPLE = 24


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def c2_full():
    import torch
    from paper_2206_11408_amd import api
    torch.cuda.init()
    spec = SPECS["c2"]
    _say("c2 full: points")
    data, qs = make_points(spec)
    _say("c2 full: graph (exact 16-NN on the GPU, symmetrize, prune, repair)")
    t0 = time.time()
    G, entry, gst = build_graph(data, knn_k=spec.knn_k, max_degree=spec.max_degree, device="cuda")
    gst["seconds"] = time.time() - t0
    piv = pick_pivots(spec.n, 4096, spec.seed)
    d_data = torch.as_tensor(data, device="cuda")
    d_G = torch.as_tensor(G, device="cuda")
    d_q = torch.as_tensor(qs, device="cuda")
    _say("c2 full: tables r=64 fp32")
    tab = api.finger_build_tables(d_data, d_G, rank=64, pivots=piv, seed=0)
    gt_ids, gt_d = api.finger_exact_knn(d_data, d_q, 10)
    sample = np.sort(np.random.default_rng(11).choice(spec.nq, N_SAMPLE, replace=False))
    return dict(api=api, data=data, qs=qs, G=G, entry=entry, gstats=gst, piv=piv, tab=tab, d_q=d_q,
                d_data=d_data,
                gt_ids=gt_ids.cpu().numpy(), gt_d=gt_d.cpu().numpy(), sample=sample)


def _properties(w, ids, dist, ctr, mode):
    import torch
    # returned distances are the exact squared distances of the returned ids
    ok = ids >= 0
    assert ok.all()
    x = w["d_data"][torch.as_tensor(ids.reshape(-1), device="cuda").long()].double()
    q = w["d_q"].double().repeat_interleave(ids.shape[1], 0)
    d64 = ((x - q) ** 2).sum(1).cpu().numpy().reshape(ids.shape)
    np.testing.assert_array_equal(dist.astype(np.float64), d64)   # integers: exact in fp32
    key_sorted = (np.diff(dist, axis=1) > 0) | ((np.diff(dist, axis=1) == 0) & (np.diff(ids, axis=1) > 0))
    assert key_sorted.all()
    assert (ctr[:, 6] == 0).all()          # no capacity overflow
    if mode == 1:
        np.testing.assert_array_equal(ctr[:, 1], ctr[:, 4] - ctr[:, 3])
        assert (ctr[:, 3] <= ctr[:, 2]).all()
    else:
        np.testing.assert_array_equal(ctr[:, 1], ctr[:, 4])
    kth = w["gt_d"][:, 9:10]
    hit = (ids[:, :, None] == w["gt_ids"][:, None, :]).any(2) | (dist <= kth)
    return float(hit.mean())


def test_fullsize_plain_parity(c2_full):
    w = c2_full
    api = w["api"]
    _say("c2 full: plain ef=48, all 10,000 queries on the GPU")
    ids, dist, ctr = (t.cpu().numpy() for t in api.finger_search(w["tab"], w["d_q"], mode=0, k=10,
                                                                  ef=48, entry=-1))
    rec = _properties(w, ids, dist, ctr, 0)
    _say(f"  recall@10 {rec:.4f}")
    assert rec >= 0.95
    s = w["sample"]
    data64 = w["data"].astype(np.float64)
    qs = w["qs"][s].astype(np.float64)
    ent = pivot_entries(qs, data64, w["piv"])
    _say(f"  oracle on {len(s)} sampled queries")
    oi, od, oc, _ = search_batch(data64, w["G"], qs, ent, 48, 10)
    np.testing.assert_array_equal(ids[s], oi)
    np.testing.assert_array_equal(dist[s].astype(np.float64), od)
    np.testing.assert_array_equal(ctr[s][:, :2], oc[:, :2])
    np.testing.assert_array_equal(ctr[s][:, 4], oc[:, 4])


def test_fullsize_finger_parity(c2_full):
    w = c2_full
    api = w["api"]
    _say("c2 full: FINGER r=64 fp32 ef=64, all 10,000 queries on the GPU")
    ids, dist, ctr = (t.cpu().numpy() for t in api.finger_search(w["tab"], w["d_q"], mode=1, k=10,
                                                                  ef=64, entry=-1))
    rec = _properties(w, ids, dist, ctr, 1)
    _say(f"  recall@10 {rec:.4f}, skipped {ctr[:, 3].mean():.1f} of {ctr[:, 2].mean():.1f} screened")
    assert rec >= 0.95
    s = w["sample"]
    data64 = w["data"].astype(np.float64)
    _say("  oracle tables (100k sampled pairs, FP64)")
    orc = oracle_build(data64, w["G"], 64, n_samples=100_000, seed=0)
    info = w["tab"].info()
    for key in ("mu", "sigma", "mu_hat", "sigma_hat", "eps"):
        assert info[key] == pytest.approx(orc[key], rel=1e-6, abs=1e-9), key
    qs = w["qs"][s].astype(np.float64)
    ent = pivot_entries(qs, data64, w["piv"])
    _say(f"  oracle on {len(s)} sampled queries")
    oi, od, oc, margin = search_batch(data64, w["G"], qs, ent, 64, 10, mode="finger", tables=orc)
    safe = margin > 1e-4
    same = (ids[s] == oi).all(1)
    _say(f"  {safe.mean():.3f} of sampled queries have margin > 1e-4; identical on "
         f"{same[safe].mean():.4f} of them, {same.mean():.4f} overall")
    assert safe.mean() > 0.5
    assert same[safe].all()
    np.testing.assert_array_equal(ctr[s][safe][:, :6], oc[safe])


def test_fullsize_graph_build_matches_the_workload_builder(c2_full):
    """The library's on-device graph construction against the workload
    builder (torch matmuls and a vectorised heuristic, a separate
    implementation of the same recipe) on the 1M-point integer workload,
    where every distance is exact: the graphs must be identical."""
    import torch
    api = c2_full["api"]
    spec = SPECS["c2"]
    torch.cuda.synchronize()
    t0 = time.time()
    G, st = api.finger_build_graph(c2_full["d_data"], knn_k=spec.knn_k, max_degree=spec.max_degree,
                                   entry=c2_full["entry"])
    torch.cuda.synchronize()
    secs = time.time() - t0
    ref = c2_full["gstats"]
    _say(f"graph build 1M x 128: library {secs:.2f} s ({st}); workload builder {ref['seconds']:.1f} s")
    G = G.cpu().numpy()
    same = (G == c2_full["G"]).all(1)
    _say(f"identical rows: {same.mean():.6f}")
    assert st["sym_degree_max"] == ref["sym_degree_max"]
    assert st["components_before_repair"] == ref["components_before_repair"]
    assert st["edges_added"] == ref["edges_added"]
    np.testing.assert_array_equal(G, c2_full["G"])
