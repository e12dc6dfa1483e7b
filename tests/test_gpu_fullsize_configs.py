"""Parity at the full sizes of the precision and batching workloads:

* 1,000,000 x 960 clustered points, r = 64, BF16 and FP8 edge codes (L2);
* 1,200,000 x 100 heavy-tailed points under the angular metric, r = 64,
  BF16 and FP8 codes;
* 10,000,000 x 96 clustered points, r = 32 FP8 codes, one persistent launch
  over 100,000 queries with K drawn from {1, 10, 100} and ef from
  {32, 64, 128, 256, 512}.

Each builds its graph on the GPU (16-NN, degree 32, repair from the medoid),
the oracle's float64 tables, and library tables on the oracle's basis (as in
the reduced-size tests: quantized codes depend on the basis itself).  Every
query is checked by properties (returned distances are the float32 squared
distances of the returned ids, keys sorted, counter identities, no capacity
overflow); 48 sampled queries are re-searched by the oracle with the same
quantized codes and must match wherever their screening margin exceeds
1e-4 (at least 8 of them must).

Building these takes minutes (the 10M-point graph alone about five), so the
module runs only with FINGER_FULLSIZE_CONFIGS=1."""
import os
import sys
import time

import numpy as np
import pytest

from oracle.build import build as oracle_build
from oracle.knn import normalize_rows
from oracle.search import pivot_entries, search_batch
from tests.test_gpu_configs import _quantized_estimator
from workloads import SPECS, make_points, medoid, pick_pivots

pytestmark = [
    pytest.mark.gpu,
    pytest.mark.skipif(os.environ.get("FINGER_FULLSIZE_CONFIGS") != "1",
                       reason="full-size workloads take minutes to build; set FINGER_FULLSIZE_CONFIGS=1"),
]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _progress(phase, done, total):
    _say(f"    graph {phase}: {done}/{total}")


def _workload(name):
    import torch
    from paper_2206_11408_amd import _lib as L
    from paper_2206_11408_amd import api
    spec = SPECS[name]
    t0 = time.time()
    data, qs = make_points(spec)
    if name == "c3b":
        rng = np.random.default_rng(3)
        data = (data * rng.uniform(0.5, 4.0, (data.shape[0], 1))).astype(np.float32)
        qs = (qs * rng.uniform(0.5, 4.0, (qs.shape[0], 1))).astype(np.float32)
        sd, sq = normalize_rows(data), normalize_rows(qs)
    else:
        sd, sq = data.astype(np.float64), qs.astype(np.float64)
    _say(f"  {name}: {spec.n} x {spec.m} points and {spec.nq} queries in {time.time() - t0:.0f} s")
    d_data = torch.as_tensor(data, device="cuda")
    metric = L.ANGULAR if name == "c3b" else L.L2
    t0 = time.time()
    dG, gst = api.finger_build_graph(d_data, knn_k=16, max_degree=32, entry=medoid(sd),
                                     metric=metric, progress=_progress)
    _say(f"  {name}: graph on the GPU in {time.time() - t0:.0f} s: {gst}")
    piv = pick_pivots(spec.n, 4096, spec.seed)
    return dict(spec=spec, data=data, qs=qs, sd=sd, sq=sq, d_data=d_data, dG=dG,
                G=dG.cpu().numpy(), piv=piv, metric=metric)


def _properties(w, ids, dist, ctr, kq=None):
    import torch
    nq, kmax = ids.shape
    ok = ids >= 0
    if kq is None:
        assert ok.all()
    else:
        assert all(ok[i, :kq[i]].all() and not ok[i, kq[i]:].any() for i in range(nq))
    sd = torch.as_tensor(w["sd"], device="cuda") if w["metric"] == 1 else w["d_data"].double()
    sq = torch.as_tensor(w["sq"], device="cuda")
    x = sd[torch.as_tensor(np.where(ok, ids, 0).reshape(-1), device="cuda").long()].double()
    q = sq.double().repeat_interleave(kmax, 0)
    d64 = ((x - q) ** 2).sum(1).cpu().numpy().reshape(ids.shape)
    np.testing.assert_allclose(dist[ok].astype(np.float64), d64[ok], rtol=2e-5, atol=1e-6)
    with np.errstate(invalid="ignore"):     # inf - inf in the padding, masked below
        dd = np.diff(dist, axis=1)
    di = np.diff(ids, axis=1)
    both = ok[:, 1:]
    assert (((dd > 0) | ((dd == 0) & (di > 0)))[both]).all()
    assert (ctr[:, 6] == 0).all()
    np.testing.assert_array_equal(ctr[:, 1], ctr[:, 4] - ctr[:, 3])
    assert (ctr[:, 3] <= ctr[:, 2]).all()


def _sampled(w, orc, code, ids, ctr, sample, ef, k):
    ent = pivot_entries(w["sq"][sample], w["sd"], w["piv"])
    t0 = time.time()
    oi, od, oc, margin = search_batch(w["sd"], w["G"], w["sq"][sample], ent, ef, k, mode="finger",
                                      tables=orc, estimator=_quantized_estimator(w["sd"], w["G"], orc, code))
    safe = margin > 1e-4
    kk = np.broadcast_to(np.asarray(k), (len(sample),))
    same = np.array([(ids[i, :kk[j]] == oi[j, :kk[j]]).all() for j, i in enumerate(sample)])
    _say(f"    oracle on {len(sample)} sampled queries in {time.time() - t0:.0f} s: {safe.mean():.3f} "
         f"with margin > 1e-4, identical on {same[safe].mean() if safe.any() else float('nan'):.4f} "
         f"of them, {same.mean():.4f} overall")
    # at full size a query makes hundreds of screening decisions, so its
    # smallest margin is smaller than at reduced n; the bar is that every
    # query clearing 1e-4 is identical, and enough of them must clear it for
    # the check to mean something
    assert safe.sum() >= 8
    assert same[safe].all()
    np.testing.assert_array_equal(ctr[sample][safe][:, :6], oc[safe])


@pytest.mark.parametrize("name", ["c3a", "c3b"])
def test_precision_workload_full_size(name):
    import torch
    from paper_2206_11408_amd import _lib as L
    from paper_2206_11408_amd import api
    torch.cuda.init()
    w = _workload(name)
    t0 = time.time()
    orc = oracle_build(w["sd"], w["G"], 64, n_samples=100_000, seed=0)
    _say(f"  {name}: oracle tables in {time.time() - t0:.0f} s")
    d_q = torch.as_tensor(w["qs"], device="cuda")
    sample = np.sort(np.random.default_rng(5).choice(w["spec"].nq, 48, replace=False))
    for code in ("bf16", "fp8"):
        ct = {"bf16": L.CODE_BF16, "fp8": L.CODE_FP8E4M3}[code]
        tab = api.finger_build_tables(w["d_data"], w["dG"], rank=64, code_type=ct, metric=w["metric"],
                                      pivots=w["piv"], seed=0, basis=orc["P"])
        info = tab.info()
        for key in ("mu", "sigma", "mu_hat", "sigma_hat", "eps"):
            assert info[key] == pytest.approx(orc[key], rel=1e-6, abs=1e-9), key
        ids, dist, ctr = (x.cpu().numpy() for x in api.finger_search(tab, d_q, mode=1, k=10, ef=48,
                                                                      entry=-1, persistent=1))
        _say(f"  {name} {code}: all {len(ids)} queries searched; skipped "
             f"{ctr[:, 3].sum() / ctr[:, 2].sum():.3f} of screened")
        _properties(w, ids, dist, ctr)
        _sampled(w, orc, code, ids, ctr, sample, 48, 10)
        tab.close()


def test_batching_workload_full_size():
    import torch
    from paper_2206_11408_amd import _lib as L
    from paper_2206_11408_amd import api
    torch.cuda.init()
    w = _workload("c4")
    t0 = time.time()
    orc = oracle_build(w["sd"], w["G"], 32, n_samples=100_000, seed=0)
    _say(f"  c4: oracle tables in {time.time() - t0:.0f} s")
    tab = api.finger_build_tables(w["d_data"], w["dG"], rank=32, code_type=L.CODE_FP8E4M3,
                                  pivots=w["piv"], seed=0, basis=orc["P"])
    nq = w["spec"].nq
    rng = np.random.default_rng(4)
    K = rng.choice([1, 10, 100], size=nq).astype(np.int32)
    EF = rng.choice([32, 64, 128, 256, 512], size=nq).astype(np.int32)
    p = api.search_params(mode=1, k=100, k_max=100, ef=32, entry=-1,
                          k_per_query=torch.as_tensor(K, device="cuda"),
                          ef_per_query=torch.as_tensor(EF, device="cuda"), ef_max=512, persistent=1)
    d_q = torch.as_tensor(w["qs"], device="cuda")
    t0 = time.time()
    ids, dist, ctr = (x.cpu().numpy() for x in api.finger_search(tab, d_q, p))
    _say(f"  c4: one persistent launch over {nq} queries in {time.time() - t0:.2f} s (incl. copies)")
    _properties(w, ids, dist, ctr, kq=K)
    sample = np.sort(rng.choice(nq, 48, replace=False))
    _sampled(w, orc, "fp8", ids, ctr, sample, EF[sample], K[sample])
    tab.close()
