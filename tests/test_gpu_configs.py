"""Parity on the shapes of the precision and batching workloads, at reduced n
(the same points per cluster, dimension, rank, code format and K/ef mix as
the full configurations):

* 960-d clustered points, r = 64, BF16 and FP8 edge codes (L2), with
  isotropic noise and with the GIST-calibrated decaying spectrum (where
  FINGER skips about three quarters of the neighbours it screens);
* 100-d heavy-tailed points under the angular metric, r = 64, BF16 and FP8;
* 96-d clustered points, r = 32, FP8 codes, one persistent launch over
  queries with K drawn from {1, 10, 100} and ef from {32, 64, 128, 256, 512}.

Quantized codes depend on the basis itself, not only on its row space: on
these workloads the eigenvalues around the rank cut-off are nearly equal,
so two correct eigensolvers return bases that differ by a rotation inside
the subspace, and codes rounded from them differ.  The search parity tests
therefore hand the oracle's float64 basis to the library build (the basis
option of the build parameters); both sides then quantize the same u_d and
a difference can only come from float32 versus float64 arithmetic before
rounding.  Queries whose smallest screening margin exceeds 1e-4 must return
identical ids and counters.  The estimate error of each code format against
float64 codes, with the library's own basis, is printed."""
import sys

import numpy as np
import pytest

from oracle.build import build as oracle_build
from oracle.codes import quantize_codes
from oracle.estimate import estimate as oracle_estimate
from oracle.knn import normalize_rows, sqdist
from oracle.search import pivot_entries, search_batch
from workloads import SPECS, build_graph, make_points, pick_pivots

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


_CACHE = {}


def _workload(name):
    """(raw data, raw queries, search-space data, search-space queries, graph, pivots)."""
    if name in _CACHE:
        return _CACHE[name]
    if name in ("c3a", "c3s"):
        spec = SPECS[name].scaled(n=20_000, n_centers=20, nq=48)
        npiv = 80
    elif name == "c3b":
        spec = SPECS["c3b"].scaled(n=24_000, n_centers=20, nq=48)
        npiv = 96
    else:
        spec = SPECS["c4"].scaled(n=100_000, n_centers=100, nq=160)
        npiv = 400
    data, qs = make_points(spec)
    if name == "c3b":
        # the angular workload: the library normalizes both sides itself
        rng = np.random.default_rng(3)
        data = (data * rng.uniform(0.5, 4.0, (data.shape[0], 1))).astype(np.float32)
        qs = (qs * rng.uniform(0.5, 4.0, (qs.shape[0], 1))).astype(np.float32)
        sd = normalize_rows(data)
        sq = normalize_rows(qs)
    else:
        sd, sq = data.astype(np.float64), qs.astype(np.float64)
    G, _, _ = build_graph(sd.astype(np.float32), knn_k=16, max_degree=32, device="cuda")
    piv = pick_pivots(spec.n, npiv, spec.seed)
    _CACHE[name] = (data, qs, sd, sq, G, piv)
    return _CACHE[name]


def _code_rows(sd, G, P, c, code):
    """Decoded stored codes of node c's slots in the oracle's basis."""
    cv = sd[c]
    rows = []
    for d in G[c]:
        if d < 0:
            rows.append(np.zeros(P.shape[0]))
            continue
        res = sd[d] - (cv @ sd[d]) / (cv @ cv) * cv
        u = P @ res
        nu = np.linalg.norm(u)
        rows.append(u / nu if nu > 0 else u)
    return quantize_codes(np.array(rows), code)


def _quantized_estimator(sd, G, orc, code):
    cache = {}

    def est(q, cur, nbrs, ub2):
        if cur not in cache:
            cache[cur] = _code_rows(sd, G, orc["P"], cur, code)
        slot = {int(v): i for i, v in enumerate(G[cur])}
        codes = cache[cur][[slot[int(v)] for v in nbrs]]
        return oracle_estimate(q, sd[cur], sd[nbrs], orc, codes=codes)
    return est


def _compare(ids, ctr, oi, oc, margin, label, thr=1e-4):
    safe = margin > thr
    same = (ids == oi).all(1)
    _say(f"{label}: {safe.mean():.3f} of queries with margin > {thr:g}, identical on "
         f"{same[safe].mean() if safe.any() else float('nan'):.4f} of them, {same.mean():.4f} overall")
    assert safe.mean() > 0.5
    assert same[safe].all()
    np.testing.assert_array_equal(ctr[safe][:, :6], oc[safe])


@pytest.mark.parametrize("name", ["c3a", "c3s", "c3b"])
def test_library_eigensolver_on_wide_and_angular_shapes(api, name):
    """The library's own basis (float64 Gram matrix, host cyclic Jacobi)
    against the oracle's SVD of D_res (Proposition 3.1) at m = 960 and at
    m = 100 under the angular metric: every eigenvalue of D_res D_res^T equals
    the oracle's squared singular value to 1e-9 of the largest, and for every
    leading block whose spectral gap is at least 1e-3 of the largest
    eigenvalue the two orthogonal projectors agree to 1e-6 (within a block
    of nearly equal eigenvalues any rotation of the basis is correct); under
    the angular metric the library works on float32 unit vectors, so the
    bars are 1e-6 and 1e-3 there."""
    from paper_2206_11408_amd import _lib as L
    _say(f"{name}: library eigensolver vs oracle SVD")
    data, qs, sd, sq, G, piv = _workload(name)
    metric = L.ANGULAR if name == "c3b" else L.L2
    r = 64
    orc = oracle_build(sd, G, r, n_samples=100_000, seed=0)
    tab = api.finger_build_tables(_t(data), _t(G), rank=r, metric=metric, seed=0)
    ev = tab.read(L.T_EIGVALS)
    P = tab.read(L.T_P_F64)
    S = orc["singular_values"]
    m = sd.shape[1]
    ev_o = np.zeros(m)
    ev_o[:S.size] = S ** 2
    top = ev_o[0]
    err = np.abs(ev - ev_o).max() / top
    gaps = (ev_o[:r] - ev_o[1:r + 1]) / top
    ks = [k for k in range(1, r + 1) if gaps[k - 1] >= 1e-3]
    worst = 0.0
    for k in ks:
        Pl, Po = P[:k], orc["P"][:k]
        worst = max(worst, np.abs(Pl.T @ Pl - Po.T @ Po).max())
    _say(f"  eigenvalues: max |diff| / max = {err:.2e}; projectors compared at {len(ks)} gap-separated "
         f"ranks (largest {max(ks) if ks else 0}), max entry difference {worst:.2e}")
    # L2: both sides start from the same float32 points; angular: the
    # library's unit vectors are float32 roundings of the oracle's float64
    # ones, a relative perturbation near 1e-7 of the Gram matrix
    ev_tol, proj_tol = (1e-9, 1e-6) if metric == L.L2 else (1e-6, 1e-3)
    assert err < ev_tol
    assert ks, "no gap-separated leading block"
    assert worst < proj_tol
    tab.close()


@pytest.mark.parametrize("name,code", [("c3a", "bf16"), ("c3a", "fp8"), ("c3s", "bf16"), ("c3s", "fp8"),
                                       ("c3b", "bf16"), ("c3b", "fp8")])
def test_precision_workloads_search_parity(api, name, code):
    from paper_2206_11408_amd import _lib as L
    _say(f"{name} {code}: FINGER search with quantized codes vs oracle")
    data, qs, sd, sq, G, piv = _workload(name)
    metric = L.ANGULAR if name == "c3b" else L.L2
    ct = {"bf16": L.CODE_BF16, "fp8": L.CODE_FP8E4M3}[code]
    orc = oracle_build(sd, G, 64, n_samples=100_000, seed=0)
    tab = api.finger_build_tables(_t(data), _t(G), rank=64, code_type=ct, metric=metric,
                                  pivots=piv, seed=0, basis=orc["P"])
    info = tab.info()
    for key in ("mu", "sigma", "mu_hat", "sigma_hat", "eps"):
        assert info[key] == pytest.approx(orc[key], rel=1e-6, abs=1e-9), key
    ef = 48
    ids, dist, ctr = (x.cpu().numpy() for x in api.finger_search(tab, _t(qs), mode=1, k=10, ef=ef,
                                                                  entry=-1))
    # every launch shape and code-request mode gives the same answer, run after run
    for v in (dict(code_prefetch=1), dict(code_prefetch=-1), dict(code_prefetch=1, waves_per_cu=2),
              dict(code_prefetch=1, persistent=1)):
        for _ in range(2):
            got = [x.cpu().numpy() for x in api.finger_search(tab, _t(qs), mode=1, k=10, ef=ef,
                                                               entry=-1, **v)]
            for x, y in zip((ids, dist, ctr), got):
                np.testing.assert_array_equal(x, y, err_msg=str(v))
    ent = pivot_entries(sq, sd, piv)
    oi, od, oc, margin = search_batch(sd, G, sq, ent, ef, 10, mode="finger", tables=orc,
                                      estimator=_quantized_estimator(sd, G, orc, code))
    _compare(ids, ctr, oi, oc, margin, f"{name} {code}")
    # returned distances: float32 squared distances of the (normalized) vectors
    ok = ids >= 0
    d64 = np.stack([sqdist(sq[i], sd[np.where(ok[i], ids[i], 0)]) for i in range(ids.shape[0])])
    np.testing.assert_allclose(dist[ok], d64[ok], rtol=2e-5, atol=1e-6)

    # estimate error of the code format against float64 codes, on sampled
    # edges, with the library's own eigenvector basis
    tab = api.finger_build_tables(_t(data), _t(G), rank=64, code_type=ct, metric=metric,
                                  pivots=piv, seed=0)
    rng = np.random.default_rng(1)
    n_items = 200
    deg = (G >= 0).sum(1)
    qi = rng.integers(0, qs.shape[0], n_items)
    ci = rng.choice(np.nonzero(deg > 0)[0], n_items)
    si = np.array([rng.integers(0, deg[c]) for c in ci])
    est, _ = api.finger_estimate_edges(tab, _t(qs), qi, ci, si)
    est = est.cpu().numpy().astype(np.float64)
    exact = np.array([oracle_estimate(sq[q], sd[c], sd[G[c, s]][None], orc)[0]
                      for q, c, s in zip(qi, ci, si)])
    d2 = np.array([sqdist(sq[q], sd[G[c, s]][None])[0] for q, c, s in zip(qi, ci, si)])
    rel = np.abs(est - exact) / np.maximum(np.abs(exact), d2)
    _say(f"{name} {code}: estimate error vs float64 codes: median {np.median(rel):.2e}, "
         f"p99 {np.quantile(rel, 0.99):.2e}, max {rel.max():.2e}")
    assert rel.max() < (2e-2 if code == "bf16" else 1e-1)


def test_batching_workload_persistent_parity(api):
    from paper_2206_11408_amd import _lib as L
    _say("c4 shape (96-d, r=32 fp8): one persistent launch, K in {1,10,100}, ef in {32..512}")
    data, qs, sd, sq, G, piv = _workload("c4")
    orc = oracle_build(sd, G, 32, n_samples=100_000, seed=0)
    tab = api.finger_build_tables(_t(data), _t(G), rank=32, code_type=L.CODE_FP8E4M3, pivots=piv,
                                  seed=0, basis=orc["P"])
    rng = np.random.default_rng(4)
    nq = qs.shape[0]
    K = rng.choice([1, 10, 100], size=nq).astype(np.int32)
    EF = rng.choice([32, 64, 128, 256, 512], size=nq).astype(np.int32)
    p = api.search_params(mode=1, k=100, k_max=100, ef=32, entry=-1, k_per_query=_t(K),
                          ef_per_query=_t(EF), ef_max=512, persistent=1)
    ids, dist, ctr = (x.cpu().numpy() for x in api.finger_search(tab, _t(qs), p))
    assert (ctr[:, 6] == 0).all()
    for i in range(nq):
        assert (ids[i, K[i]:] == -1).all()
    sub = np.arange(0, nq, 4)
    ent = pivot_entries(sq[sub], sd, piv)
    oi, od, oc, margin = search_batch(sd, G, sq[sub], ent, EF[sub], K[sub], mode="finger",
                                      tables=orc, estimator=_quantized_estimator(sd, G, orc, "fp8"))
    safe = margin > 1e-4
    same = np.array([(ids[i, :K[i]] == oi[j, :K[i]]).all() for j, i in enumerate(sub)])
    _say(f"c4 persistent: {safe.mean():.3f} of sampled queries with margin > 1e-4, identical on "
         f"{same[safe].mean() if safe.any() else float('nan'):.4f} of them, {same.mean():.4f} overall")
    assert safe.mean() > 0.5
    assert same[safe].all()
    np.testing.assert_array_equal(ctr[sub][safe][:, :6], oc[safe])
