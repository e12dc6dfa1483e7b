"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs."""
import sys

import numpy as np
import pytest

from oracle.build import build as oracle_build
from oracle.estimate import estimate as oracle_estimate
from oracle.knn import brute_force_knn, sqdist
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


def test_exact_knn_c1(api):
    _say("exact_knn c1 n=10000 m=32 nq=300 k=10")
    data, qs, _, _, _ = helpers.c1()
    qs = qs[:300]
    ids, dist = api.finger_exact_knn(_t(data), _t(qs), 10)
    ids, dist = ids.cpu().numpy(), dist.cpu().numpy()
    gi, gd = brute_force_knn(data, qs, 10)
    same = (ids == gi).all(1)
    assert same.mean() >= 0.999
    np.testing.assert_allclose(dist, gd, rtol=1e-5, atol=1e-6)


def test_exact_knn_integer_bit_exact(api):
    _say("exact_knn c2-small n=20000 m=128 nq=200 k=10")
    data, qs, _, _, _ = helpers.c2_small()
    ids, dist = api.finger_exact_knn(_t(data), _t(qs), 10)
    gi, gd = brute_force_knn(data, qs, 10)
    np.testing.assert_array_equal(ids.cpu().numpy(), gi)
    np.testing.assert_array_equal(dist.cpu().numpy().astype(np.float64), gd)


def test_exact_knn_ragged_and_k_gt_n(api):
    _say("exact_knn ragged n=77 nq=5 k=64")
    rng = np.random.default_rng(5)
    data = rng.normal(size=(77, 12)).astype(np.float32)
    qs = rng.normal(size=(5, 12)).astype(np.float32)
    ids, dist = api.finger_exact_knn(_t(data), _t(qs), 64)
    gi, gd = brute_force_knn(data, qs, 64)
    assert (ids.cpu().numpy() == gi).mean() > 0.99
    np.testing.assert_allclose(dist.cpu().numpy(), gd, rtol=1e-5, atol=1e-5)


@pytest.mark.parametrize("ef", [16, 64])
def test_plain_search_parity_c1(api, ef):
    _say(f"plain search c1 ef={ef} nq=1000")
    data, qs, G, entry, _ = helpers.c1()
    tab = api.finger_build_tables(_t(data), _t(G), rank=0)
    ids, dist, ctr = api.finger_search(tab, _t(qs), mode=0, k=10, ef=ef, entry=entry)
    ids, dist, ctr = ids.cpu().numpy(), dist.cpu().numpy(), ctr.cpu().numpy()
    oi, od, oc, _ = search_batch(data, G, qs, entry, ef, 10)
    same = (ids == oi).all(1)
    _say(f"identical ids on {same.mean():.4f} of queries")
    assert same.mean() >= 0.999
    np.testing.assert_allclose(dist[same], od[same], rtol=1e-5, atol=1e-6)
    # on queries that took the same path the counters agree exactly
    np.testing.assert_array_equal(ctr[same][:, :6], oc[same])
    assert (ctr[:, 6] == 0).all()


def test_plain_search_parity_integer_pivots(api):
    _say("plain search c2-small pivots ef=32")
    data, qs, G, _, piv = helpers.c2_small()
    tab = api.finger_build_tables(_t(data), _t(G), rank=0, pivots=piv)
    ids, dist, ctr = api.finger_search(tab, _t(qs), mode=0, k=10, ef=32, entry=-1)
    ent = pivot_entries(qs, data, piv)
    oi, od, oc, _ = search_batch(data, G, qs, ent, 32, 10)
    np.testing.assert_array_equal(ids.cpu().numpy(), oi)
    np.testing.assert_array_equal(dist.cpu().numpy().astype(np.float64), od)
    np.testing.assert_array_equal(ctr.cpu().numpy()[:, :6], oc)


def test_build_refuses_malformed_graph_rows(api):
    """The build refuses a graph row with a repeated id, a self loop, an id
    out of range or a gap before the -1 padding (EINVAL).  The search relies
    on the first: neighbours of one row are distinct, so lanes never insert
    one id into the visited set twice."""
    from paper_2206_11408_amd import _lib as L
    data, qs, G, entry, _ = helpers.c1(nq=10)
    row = int(np.nonzero((G >= 0).sum(1) >= 3)[0][0])

    def repeated(g):
        g[row, 1] = g[row, 0]

    def self_loop(g):
        g[row, 0] = row

    def out_of_range(g):
        g[row, 0] = data.shape[0]

    def gap(g):
        g[row, 0] = -1

    for name, edit in (("repeated id", repeated), ("self loop", self_loop), ("out of range", out_of_range),
                       ("gap", gap)):
        g = G.copy()
        edit(g)
        with pytest.raises(L.FingerError) as e:
            api.finger_build_tables(_t(data), _t(g), rank=0)
        assert e.value.status == L.FINGER_EINVAL, name
        assert "graph" in str(e.value), name
    api.finger_build_tables(_t(data), _t(G), rank=0).close()


def test_tables_against_oracle(api):
    _say("tables c2-small r=16")
    data, qs, G, _, piv = helpers.c2_small()
    r = 16
    tab = api.finger_build_tables(_t(data), _t(G), rank=r, seed=3)
    orc = oracle_build(data, G, r, n_samples=100_000, seed=3)
    from paper_2206_11408_amd import _lib as L
    smp = tab.read(L.T_SAMPLES)
    c, d, dp, _ = orc["samples"]
    np.testing.assert_array_equal(smp, np.stack([c, d, dp], 1))
    P = tab.read(L.T_P_F64)
    np.testing.assert_allclose(P.T @ P, orc["P"].T @ orc["P"], atol=1e-9)
    # canonical signs make the bases equal row by row
    np.testing.assert_allclose(P, orc["P"], atol=1e-8)
    ev = tab.read(L.T_EIGVALS)
    np.testing.assert_allclose(np.sqrt(np.maximum(ev[:r], 0)), orc["singular_values"][:r], rtol=1e-9)
    inf = tab.info()
    for key in ("mu", "sigma", "mu_hat", "sigma_hat", "eps"):
        assert inf[key] == pytest.approx(orc[key], rel=1e-9, abs=1e-12), key
    xy = tab.read(L.T_XY)
    np.testing.assert_allclose(xy[:, 0], orc["X"], atol=1e-12)
    np.testing.assert_allclose(xy[:, 1], orc["Y"], atol=1e-9)
    # node and edge tables against float64 definitions
    cc = tab.read(L.T_NODE_CC)
    np.testing.assert_allclose(cc, (data.astype(np.float64) ** 2).sum(1), rtol=1e-6)
    alpha = tab.read(L.T_EDGE_ALPHA)
    rho = tab.read(L.T_EDGE_RHO)
    codes = tab.read(L.T_EDGE_CODES)
    Pf = orc["P"]
    rng = np.random.default_rng(0)
    for c_ in rng.integers(0, data.shape[0], 50):
        cv = data[c_].astype(np.float64)
        for s in range(G.shape[1]):
            dd = G[c_, s]
            if dd < 0:
                assert alpha[c_, s] == 0 and rho[c_, s] == 0 and not codes[c_, s].any()
                continue
            dv = data[dd].astype(np.float64)
            a = cv @ dv / (cv @ cv)
            res = dv - a * cv
            assert alpha[c_, s] == pytest.approx(a, rel=1e-5)
            assert rho[c_, s] == pytest.approx(np.sqrt(res @ res), rel=1e-4)
            u = Pf @ res
            u /= np.linalg.norm(u)
            # compare through the projector (sign of each basis row is free)
            got = codes[c_, s, :r].astype(np.float64) @ P
            want = u @ Pf
            np.testing.assert_allclose(got, want, atol=2e-4)


def test_estimates_against_direct_form(api):
    _say("estimates c2-small r=16 vs oracle Algorithm 3")
    data, qs, G, _, _ = helpers.c2_small()
    tab = api.finger_build_tables(_t(data), _t(G), rank=16, seed=1)
    orc = oracle_build(data, G, 16, n_samples=100_000, seed=1)
    rng = np.random.default_rng(2)
    n_items = 400
    qi = rng.integers(0, qs.shape[0], n_items)
    ci = rng.integers(0, data.shape[0], n_items)
    deg = (G >= 0).sum(1)
    si = np.array([rng.integers(0, deg[c]) for c in ci])
    est, that = api.finger_estimate_edges(tab, _t(qs), qi, ci, si)
    est = est.cpu().numpy().astype(np.float64)
    want = np.array([oracle_estimate(qs[q], data[c], data[G[c, s]][None], orc)[0]
                     for q, c, s in zip(qi, ci, si)])
    exact = np.array([sqdist(qs[q], data[G[c, s]][None])[0] for q, c, s in zip(qi, ci, si)])
    err = np.abs(est - want) / np.maximum(np.abs(want), exact)
    _say(f"max relative estimate error {err.max():.3e}")
    assert err.max() < 1e-4


def test_fullrank_identity_finger_equals_plain(api):
    _say("full-rank identity-DM FINGER vs plain on c1")
    data, qs, G, entry, _ = helpers.c1(nq=300)
    tabp = api.finger_build_tables(_t(data), _t(G), rank=0)
    tabf = api.finger_build_tables(_t(data), _t(G), rank=32, dm_override=(0, 1, 0, 1, 0))
    a = api.finger_search(tabp, _t(qs), mode=0, k=10, ef=32, entry=entry)
    b = api.finger_search(tabf, _t(qs), mode=1, k=10, ef=32, entry=entry)
    same = (a[0].cpu().numpy() == b[0].cpu().numpy()).all(1)
    _say(f"identical on {same.mean():.4f}")
    assert same.mean() >= 0.99
    assert b[2].cpu().numpy()[:, 3].sum() > 0


def test_warmup_infinite_equals_plain(api):
    _say("FINGER with W=inf vs plain on c1")
    data, qs, G, entry, _ = helpers.c1(nq=300)
    tabf = api.finger_build_tables(_t(data), _t(G), rank=8)
    a = api.finger_search(tabf, _t(qs), mode=0, k=10, ef=32, entry=entry)
    b = api.finger_search(tabf, _t(qs), mode=1, k=10, ef=32, entry=entry, warmup=1 << 30)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x.cpu().numpy(), y.cpu().numpy())


@pytest.mark.parametrize("r,ef", [(16, 32), (64, 24)])
def test_finger_search_parity_margin_aware(api, r, ef):
    _say(f"FINGER search c2-small r={r} ef={ef} margin-aware parity")
    data, qs, G, _, piv = helpers.c2_small()
    tab = api.finger_build_tables(_t(data), _t(G), rank=r, seed=0, pivots=piv)
    orc = oracle_build(data, G, r, n_samples=100_000, seed=0)
    ids, dist, ctr = api.finger_search(tab, _t(qs), mode=1, k=10, ef=ef, entry=-1)
    ids, dist, ctr = ids.cpu().numpy(), dist.cpu().numpy(), ctr.cpu().numpy()
    ent = pivot_entries(qs, data, piv)
    oi, od, oc, margin = search_batch(data, G, qs, ent, ef, 10, mode="finger", tables=orc)
    safe = margin > 1e-4
    same = (ids == oi).all(1)
    _say(f"{safe.mean():.3f} of queries have margin > 1e-4; identical ids on "
         f"{same[safe].mean():.4f} of them, {same.mean():.4f} overall")
    assert safe.mean() > 0.5
    assert same[safe].all()
    np.testing.assert_array_equal(ctr[safe][:, :6], oc[safe])
    # returned distances are exact for the returned ids
    for i in range(0, qs.shape[0], 7):
        ok = ids[i] >= 0
        np.testing.assert_array_equal(dist[i][ok].astype(np.float64),
                                      sqdist(qs[i], data[ids[i][ok]]))
