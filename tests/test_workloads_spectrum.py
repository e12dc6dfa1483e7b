"""The decaying-spectrum variant of the integer workload: the noise mix has
the stated spectrum, and at reduced size the rank rule of Supplementary E
(run by the oracle) settles on r = 16, the rank the paper reports for
SIFT-1M-128.  CPU only."""
import numpy as np

from oracle.build import select_rank
from workloads import SPECS, build_graph, make_points
from workloads.gen import noise_mix


def test_noise_mix_has_the_stated_spectrum():
    spec = SPECS["c2s"]
    A = noise_mix(spec, np.random.default_rng(1))
    np.testing.assert_allclose(A, A.T, atol=1e-12)
    ev = np.sort(np.linalg.eigvalsh(A))[::-1]
    i = np.arange(1, spec.m + 1)
    want = i ** -spec.decay
    want /= np.sqrt((want ** 2).mean())
    np.testing.assert_allclose(ev, want, rtol=1e-10)
    # the same total noise variance as the isotropic workload
    assert abs((A * A).sum() / spec.m - 1.0) < 1e-10


def test_rank_rule_settles_on_sixteen():
    spec = SPECS["c2s"].scaled(n=20_000, n_centers=20, nq=1)
    data, _ = make_points(spec)
    G, _, _ = build_graph(data, knn_k=16, max_degree=32)
    r, tab = select_rank(data.astype(np.float64), G, target=0.7, n_samples=100_000, seed=0)
    assert r == 16, (r, tab["corr"])
