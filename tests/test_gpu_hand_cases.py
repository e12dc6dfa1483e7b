"""The hand-worked cases of tests/golden/ on the library: Algorithm 2's
residual cosines and distribution-matching statistics (the build's FP64
path), Algorithm 3's estimate with non-trivial matching (the search's
factorized FP32 form, through finger_estimate_edges), and the gate
network's forward and backward kernels on bf16-exact values.  Points are
padded with zero coordinates to m = 4, which changes no residual, cosine
or distance."""
import json
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def _pad4(a):
    a = np.atleast_2d(np.asarray(a, dtype=np.float64))
    out = np.zeros((a.shape[0], 4))
    out[:, :a.shape[1]] = a
    return out


@pytest.mark.parametrize("mode", ["std", "variance"])
def test_algorithm2_hand_case_on_gpu(mode):
    import torch
    from paper_2206_11408_amd import _lib as L
    from paper_2206_11408_amd import api
    case = _load("algorithm2_case.json")
    print(f"Algorithm 2 hand case ({mode}) on the GPU", flush=True)
    sys.stdout.flush()
    data = torch.as_tensor(_pad4(case["points"]), dtype=torch.float32, device="cuda")
    G = torch.as_tensor(np.array(case["graph"], dtype=np.int32), device="cuda")
    tab = api.finger_build_tables(data, G, rank=2, seed=0, basis=_pad4(case["basis"]),
                                  sigma_mode=L.SIGMA_STD if mode == "std" else L.SIGMA_VARIANCE)
    samples = tab.read(L.T_SAMPLES)
    assert samples[:, 0].tolist() == case["centres"]
    xy = tab.read(L.T_XY)
    np.testing.assert_allclose(xy[:, 0], case["X"], rtol=0, atol=1e-12)
    np.testing.assert_allclose(xy[:, 1], case["Y"], rtol=0, atol=1e-7)
    info = tab.info()
    for key, v in case[mode].items():
        assert info[key] == pytest.approx(v, abs=1e-7), key
    assert info["corr_xy"] == pytest.approx(case["corr"], abs=1e-7)
    tab.close()


def test_algorithm3_hand_case_on_gpu():
    import torch
    from paper_2206_11408_amd import api
    case = _load("algorithm3_case.json")
    print("Algorithm 3 hand case on the GPU", flush=True)
    pts = np.vstack([case["centre"], case["neighbours"]]).astype(np.float32)
    G = np.array([[1, 2], [0, 2], [0, 1]], dtype=np.int32)
    dm = case["dm"]
    for identity, want in ((False, case["est"]), (True, case["est_identity_dm"])):
        dmo = (0, 1, 0, 1, 0) if identity else (dm["mu"], dm["sigma"], dm["mu_hat"], dm["sigma_hat"], dm["eps"])
        tab = api.finger_build_tables(torch.as_tensor(pts, device="cuda"), torch.as_tensor(G, device="cuda"),
                                      rank=2, seed=0, basis=np.array(case["basis"], dtype=np.float64),
                                      dm_override=dmo)
        q = torch.as_tensor(np.array([case["query"]], dtype=np.float32), device="cuda")
        est, that = api.finger_estimate_edges(tab, q, [0, 0], [0, 0], [0, 1])
        np.testing.assert_allclose(est.cpu().numpy(), want, rtol=1e-5, atol=1e-5)
        np.testing.assert_allclose(that.cpu().numpy(), case["t_hat"], rtol=1e-6, atol=1e-7)
        tab.close()


def _gate_params(case):
    w = case["weights"]
    return np.concatenate([np.ravel(w["W1"]), w["b1"], np.ravel(w["W2"]), w["b2"], w["W3"],
                           [w["b3"]]]).astype(np.float32)


def test_gate_hand_case_on_gpu():
    import torch
    from paper_2206_11408_amd import api
    case = _load("gate_mlp_case.json")
    print("gate network hand case on the GPU", flush=True)
    ind, H = case["in_dim"], case["hidden"]
    w = torch.as_tensor(_gate_params(case), device="cuda")
    X = torch.as_tensor(np.array([r["x"] for r in case["forward"]], dtype=np.float32), device="cuda")
    y = api.finger_mlp_forward(w, ind, H, X).cpu().numpy()
    assert y.tolist() == [r["y"] for r in case["forward"]]
    b = case["backward"]
    xb = torch.as_tensor(np.array(b["x"], dtype=np.float32), device="cuda")
    tb = torch.as_tensor(np.array(b["target"], dtype=np.float32), device="cuda")
    g, loss = api.finger_mlp_backward(w, ind, H, xb, tb)
    gg = b["grad"]
    want = np.concatenate([np.ravel(gg["W1"]), gg["b1"], np.ravel(gg["W2"]), gg["b2"], gg["W3"],
                           [gg["b3"]]])
    assert g.cpu().numpy().tolist() == want.tolist()
    assert float(loss.item()) == b["loss"]
