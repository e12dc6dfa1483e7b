"""The hand-traced runs of Algorithm 4 (tests/golden/finger_traces.json) on
the GPU kernel: the points padded with zeros to m = 4, the identity basis
(r = m) and each case's distribution-matching constants (the identity, or
the hand-chosen affine maps of the three-dimensional cases), so every
screening decision and counter must match the hand derivation."""
import json
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")
COUNTERS = ("expansions", "exact", "screened", "skipped", "visited", "preps")


def _cases():
    with open(os.path.join(GOLD, "finger_traces.json")) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c["name"])
def test_hand_traced_finger_search_on_gpu(case):
    import torch
    from paper_2206_11408_amd import api
    torch.cuda.init()
    print(f"hand trace {case['name']} on the GPU", flush=True)
    sys.stdout.flush()
    m = 4
    pts = np.array(case["points"], dtype=np.float32)
    data = np.zeros((pts.shape[0], m), dtype=np.float32)
    data[:, :pts.shape[1]] = pts
    q = np.zeros((1, m), dtype=np.float32)
    q[0, :pts.shape[1]] = case["query"]
    G = np.array(case["graph"], dtype=np.int32)
    assert G.shape[0] == data.shape[0] and G.max() < data.shape[0]
    tab = api.finger_build_tables(torch.as_tensor(data, device="cuda"), torch.as_tensor(G, device="cuda"),
                                  rank=m, seed=0, basis=np.eye(m),
                                  dm_override=tuple(case.get("dm", (0, 1, 0, 1, 0))))
    ids, d2, ctr = (x.cpu().numpy() for x in api.finger_search(
        tab, torch.as_tensor(q, device="cuda"), mode=1, k=case["k"], ef=case["ef"],
        entry=case["entry"], warmup=case["warmup"]))
    assert ids[0].tolist() == case["expect_ids"]
    np.testing.assert_allclose(d2[0], case["expect_d2"], rtol=1e-5, atol=1e-6)
    for kname, v in case["expect_counters"].items():
        assert ctr[0, COUNTERS.index(kname)] == v, kname
    tab.close()
