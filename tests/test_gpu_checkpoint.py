"""Tables checkpoint round trip, the visited-set overflow error and the
allocation-failure path, on the GPU.  A search on imported tables must return exactly what it returns on
the handle that was exported; an image over other points or another graph,
or with a damaged byte, is refused.  A visited set forced far below what a
query needs must be reported as EOVERFLOW (every kernel still exits
normally: the overflow path only stops inserting)."""
import sys

import numpy as np
import pytest

from tests import helpers

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _t(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), device="cuda")


@pytest.mark.parametrize("code", [0, 2])
def test_export_import_round_trip(code, tmp_path):
    from paper_2206_11408_amd import _lib as L
    from paper_2206_11408_amd import api
    from workloads import gate_weights
    _say(f"tables export/import round trip (code type {code})")
    data, qs, G, _, piv = helpers.c2_small()
    dd, Gd = _t(data), _t(G)
    tab = api.finger_build_tables(dd, Gd, rank=64, pivots=piv, seed=3, code_type=code)
    if code == 0:
        api.finger_gate_attach(tab, gate_weights(2 * 64 + 4, 64, seed=5), 2 * 64 + 4, 64, 0.02)
    path = str(tmp_path / "tables.bin")
    size = api.finger_tables_save(tab, path)
    tab2 = api.finger_tables_load(path, dd, Gd)
    i1, i2 = tab.info(), tab2.info()
    assert i1 == i2
    for which in (L.T_P_F64, L.T_P_F32, L.T_NODE_CC, L.T_NODE_PC, L.T_EDGE_ALPHA, L.T_EDGE_RHO,
                  L.T_EDGE_CODES, L.T_EDGE_SCALE, L.T_SAMPLES, L.T_XY):
        np.testing.assert_array_equal(tab.read(which), tab2.read(which))
    modes = (0, 1, 2) if code == 0 else (0, 1)
    for mode in modes:
        a = [x.cpu().numpy() for x in api.finger_search(tab, _t(qs), mode=mode, k=10, ef=32, entry=-1)]
        b = [x.cpu().numpy() for x in api.finger_search(tab2, _t(qs), mode=mode, k=10, ef=32, entry=-1)]
        for x, y in zip(a, b):
            np.testing.assert_array_equal(x, y)
    _say(f"image {size} bytes; searches identical in modes {modes}")
    img = np.fromfile(path, dtype=np.uint8)
    # another graph (one row permuted) or other points are refused
    G2 = G.copy()
    G2[5, :2] = G2[5, 1::-1]
    with pytest.raises(L.FingerError) as e:
        api.finger_tables_import(img, dd, _t(G2))
    assert e.value.status == L.FINGER_EINVAL and "graph" in str(e.value)
    data2 = data.copy()
    data2[7, 3] += 1
    with pytest.raises(L.FingerError) as e:
        api.finger_tables_import(img, _t(data2), Gd)
    assert e.value.status == L.FINGER_EINVAL and "data" in str(e.value)
    bad = img.copy()
    bad[len(bad) // 2] ^= 0x10
    with pytest.raises(L.FingerError) as e:
        api.finger_tables_import(bad, dd, Gd)
    assert e.value.status == L.FINGER_ECORRUPT
    tab.close()
    tab2.close()


def test_visited_overflow_is_an_error():
    from paper_2206_11408_amd import _lib as L
    from paper_2206_11408_amd import api
    _say("visited-set overflow reported as EOVERFLOW (tiny LDS and spill tables)")
    data, qs, G, entry, _ = helpers.c1()
    tab = api.finger_build_tables(_t(data), _t(G), rank=0)
    # default capacities: no overflow
    ids, _, ctr = api.finger_search(tab, _t(qs[:64]), mode=0, k=10, ef=256, entry=entry)
    assert ((ctr.cpu().numpy()[:, 6] & 1) == 0).all()
    visited = int(ctr.cpu().numpy()[:, 4].max())
    assert visited > 256 + 64
    with pytest.raises(L.FingerError) as e:
        api.finger_search(tab, _t(qs[:64]), mode=0, k=10, ef=256, entry=entry,
                          visited_capacity=256, spill_capacity=64)
    assert e.value.status == L.FINGER_EOVERFLOW
    # asynchronous form: the status bit, checked by the caller
    _, _, ctr = api.finger_search(tab, _t(qs[:64]), mode=0, k=10, ef=256, entry=entry,
                                  visited_capacity=256, spill_capacity=64, check=False)
    st = ctr.cpu().numpy()[:, 6]
    _say(f"{int((st & 1).sum())} of 64 queries report the overflow (largest |V| at full capacity {visited})")
    assert (st & 1).sum() > 0
    # a spill table large enough for every query: exact again
    ids2, _, ctr2 = api.finger_search(tab, _t(qs[:64]), mode=0, k=10, ef=256, entry=entry,
                                      visited_capacity=256, spill_capacity=8192)
    np.testing.assert_array_equal(ids.cpu().numpy(), ids2.cpu().numpy())
    tab.close()


def test_allocation_failure_is_enomem():
    """With FINGER_FAULT_INJECT=alloc every device allocation of the library
    fails: the table build and the graph construction (the calls that
    allocate; searches and the exact kNN take a caller workspace) return
    ENOMEM with a message naming the allocation, and release what they had
    taken (a normal build afterwards succeeds and searches)."""
    import os
    from paper_2206_11408_amd import _lib as L
    from paper_2206_11408_amd import api
    _say("injected allocation failures -> ENOMEM")
    data, qs, G, entry, _ = helpers.c1(nq=20)
    dd, Gd = _t(data), _t(G)
    os.environ["FINGER_FAULT_INJECT"] = "alloc"
    try:
        calls = (("build", lambda: api.finger_build_tables(dd, Gd, rank=8)),
                 ("graph", lambda: api.finger_build_graph(dd, knn_k=8, max_degree=16, entry=entry)))
        for name, call in calls:
            with pytest.raises(L.FingerError) as e:
                call()
            assert e.value.status == L.FINGER_ENOMEM, name
            assert "injected" in str(e.value), name
    finally:
        del os.environ["FINGER_FAULT_INJECT"]
    tab = api.finger_build_tables(dd, Gd, rank=8)
    ids, _, ctr = api.finger_search(tab, _t(qs), mode=1, k=10, ef=32, entry=entry)
    assert (ids.cpu().numpy() >= 0).all()
    tab.close()
