"""finger_search_noalloc, the search entry point that allocates nothing (its
scratch is a fixed device array the library holds per GPU), against
finger_search with a caller workspace: identical results on two calls in a
row, the second with fewer queries, in plain and FINGER modes and with the
persistent queue; a request beyond the array is refused with EOVERFLOW
before any device work."""
import ctypes as C
import sys

import numpy as np
import pytest

from tests import helpers

pytestmark = pytest.mark.gpu


def test_noalloc_search_matches_workspace_search():
    import torch
    from paper_2206_11408_amd import _lib as L
    from paper_2206_11408_amd import api
    print("finger_search_noalloc vs finger_search", flush=True)
    sys.stdout.flush()
    lib = L.load()
    data, qs, G, _, piv = helpers.c2_small()
    dq = torch.as_tensor(qs, device="cuda")
    tab = api.finger_build_tables(torch.as_tensor(data, device="cuda"), torch.as_tensor(G, device="cuda"),
                                  rank=64, pivots=piv, seed=0)
    stream = torch.cuda.current_stream().cuda_stream
    for mode, persistent in ((0, 0), (1, 0), (1, 1)):
        for nq in (200, 37):
            p = api.search_params(mode=mode, k=10, ef=48, entry=-1, persistent=persistent)
            ref = [x.cpu().numpy() for x in api.finger_search(tab, dq[:nq], p)]
            ids = torch.full((nq, 10), -7, dtype=torch.int32, device="cuda")
            dist = torch.full((nq, 10), -7.0, dtype=torch.float32, device="cuda")
            ctr = torch.full((nq, L.NCOUNTERS), -7, dtype=torch.int32, device="cuda")
            L.check(lib.finger_search_noalloc(tab.handle, dq.data_ptr(), nq, C.byref(p), ids.data_ptr(),
                                              dist.data_ptr(), ctr.data_ptr(), stream))
            torch.cuda.synchronize()
            for a, b in zip((ids, dist, ctr), ref):
                np.testing.assert_array_equal(a.cpu().numpy(), b)
    assert lib.finger_search_noalloc_capacity() == 64 << 20
    # more scratch than the array holds: refused before any launch
    p = api.search_params(mode=1, k=10, ef=48, entry=-1)
    st = lib.finger_search_noalloc(tab.handle, dq.data_ptr(), 2_000_000, C.byref(p), dq.data_ptr(),
                                   dq.data_ptr(), None, stream)
    assert st == L.FINGER_EOVERFLOW, lib.finger_last_error().decode()
    tab.close()
