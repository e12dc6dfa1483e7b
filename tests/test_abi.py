"""C ABI checks that need no GPU: the library loads, exports every entry
point include/finger.h declares, the ctypes structures match the C layout,
and argument errors are reported before any device work."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

from paper_2206_11408_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "finger.h")


def _declared():
    with open(HEADER) as f:
        txt = f.read()
    return sorted(set(re.findall(r"FINGER_API\s+[\w\s\*]+?\b(finger_\w+)\s*\(", txt)))


def test_header_declares_what_binding_lists():
    assert set(_declared()) == set(L.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = L.load()
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (finger_\w+)", out))
    for name in _declared():
        assert name in exported, name
        assert hasattr(lib, name)


def test_struct_layout_matches_header():
    src = r"""
#include <stdio.h>
#include <stddef.h>
#include "finger.h"
#define P(s, f) printf(#s "." #f " %zu\n", offsetof(s, f))
int main(void) {
  printf("build %zu\nsearch %zu\ninfo %zu\n", sizeof(finger_build_params),
         sizeof(finger_search_params), sizeof(finger_tables_info));
  P(finger_build_params, n_samples); P(finger_build_params, pivots); P(finger_build_params, dm);
  P(finger_search_params, k_per_query); P(finger_search_params, ef_max);
  P(finger_search_params, log_features); P(finger_search_params, log_count);
  P(finger_tables_info, n_samples_used); P(finger_tables_info, mu); P(finger_tables_info, gate_attached);
  P(finger_tables_info, edge_table_bytes); P(finger_tables_info, corr_xy);
  P(finger_tables_info, hierarchy_top); P(finger_tables_info, hierarchy_rows);
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "l.c")
        exe = os.path.join(d, "l")
        with open(c, "w") as f:
            f.write(src)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    vals = dict(line.rsplit(" ", 1) for line in out.strip().splitlines())
    assert int(vals["build"]) == C.sizeof(L.BuildParams)
    assert int(vals["search"]) == C.sizeof(L.SearchParams)
    assert int(vals["info"]) == C.sizeof(L.TablesInfo)
    for key, v in vals.items():
        if "." not in key:
            continue
        sname, field = key.split(".")
        cls = {"finger_build_params": L.BuildParams, "finger_search_params": L.SearchParams,
               "finger_tables_info": L.TablesInfo}[sname]
        assert getattr(cls, field).offset == int(v), key


def _bp(**kw):
    p = L.BuildParams()
    L.load().finger_build_params_init(C.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


@pytest.mark.parametrize("n,m,deg,rank,code,metric,msg", [
    (0, 32, 8, 0, 0, 0, "n = 0"),
    (10, 30, 8, 0, 0, 0, "multiple of 4"),
    (10, 4096, 8, 0, 0, 0, "multiple of 4"),
    (10, 32, 0, 0, 0, 0, "max_degree"),
    (10, 32, 65, 0, 0, 0, "max_degree"),
    (10, 32, 8, 33, 0, 0, "rank"),
    (10, 32, 8, -1, 0, 0, "rank"),
    (10, 32, 8, 8, 7, 0, "code_type"),
    (10, 32, 8, 8, 0, 5, "metric"),
])
def test_build_rejects_bad_arguments(n, m, deg, rank, code, metric, msg):
    lib = L.load()
    p = _bp(rank=rank, code_type=code, metric=metric)
    h = C.c_void_p()
    fake = 1 << 20  # never dereferenced: validation happens first
    st = lib.finger_build_tables(fake, n, m, fake, deg, C.byref(p), C.byref(h), None)
    assert st == L.FINGER_EINVAL
    assert msg in lib.finger_last_error().decode()
    assert h.value is None


def test_build_rejects_null_pointers():
    lib = L.load()
    p = _bp()
    h = C.c_void_p()
    assert lib.finger_build_tables(None, 10, 32, 1 << 20, 8, C.byref(p), C.byref(h), None) == L.FINGER_EINVAL
    assert "data is NULL" in lib.finger_last_error().decode()
    assert lib.finger_build_tables(1 << 20, 10, 32, None, 8, C.byref(p), C.byref(h), None) == L.FINGER_EINVAL
    assert lib.finger_build_tables(1 << 20, 10, 32, 1 << 20, 8, None, C.byref(h), None) == L.FINGER_EINVAL
    assert lib.finger_build_tables(1 << 20, 10, 32, 1 << 20, 8, C.byref(p), None, None) == L.FINGER_EINVAL


def test_build_rejects_non_finite_basis():
    import numpy as np
    lib = L.load()
    p = _bp()
    p.rank = 4
    basis = np.zeros((4, 32))
    basis[2, 5] = np.nan
    p.basis = basis.ctypes.data
    h = C.c_void_p()
    assert lib.finger_build_tables(1 << 20, 10, 32, 1 << 20, 8, C.byref(p), C.byref(h), None) == L.FINGER_EINVAL
    assert "basis entry 69 is not finite" in lib.finger_last_error().decode()


def test_misaligned_data_rejected():
    lib = L.load()
    p = _bp()
    h = C.c_void_p()
    assert lib.finger_build_tables((1 << 20) + 4, 10, 32, 1 << 20, 8, C.byref(p), C.byref(h), None) == L.FINGER_EINVAL
    assert "aligned" in lib.finger_last_error().decode()


def test_no_device_reports_enodev():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    lib = L.load()
    p = _bp()
    h = C.c_void_p()
    st = lib.finger_build_tables(1 << 20, 10, 32, 1 << 20, 8, C.byref(p), C.byref(h), None)
    assert st == L.FINGER_ENODEV


def test_exact_knn_workspace_validation():
    lib = L.load()
    nb = C.c_size_t(0)
    assert lib.finger_exact_knn_workspace_size(100, 32, 10, 0, C.byref(nb)) == L.FINGER_EINVAL
    assert lib.finger_exact_knn_workspace_size(100, 30, 10, 5, C.byref(nb)) == L.FINGER_EINVAL
    assert lib.finger_exact_knn_workspace_size(100, 32, 10, 129, C.byref(nb)) == L.FINGER_EINVAL
    assert lib.finger_exact_knn_workspace_size(100, 32, 10, 5, C.byref(nb)) == L.FINGER_OK
    assert nb.value > 0


def test_null_handle_search_calls():
    lib = L.load()
    sp = L.SearchParams()
    lib.finger_search_params_init(C.byref(sp))
    nb = C.c_size_t(0)
    assert lib.finger_search_workspace_size(None, 1, C.byref(sp), C.byref(nb)) == L.FINGER_EINVAL
    assert lib.finger_search(None, None, 0, C.byref(sp), None, None, None, None, 0, None) == L.FINGER_EINVAL
    info = L.TablesInfo()
    assert lib.finger_tables_info_get(None, C.byref(info)) == L.FINGER_EINVAL
    assert lib.finger_hierarchy_attach(None, 1 << 20, 1 << 20, 4, 16) == L.FINGER_EINVAL
    assert lib.finger_descend(None, 1 << 20, 4, 1 << 20, None, None) == L.FINGER_EINVAL
    assert lib.finger_build_graph(None, 100, 32, 16, 32, 0, 0, 1 << 20, None, L.PROGRESS_FN(), None,
                                  None) == L.FINGER_EINVAL
    # argument checks run before any device work
    for bad in [dict(n=1), dict(m=30), dict(k=0), dict(k=100), dict(W=65), dict(metric=2),
                dict(entry=100), dict(n=1 << 27, k=16)]:
        a = dict(n=100, m=32, k=16, W=32, metric=0, entry=0) | bad
        st = lib.finger_build_graph(1 << 20, a["n"], a["m"], a["k"], a["W"], a["metric"], a["entry"],
                                    1 << 20, None, L.PROGRESS_FN(), None, None)
        assert st in (L.FINGER_EINVAL, L.FINGER_EOVERFLOW), bad
    lib.finger_free_tables(None)  # no-op


def test_gate_param_count():
    lib = L.load()
    # in = 2r + 4 with r = 64, H = 64: 64*132 + 64 + 64*64 + 64 + 64 + 1
    assert lib.finger_gate_param_count(132, 64) == 12737
    assert lib.finger_gate_param_count(0, 64) == 0


# ----------------------------------------------------------- checkpoint

_M = (1 << 64) - 1


def _checksum_spec(data: bytes) -> int:
    """finger_checksum64 written out from its definition in finger.h."""
    h = [0x243F6A8885A308D3, 0x13198A2E03707344, 0xA4093822299F31D0, 0x082EFA98EC4E6C89]
    pad = data + b"\0" * (-len(data) % 8)
    for i in range(len(pad) // 8):
        w = int.from_bytes(pad[8 * i:8 * i + 8], "little")
        x = ((h[i % 4] ^ w) * 0x9E3779B97F4A7C15) & _M
        h[i % 4] = ((x << 31) | (x >> 33)) & _M
    x = len(data)
    for j in range(4):
        x = ((x ^ h[j]) * 0xBF58476D1CE4E5B9) & _M
        x ^= x >> 29
    return x ^ (x >> 32)


@pytest.mark.parametrize("n", [0, 1, 7, 8, 9, 31, 32, 33, 200])
def test_checksum_matches_its_definition(n):
    lib = L.load()
    data = bytes((37 * i + 11) & 0xFF for i in range(n))
    buf = C.create_string_buffer(data, max(n, 1))
    assert lib.finger_checksum64(buf if n else None, n) == _checksum_spec(data)


def _image(n=10, m=32, deg=8, version=1, magic=b"FINGERTB", extra=b""):
    import struct
    hdr = bytearray(200)
    hdr[0:8] = magic
    struct.pack_into("<IIq", hdr, 8, version, 0, n)
    struct.pack_into("<iii", hdr, 24, m, 0, deg)
    body = bytes(hdr) + extra
    return body + _checksum_spec(body).to_bytes(8, "little")


def test_import_checks_the_image_on_the_host():
    """Damaged images are refused before any device call (this runs without
    a GPU); an intact one gets past the host checks."""
    import torch
    lib = L.load()
    h = C.c_void_p()

    def imp(img, n=10, m=32, deg=8):
        b = C.create_string_buffer(img, len(img))
        return lib.finger_tables_import(b, len(img), 1 << 20, n, m, 1 << 20, deg, C.byref(h), None)

    good = _image()
    flipped = bytearray(good)
    flipped[40] ^= 1
    assert imp(bytes(flipped)) == L.FINGER_ECORRUPT
    assert "checksum" in lib.finger_last_error().decode()
    assert imp(good[:100]) == L.FINGER_ECORRUPT
    assert imp(_image(magic=b"NOTFINGR")) == L.FINGER_ECORRUPT
    assert imp(_image(version=2)) == L.FINGER_ECORRUPT
    assert imp(good, n=11) == L.FINGER_EINVAL
    assert imp(good, m=36) == L.FINGER_EINVAL
    st = imp(good)
    if not torch.cuda.is_available():
        assert st == L.FINGER_ENODEV, lib.finger_last_error().decode()
    assert lib.finger_tables_export(None, None, C.byref(C.c_size_t(0))) == L.FINGER_EINVAL


def test_mlp_backward_needs_a_workspace():
    lib = L.load()
    nb = C.c_size_t(0)
    assert lib.finger_mlp_backward_workspace_size(132, 64, 4096, C.byref(nb)) == L.FINGER_OK
    # 128 tiles of 32 samples, each a partial gradient plus its loss term
    assert nb.value == (128 * 12737 + 128) * 4
    assert lib.finger_mlp_backward_workspace_size(600, 64, 10, C.byref(nb)) == L.FINGER_EINVAL
    st = lib.finger_mlp_backward(1 << 20, 132, 64, 1 << 20, 1 << 20, 4096, 1 << 20, None, 1 << 20,
                                 16, None)
    assert st == L.FINGER_EINVAL and "workspace" in lib.finger_last_error().decode()
    st = lib.finger_mlp_backward(1 << 20, 132, 64, 1 << 20, 1 << 20, 4096, 1 << 20, None, None, 0, None)
    assert st == L.FINGER_EINVAL
