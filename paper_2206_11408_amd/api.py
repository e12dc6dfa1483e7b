"""Python binding of libfinger with the C entry points' names.

Only argument marshalling happens here: torch supplies device memory and
the current HIP stream; every step of build and search runs in the
library's kernels.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _ptr(t: torch.Tensor | None) -> int | None:
    return None if t is None else t.data_ptr()


def _dev_i32(x, device="cuda") -> torch.Tensor:
    if isinstance(x, torch.Tensor):
        return x.to(device=device, dtype=torch.int32).contiguous()
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.int32, device=device)


def _dev_f32(x, device="cuda") -> torch.Tensor:
    if isinstance(x, torch.Tensor):
        return x.to(device=device, dtype=torch.float32).contiguous()
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float32, device=device)


def _workspace(nbytes: int, device) -> torch.Tensor:
    # torch's caching allocator hands out 512-byte aligned blocks
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)


class Tables:
    """Owns a finger_tables handle and keeps the borrowed data/graph alive."""

    def __init__(self, handle: int, data: torch.Tensor, graph: torch.Tensor, extra=()):
        self.handle = handle
        self._keep = (data, graph, *extra)
        self.data = data
        self.graph = graph
        self._ws = None

    def info(self) -> dict:
        inf = L.TablesInfo()
        L.check(L.load().finger_tables_info_get(self.handle, C.byref(inf)))
        return {name: getattr(inf, name) for name, _ in L.TablesInfo._fields_}

    def read(self, which: int) -> np.ndarray:
        """finger_tables_read into a numpy array of the table's element type."""
        lib = L.load()
        nbytes = C.c_size_t(0)
        L.check(lib.finger_tables_read(self.handle, which, None, C.byref(nbytes)))
        buf = np.empty(nbytes.value, dtype=np.uint8)
        L.check(lib.finger_tables_read(self.handle, which, buf.ctypes.data, C.byref(nbytes)))
        inf = self.info()
        n, m, r, deg = inf["n"], inf["m"], inf["rank"], inf["max_degree"]
        rpad = (r + 31) // 32 * 32
        if which in (L.T_P_F64,):
            return buf.view(np.float64).reshape(r, m)
        if which == L.T_EIGVALS:
            return buf.view(np.float64)
        if which == L.T_P_F32:
            return buf.view(np.float32).reshape(r, m)
        if which == L.T_NODE_CC:
            return buf.view(np.float32)
        if which == L.T_NODE_PC:
            return buf.view(np.float32).reshape(n, r)
        if which in (L.T_EDGE_ALPHA, L.T_EDGE_RHO):
            return buf.view(np.float32).reshape(n, deg)
        if which == L.T_EDGE_CODES:
            dt = {L.CODE_F32: np.float32, L.CODE_BF16: np.uint16, L.CODE_FP8E4M3: np.uint8}[inf["code_type"]]
            return buf.view(dt).reshape(n, deg, rpad)
        if which == L.T_EDGE_SCALE:
            return buf.view(np.float32)
        if which == L.T_SAMPLES:
            return buf.view(np.int32).reshape(-1, 3)
        if which == L.T_XY:
            return buf.view(np.float64).reshape(-1, 2)
        return buf

    def close(self) -> None:
        if self.handle:
            L.load().finger_free_tables(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def finger_build_tables(data: torch.Tensor, graph: torch.Tensor, rank: int = 0,
                        code_type: int = L.CODE_F32, metric: int = L.L2,
                        sigma_mode: int = L.SIGMA_STD, n_samples: int = 0, seed: int = 0,
                        pivots=None, dm_override=None, basis=None) -> Tables:
    """FINGER tables for ``data`` over ``graph`` (finger_build_tables).
    ``basis``: optional float64 [rank][m] array used as P instead of the
    eigenvector basis."""
    lib = L.load()
    data = _dev_f32(data)
    graph = _dev_i32(graph)
    n, m = data.shape
    deg = graph.shape[1]
    p = L.BuildParams()
    lib.finger_build_params_init(C.byref(p))
    p.rank = rank
    p.code_type = code_type
    p.metric = metric
    p.sigma_mode = sigma_mode
    p.n_samples = n_samples
    p.seed = seed
    piv = None
    if pivots is not None:
        piv = _dev_i32(pivots)
        p.pivots = piv.data_ptr()
        p.n_pivots = piv.numel()
    if dm_override is not None:
        p.dm_override = 1
        for i, v in enumerate(dm_override):
            p.dm[i] = float(v)
    bas = None
    if basis is not None:
        bas = np.ascontiguousarray(np.asarray(basis, dtype=np.float64))
        if bas.shape != (rank, m):
            raise ValueError(f"basis must be [{rank}][{m}], got {bas.shape}")
        p.basis = bas.ctypes.data
    h = C.c_void_p()
    L.check(lib.finger_build_tables(data.data_ptr(), n, m, graph.data_ptr(), deg, C.byref(p),
                                    C.byref(h), _stream()))
    return Tables(h.value, data, graph, (piv,) if piv is not None else ())


def search_params(mode=L.MODE_PLAIN, k=10, ef=64, entry=0, warmup=5, k_max=None,
                  k_per_query=None, ef_per_query=None, ef_max=0, persistent=0,
                  waves_per_cu=0, visited_capacity=0, code_prefetch=0,
                  log=None, spill_capacity=0, screen_layout=0, ef_classes=0,
                  gate_band=0.0, visited_probe=0) -> L.SearchParams:
    p = L.SearchParams()
    L.load().finger_search_params_init(C.byref(p))
    p.mode, p.k, p.ef, p.entry, p.warmup = mode, k, ef, entry, warmup
    p.k_max = k if k_max is None else k_max
    p.k_per_query = _ptr(k_per_query)
    p.ef_per_query = _ptr(ef_per_query)
    p.ef_max, p.persistent = ef_max, persistent
    p.waves_per_cu, p.visited_capacity = waves_per_cu, visited_capacity
    p.spill_capacity = spill_capacity
    p.visited_probe = visited_probe
    p.screen_layout = screen_layout
    p.ef_classes = ef_classes
    p.gate_band = gate_band
    p.code_prefetch = code_prefetch
    if log is not None:
        feats, targs, count = log
        p.log_features, p.log_targets = feats.data_ptr(), targs.data_ptr()
        p.log_capacity = feats.shape[0]
        p.log_count = count.data_ptr()
    # the struct holds raw device pointers: keep their tensors alive with it
    p._keep = (k_per_query, ef_per_query, log)
    return p


def finger_search_workspace_size(tables: Tables, nq: int, p: L.SearchParams) -> int:
    nbytes = C.c_size_t(0)
    L.check(L.load().finger_search_workspace_size(tables.handle, nq, C.byref(p), C.byref(nbytes)))
    return nbytes.value


def check_status(ctr: torch.Tensor) -> None:
    """Raise FingerError(EOVERFLOW) if any query's status counter reports a
    visited-set overflow (its results are not valid).  Synchronizes."""
    bad = int(((ctr[:, L.NCOUNTERS - 1] & 1) != 0).sum().item())
    if bad:
        raise L.FingerError(L.FINGER_EOVERFLOW,
                            f"visited set overflowed on {bad} queries; raise visited_capacity "
                            f"or spill_capacity")


def finger_search(tables: Tables, queries: torch.Tensor, p: L.SearchParams | None = None,
                  out=None, counters: bool = True, check: bool = True, **kw):
    """Run finger_search; returns (ids int32 [nq, k_max], dist f32 [nq, k_max],
    counters int32 [nq, 7] or None).  Pass ``out=(ids, dist, ctr)`` to reuse
    buffers (timing loops).  With counters and ``check`` the call waits for
    the search and raises FingerError(EOVERFLOW) if a query's visited set
    overflowed; ``check=False`` keeps it asynchronous (then call
    ``check_status`` on the counters)."""
    lib = L.load()
    if p is None:
        p = search_params(**kw)
    queries = _dev_f32(queries)
    nq = queries.shape[0]
    need = finger_search_workspace_size(tables, nq, p)
    if tables._ws is None or tables._ws.numel() < need:
        tables._ws = _workspace(need, queries.device)
    if out is None:
        ids = torch.empty((nq, p.k_max), dtype=torch.int32, device=queries.device)
        dist = torch.empty((nq, p.k_max), dtype=torch.float32, device=queries.device)
        ctr = torch.empty((nq, L.NCOUNTERS), dtype=torch.int32, device=queries.device) if counters else None
    else:
        ids, dist, ctr = out
    L.check(lib.finger_search(tables.handle, queries.data_ptr(), nq, C.byref(p), ids.data_ptr(),
                              dist.data_ptr(), _ptr(ctr), tables._ws.data_ptr(),
                              tables._ws.numel(), _stream()))
    if check and ctr is not None:
        check_status(ctr)
    return ids, dist, ctr


def finger_build_graph(data: torch.Tensor, knn_k: int = 16, max_degree: int = 32, entry: int = 0,
                       metric: int = L.L2, progress=None):
    """The flat graph built on the GPU (finger_build_graph): returns
    (graph int32 [n, max_degree] on the data's device, stats dict).
    ``progress(phase, done, total)`` is called after each step."""
    data = _dev_f32(data)
    n, m = data.shape
    G = torch.empty((n, max_degree), dtype=torch.int32, device=data.device)
    st = L.GraphStats()
    cb = L.PROGRESS_FN(lambda ph, d, t, _u: progress(ph.decode(), d, t)) if progress else L.PROGRESS_FN()
    L.check(L.load().finger_build_graph(data.data_ptr(), n, m, knn_k, max_degree, metric, entry,
                                        G.data_ptr(), C.byref(st), cb, None, _stream()))
    return G, {name: getattr(st, name) for name, _ in L.GraphStats._fields_}


def finger_build_graph_grouped(data: torch.Tensor, group_offsets, knn_k: int = 16,
                               max_degree: int = 32, entry: int = 0, metric: int = L.L2,
                               progress=None):
    """finger_build_graph with each point's kNN taken inside its own group
    (finger_build_graph_grouped); ``group_offsets`` [n_groups + 1] from 0 to n
    delimits contiguous groups of rows."""
    data = _dev_f32(data)
    n, m = data.shape
    off = np.ascontiguousarray(np.asarray(group_offsets, dtype=np.int64))
    G = torch.empty((n, max_degree), dtype=torch.int32, device=data.device)
    st = L.GraphStats()
    cb = L.PROGRESS_FN(lambda ph, d, t, _u: progress(ph.decode(), d, t)) if progress else L.PROGRESS_FN()
    L.check(L.load().finger_build_graph_grouped(data.data_ptr(), n, m, knn_k, max_degree, metric, entry,
                                                off.ctypes.data, off.size - 1, G.data_ptr(), C.byref(st),
                                                cb, None, _stream()))
    return G, {name: getattr(st, name) for name, _ in L.GraphStats._fields_}


def finger_hierarchy_attach(tables: Tables, levels, upper) -> None:
    """Attach the upper layers of an HNSW-style hierarchy (levels [n],
    node-major rows upper [rows][width]); searches may then use
    entry=L.ENTRY_DESCENT."""
    lv = _dev_i32(levels)
    up = _dev_i32(upper)
    if up.dim() != 2:
        raise ValueError("upper must be [rows][width]")
    L.check(L.load().finger_hierarchy_attach(tables.handle, lv.data_ptr(), up.data_ptr(),
                                             up.shape[0], up.shape[1]))


def finger_descend(tables: Tables, queries: torch.Tensor, calls: bool = True):
    """Start point of each query from the attached upper layers:
    (entries int32 [nq], distance evaluations int32 [nq] or None)."""
    queries = _dev_f32(queries)
    nq = queries.shape[0]
    ent = torch.empty(nq, dtype=torch.int32, device=queries.device)
    cnt = torch.empty(nq, dtype=torch.int32, device=queries.device) if calls else None
    L.check(L.load().finger_descend(tables.handle, queries.data_ptr(), nq, ent.data_ptr(),
                                    cnt.data_ptr() if cnt is not None else None, _stream()))
    return ent, cnt


def finger_estimate_edges(tables: Tables, queries: torch.Tensor, q_index, centers, slots):
    lib = L.load()
    queries = _dev_f32(queries)
    qi, ci, si = _dev_i32(q_index), _dev_i32(centers), _dev_i32(slots)
    n_items = qi.numel()
    est = torch.empty(n_items, dtype=torch.float32, device=queries.device)
    that = torch.empty(n_items, dtype=torch.float32, device=queries.device)
    L.check(lib.finger_estimate_edges(tables.handle, queries.data_ptr(), queries.shape[0],
                                      qi.data_ptr(), ci.data_ptr(), si.data_ptr(), n_items,
                                      est.data_ptr(), that.data_ptr(), _stream()))
    return est, that


def finger_exact_knn(data: torch.Tensor, queries: torch.Tensor, k: int, metric: int = L.L2):
    lib = L.load()
    data = _dev_f32(data)
    queries = _dev_f32(queries)
    n, m = data.shape
    nq = queries.shape[0]
    nbytes = C.c_size_t(0)
    L.check(lib.finger_exact_knn_workspace_size(n, m, nq, k, C.byref(nbytes)))
    ws = _workspace(nbytes.value, data.device)
    ids = torch.empty((nq, k), dtype=torch.int32, device=data.device)
    dist = torch.empty((nq, k), dtype=torch.float32, device=data.device)
    L.check(lib.finger_exact_knn(data.data_ptr(), n, m, queries.data_ptr(), nq, k, metric,
                                 ids.data_ptr(), dist.data_ptr(), ws.data_ptr(), ws.numel(),
                                 _stream()))
    return ids, dist


# ---------------------------------------------------------------- gate

def finger_gate_param_count(in_dim: int, hidden: int) -> int:
    return int(L.load().finger_gate_param_count(in_dim, hidden))


def finger_gate_attach(tables: Tables, weights, in_dim: int, hidden: int, eps_gate: float) -> None:
    w = np.ascontiguousarray(np.asarray(weights, dtype=np.float32))
    L.check(L.load().finger_gate_attach(tables.handle, w.ctypes.data, in_dim, hidden, float(eps_gate)))


def finger_mlp_forward(weights: torch.Tensor, in_dim: int, hidden: int, x: torch.Tensor,
                       y: torch.Tensor | None = None) -> torch.Tensor:
    if y is None:
        y = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
    L.check(L.load().finger_mlp_forward(weights.data_ptr(), in_dim, hidden, x.data_ptr(),
                                        x.shape[0], y.data_ptr(), _stream()))
    return y


def finger_mlp_backward_workspace_size(in_dim: int, hidden: int, batch: int) -> int:
    nbytes = C.c_size_t(0)
    L.check(L.load().finger_mlp_backward_workspace_size(in_dim, hidden, batch, C.byref(nbytes)))
    return nbytes.value


def finger_mlp_backward(weights: torch.Tensor, in_dim: int, hidden: int, x: torch.Tensor,
                        target: torch.Tensor, grad: torch.Tensor | None = None,
                        loss: torch.Tensor | None = None, workspace: torch.Tensor | None = None):
    """Gradient of the mean squared error (finger_mlp_backward).  Pass a
    ``workspace`` of finger_mlp_backward_workspace_size bytes to reuse it."""
    if grad is None:
        grad = torch.empty_like(weights)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
    need = finger_mlp_backward_workspace_size(in_dim, hidden, x.shape[0])
    if workspace is None or workspace.numel() < need:
        workspace = _workspace(need, x.device)
    L.check(L.load().finger_mlp_backward(weights.data_ptr(), in_dim, hidden, x.data_ptr(),
                                         target.data_ptr(), x.shape[0], grad.data_ptr(),
                                         loss.data_ptr(), workspace.data_ptr(), workspace.numel(),
                                         _stream()))
    return grad, loss


def finger_gate_calibrate(weights: torch.Tensor, in_dim: int, hidden: int, x: torch.Tensor,
                          target: torch.Tensor) -> float:
    """eps_gate = mean |target - f(x)| over the rows (finger_gate_calibrate)."""
    out = C.c_double(0.0)
    L.check(L.load().finger_gate_calibrate(weights.data_ptr(), in_dim, hidden, x.data_ptr(),
                                           target.data_ptr(), x.shape[0], C.byref(out), _stream()))
    return out.value


def finger_gate_targets(log_features: torch.Tensor, log_targets: torch.Tensor, rows: int,
                        rank: int) -> torch.Tensor:
    out = torch.empty(rows, dtype=torch.float32, device=log_features.device)
    L.check(L.load().finger_gate_targets(log_features.data_ptr(), log_targets.data_ptr(), rows,
                                         rank, out.data_ptr(), _stream()))
    return out


def finger_adam_step(weights, grad, m1, m2, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, step=1):
    L.check(L.load().finger_adam_step(weights.data_ptr(), grad.data_ptr(), m1.data_ptr(),
                                      m2.data_ptr(), weights.numel(), lr, beta1, beta2, eps,
                                      step, _stream()))


# ----------------------------------------------------------- checkpoint

def finger_tables_export(tables: Tables) -> np.ndarray:
    """The handle's tables image (finger_tables_export) as a uint8 array."""
    lib = L.load()
    nbytes = C.c_size_t(0)
    L.check(lib.finger_tables_export(tables.handle, None, C.byref(nbytes)))
    buf = np.empty(nbytes.value, dtype=np.uint8)
    L.check(lib.finger_tables_export(tables.handle, buf.ctypes.data, C.byref(nbytes)))
    return buf


def finger_tables_import(image, data: torch.Tensor, graph: torch.Tensor) -> Tables:
    """A handle from an image (finger_tables_import) over ``data`` and
    ``graph``, which must be the points and graph the tables were built on."""
    buf = np.ascontiguousarray(np.frombuffer(image, dtype=np.uint8) if not isinstance(image, np.ndarray)
                               else image.view(np.uint8).ravel())
    data = _dev_f32(data)
    graph = _dev_i32(graph)
    h = C.c_void_p()
    L.check(L.load().finger_tables_import(buf.ctypes.data, buf.size, data.data_ptr(), data.shape[0],
                                          data.shape[1], graph.data_ptr(), graph.shape[1],
                                          C.byref(h), _stream()))
    return Tables(h.value, data, graph)


def finger_tables_save(tables: Tables, path: str) -> int:
    """Write the tables image to ``path``; returns its size in bytes."""
    buf = finger_tables_export(tables)
    buf.tofile(path)
    return int(buf.size)


def finger_tables_load(path: str, data: torch.Tensor, graph: torch.Tensor) -> Tables:
    return finger_tables_import(np.fromfile(path, dtype=np.uint8), data, graph)
