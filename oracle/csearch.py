"""Loader for ``csearch.c``: the oracle's greedy search (Algorithm 1) and
approximate greedy search (Algorithm 4) compiled as plain C in float64.
Test infrastructure only.

``search_batch`` has the same inputs and outputs as
``oracle.search.search_batch`` for one ef and K over all queries, with the
one-bound-per-expansion reading of Algorithm 4 and the L2 or inner-product
metric; ``threads`` splits the queries into contiguous ranges searched at
once (the C code is reentrant and ctypes releases the interpreter lock).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csearch.c")
LIB = os.path.join(HERE, "libcsearch.so")

_lib = None


def build() -> str:
    """Compile the shared library next to its source (plain -O2, no fused
    multiply-add, so every operation rounds as written)."""
    tmp = LIB + f".tmp{os.getpid()}"
    subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared", "-o", tmp,
                    SRC, "-lm"], check=True)
    os.replace(tmp, LIB)
    return LIB


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        lib = ctypes.CDLL(LIB)
        p, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        lib.oracle_search_batch.argtypes = [p, i64, i32, p, i32, p, i64, p, i32, i32, i32, i32, i32,
                                            p, i32, p, p, p, p, p]
        lib.oracle_search_batch.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def search_batch(data, graph, queries, entries, ef: int, k: int, mode: str = "plain",
                 tables: dict | None = None, warmup: int = 5, metric: str = "l2",
                 threads: int = 1):
    """Returns (ids int64 [nq, k], d2 float64 [nq, k], counters int64 [nq, 6]
    in the order expansions, exact, screened, skipped, visited, preps,
    margins float64 [nq])."""
    lib = load()
    X = np.ascontiguousarray(data, dtype=np.float64)
    G = np.ascontiguousarray(graph, dtype=np.int32)
    Q = np.ascontiguousarray(np.atleast_2d(queries), dtype=np.float64)
    n, m = X.shape
    nq = Q.shape[0]
    E = np.ascontiguousarray(np.broadcast_to(np.asarray(entries, dtype=np.int64), (nq,)))
    assert G.shape[0] == n and Q.shape[1] == m
    md = {"plain": 0, "finger": 1}[mode]
    mt = {"l2": 0, "ip": 2}[metric]
    P = dm = None
    r = 0
    if md == 1:
        P = np.ascontiguousarray(tables["P"], dtype=np.float64)
        r = P.shape[0]
        dm = np.array([tables["mu"], tables["sigma"], tables["mu_hat"], tables["sigma_hat"],
                       tables["eps"]], dtype=np.float64)
    ids = np.empty((nq, k), dtype=np.int64)
    d2 = np.empty((nq, k), dtype=np.float64)
    cnt = np.empty((nq, 6), dtype=np.int64)
    mg = np.empty(nq, dtype=np.float64)

    def run(lo, hi):
        if hi <= lo:
            return 0
        return lib.oracle_search_batch(_ptr(X), n, m, _ptr(G), G.shape[1], _ptr(Q[lo:hi]), hi - lo,
                                       _ptr(E[lo:hi]), int(ef), int(k), md, mt, int(warmup), _ptr(P),
                                       r, _ptr(dm), _ptr(ids[lo:hi]), _ptr(d2[lo:hi]),
                                       _ptr(cnt[lo:hi]), _ptr(mg[lo:hi]))

    threads = max(1, min(int(threads), nq))
    bounds = [nq * t // threads for t in range(threads + 1)]
    if threads == 1:
        rcs = [run(0, nq)]
    else:
        with ThreadPoolExecutor(threads) as ex:
            rcs = list(ex.map(run, bounds[:-1], bounds[1:]))
    if any(rc != 0 for rc in rcs):
        raise RuntimeError(f"oracle_search_batch failed: {rcs}")
    return ids, d2, cnt, mg
