"""Launch-geometry autotuner for finger_search.

The search is one wavefront per query; its throughput depends on how many
query waves each CU keeps resident (latency hiding versus LDS and register
pressure), on whether queries are handed out by an atomic work queue
(uneven K/ef) or statically, and, in FINGER mode, on whether every slot's
edge code is requested with the adjacency row.  ``autotune`` times a
sample of queries for each candidate, keeps the fastest, and caches the
choice in a JSON file keyed by the workload's shape; none of the choices
changes results (a property the tests check).
"""
from __future__ import annotations

import json
import os

import torch

from . import _lib as L
from . import api

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "finger_tune.json")


def _key(tables: api.Tables, mode: int, ef_max: int, mixed: bool) -> str:
    inf = tables.info()
    dev = torch.cuda.get_device_properties(torch.cuda.current_device())
    return (f"{dev.gcnArchName}|n{inf['n']}|m{inf['m']}|r{inf['rank']}|deg{inf['max_degree']}|"
            f"code{inf['code_type']}|mode{mode}|ef{ef_max}|mixed{int(mixed)}")


def candidates(mode: int, ef_max: int = 64, mixed: bool = False):
    # visited-set capacity trades LDS per wave (resident waves) against probe
    # length and spills; the library default is 2048.  With the small table a
    # shorter LDS probe (8 slots instead of 24) spills sooner but walks less
    # of a nearly full table.  Searches with per-query K or ef always run
    # persistent launches.
    vis = ((1024, 24), (1024, 8), (2048, 24), (4096, 24))
    out = []
    for wpc in (8, 12, 16, 20, 24, 32):
        for persistent in ((1,) if mixed else (0, 1)):
            pfs = (0,) if mode == L.MODE_PLAIN else (-1, 1)
            for pf in pfs:
                for vc, vp in vis:
                    out.append({"waves_per_cu": wpc, "persistent": persistent, "code_prefetch": pf,
                                "visited_capacity": vc, "visited_probe": vp})
    return out


def autotune(tables: api.Tables, queries: torch.Tensor, base: dict, repeats: int = 3,
             cache_path: str | None = DEFAULT_CACHE, force: bool = False, log=None) -> dict:
    """Pick launch settings for ``finger_search`` with parameters ``base``
    (keyword arguments of api.search_params).  Returns the chosen settings
    plus the measured milliseconds of each candidate."""
    mode = base.get("mode", L.MODE_PLAIN)
    mixed = base.get("ef_per_query") is not None or base.get("k_per_query") is not None
    ef_max = base.get("ef_max", 0) or max(base.get("ef", 64), base.get("k", 10))
    key = _key(tables, mode, ef_max, mixed)
    cache = {}
    if cache_path and os.path.exists(cache_path) and not force:
        try:
            with open(cache_path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
        if key in cache:
            return cache[key]
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    timings = []
    for cand in candidates(mode, ef_max, mixed):
        p = api.search_params(**{**base, **cand})
        try:
            api.finger_search(tables, queries, p)
        except L.FingerError:
            continue  # e.g. more waves than LDS allows
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(repeats):
            ev0.record()
            api.finger_search(tables, queries, p, check=False)
            ev1.record()
            ev1.synchronize()
            best = min(best, ev0.elapsed_time(ev1))
        timings.append((best, cand))
        if log:
            log(f"tune {cand}: {best:.3f} ms")
    timings.sort(key=lambda x: x[0])
    choice = dict(timings[0][1])
    choice["ms"] = timings[0][0]
    choice["all"] = [[t, c] for t, c in timings]
    if cache_path:
        cache[key] = choice
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return choice
