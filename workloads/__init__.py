"""Seeded synthetic inputs shared by the HIP path's tests/bench and the oracle.

This package holds only input construction: point sets drawn from seeded
mixtures, and the proximity graph a search runs over (exact kNN, symmetrize,
neighbour-selection pruning, reachability repair, entry choice, and the
upper layers of an HNSW-style hierarchy).  It holds
none of FINGER's arithmetic (no residual split, basis, distribution matching,
estimate or search); both the oracle and the GPU path consume what it
produces and neither is imported here.
"""
from .gen import (  # noqa: F401
    WorkloadSpec,
    SPECS,
    gate_weights,
    gaussian_projection,
    make_points,
)
from .graph import (  # noqa: F401
    knn_lists,
    symmetrize,
    prune_heuristic,
    repair_reachability,
    medoid,
    build_graph,
    pick_pivots,
    draw_levels,
    build_hierarchy,
)
