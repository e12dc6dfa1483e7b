"""FP64 CPU oracle for FINGER search (Chen et al., "FINGER: Fast Inference for
Graph-based Approximate Nearest Neighbor Search").

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call,
link or execute anything in this package: only ``tests/``, the smoke check
in ``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` use it.  It
shares no code with the HIP library; the only thing both sides consume is
the seeded inputs from ``workloads``.

Everything here is plain, slow, single-threaded float64 (NumPy, and one
C file):

* ``knn``       exact distances and brute-force kNN, recall@K (Section 1).
* ``rng``       the counter-based generator used to draw build samples.
* ``build``     FINGER construction (Algorithm 2; Section 3.3, Eq. 3,
                Proposition 3.1, distribution matching).
* ``estimate``  the approximate distance (Algorithm 3 with Eq. 1 and Eq. 2),
                written from the definitions, not from the factorized tables.
* ``search``    greedy graph search (Algorithm 1) and approximate greedy
                search (Algorithm 4, Supplementary C).
* ``csearch``   the same two searches compiled as plain C (``csearch.c``),
                for timing the host's cores; cross-checked against
                ``search`` by the tests.
* ``codes``     BF16 / OCP FP8-E4M3 rounding of edge codes (extension; not in
                the paper).
* ``mlp``       the skip-gate network: forward, backward, Adam (extension).

Each function names the passage it follows.  Readings of ambiguous passages
are listed in the module that applies them.
"""
