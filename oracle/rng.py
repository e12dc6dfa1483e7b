"""Counter-based generator for FINGER's build-time sampling.  Test
infrastructure only.

Algorithm 2 samples, for each node c, a pair of distinct neighbours d, d'.
The paper does not fix the generator; both the oracle and the library use
SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014), each written independently from that definition:
the j-th output (j = 0, 1, ...) of the stream seeded with s is
mix(s + (j + 1) * 0x9E3779B97F4A7C15 mod 2^64), where
mix(z) = z ^ (z >> 31) after z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9 and
z = (z ^ (z >> 27)) * 0x94D049BB133111EB, all mod 2^64.

Sampling recipe for sample i of N_s = min(n, n_samples):
  * c_i = i when N_s == n, else c_i = h(3i) mod n (with replacement);
  * deg = number of valid (>= 0) slots of row c_i (valid slots come first);
    a sample whose node has deg < 2 is dropped;
  * slot a = h(3i+1) mod deg, slot b = (a + 1 + h(3i+2) mod (deg - 1)) mod deg,
    so a != b; d = G[c_i][a], d' = G[c_i][b].
"""
from __future__ import annotations

import numpy as np

_MASK = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15


def splitmix64(seed: int, j: int) -> int:
    """The j-th output of the SplitMix64 stream seeded with ``seed``."""
    z = (int(seed) + (int(j) + 1) * GAMMA) & _MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
    return z ^ (z >> 31)


def sample_pairs(graph: np.ndarray, n_samples: int, seed: int):
    """Return int64 arrays (c, d, d') of the kept samples, in sample order,
    and the sample indices i they came from."""
    n = graph.shape[0]
    ns = min(n, int(n_samples))
    cs, ds, dps, idx = [], [], [], []
    for i in range(ns):
        c = i if ns == n else splitmix64(seed, 3 * i) % n
        row = graph[c]
        deg = 0
        while deg < row.shape[0] and row[deg] >= 0:
            deg += 1
        if deg < 2:
            continue
        a = splitmix64(seed, 3 * i + 1) % deg
        b = (a + 1 + splitmix64(seed, 3 * i + 2) % (deg - 1)) % deg
        cs.append(c)
        ds.append(int(row[a]))
        dps.append(int(row[b]))
        idx.append(i)
    return (np.array(cs, dtype=np.int64), np.array(ds, dtype=np.int64),
            np.array(dps, dtype=np.int64), np.array(idx, dtype=np.int64))
