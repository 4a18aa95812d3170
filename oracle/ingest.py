"""Edge-list clean-up -- the oracle's version.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper counts on undirected simple graphs and prepares its inputs that
way (Section 6: direction ignored, self-loops and repeated edges removed).
Here every pair (a, b) is the undirected edge {a, b}; a == b is dropped; the
neighbour sets are plain Python sets, listed in ascending order.
"""
from __future__ import annotations

import numpy as np


def csr_from_edges(n: int, src, dst):
    """(row_offsets int64[n+1], cols int32[2m]) of the graph of the pairs."""
    adj = [set() for _ in range(n)]
    for a, b in zip(np.asarray(src).tolist(), np.asarray(dst).tolist()):
        if not (0 <= a < n and 0 <= b < n):
            raise ValueError("an endpoint is not a vertex id")
        if a == b:
            continue
        adj[a].add(b)
        adj[b].add(a)
    off = [0]
    col = []
    for v in range(n):
        col.extend(sorted(adj[v]))
        off.append(len(col))
    return np.array(off, dtype=np.int64), np.array(col, dtype=np.int32)
