"""The symmetry check the graph build makes, as a property of CSR inputs.

Order the slots stably by column and let rev[i] be the i-th of them.  The
build accepts the adjacency as symmetric when, for every slot i of row u with
column v, slot rev[i] lies in row v.  Pinned here against the plain
definition (the edge set equals its reverse) on many small directed graphs,
including degree-balanced asymmetric ones (directed cycles), where counting
degrees alone would pass."""
import numpy as np


def _csr(n, edges):
    edges = sorted(set(edges))
    off = np.zeros(n + 1, np.int64)
    for u, _ in edges:
        off[u + 1] += 1
    off = np.cumsum(off)
    col = np.array([v for _, v in edges], np.int64)
    return off, col


def _check(off, col):
    rev = np.argsort(col, kind="stable")
    ok = True
    for u in range(len(off) - 1):
        for i in range(off[u], off[u + 1]):
            v = col[i]
            if not (off[v] <= rev[i] < off[v + 1]):
                ok = False
    return ok


def _symmetric(n, edges):
    es = set(edges)
    return all((v, u) in es for u, v in es)


def test_check_equals_symmetry_on_random_digraphs():
    rng = np.random.default_rng(3)
    seen = {True: 0, False: 0}
    for _ in range(3000):
        n = int(rng.integers(1, 8))
        m = int(rng.integers(0, n * (n - 1) + 1))
        edges = set()
        for _ in range(m):
            u, v = (int(x) for x in rng.integers(0, n, size=2))
            if u != v:
                edges.add((u, v))
                if rng.random() < 0.7:  # mostly symmetric, so both outcomes occur
                    edges.add((v, u))
        off, col = _csr(n, edges)
        want = _symmetric(n, edges)
        assert _check(off, col) == want, (n, sorted(edges))
        seen[want] += 1
    assert seen[True] > 100 and seen[False] > 100


def test_degree_balanced_asymmetric_graphs_fail_the_check():
    for n in range(3, 9):
        cycle = [(i, (i + 1) % n) for i in range(n)]  # in-degree = out-degree = 1
        off, col = _csr(n, cycle)
        assert not _check(off, col)
    # two opposite triangles on shared vertices plus one directed 3-cycle
    edges = [(0, 1), (1, 0), (1, 2), (2, 1), (2, 3), (3, 4), (4, 2)]
    off, col = _csr(5, edges)
    assert not _check(off, col) and not _symmetric(5, edges)
    off, col = _csr(4, [(0, 1), (1, 0), (2, 3), (3, 2), (0, 2), (2, 0)])
    assert _check(off, col)
