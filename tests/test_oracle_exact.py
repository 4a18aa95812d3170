"""Pins for the oracle's exact counters (ground truth of the 1% checks).

The brute-force counter is the definition (every 4-subset, Section 2); the
formula counter follows the paper's enumeration-code split (Section 6) plus
Eq. 1.  Both are checked against closed forms, against each other, against
an independent connectivity count, and Eq. 1 itself against the motif graphs.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from paper_1411_4942_amd import synth

# Figure 1, spelled out as edge sets on vertices 0..3
MOTIF_EDGES = {
    1: [(0, 1), (0, 2), (0, 3)],                          # 3-star
    2: [(0, 1), (1, 2), (2, 3)],                          # 3-path
    3: [(0, 1), (1, 2), (0, 2), (2, 3)],                  # tailed-triangle
    4: [(0, 1), (1, 2), (2, 3), (3, 0)],                  # 4-cycle
    5: [(0, 1), (1, 2), (2, 3), (3, 0), (0, 2)],          # chordal-4-cycle
    6: [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)],  # 4-clique
}


def _canon(edges):
    return frozenset(frozenset(e) for e in edges)


def _isomorphic(edges, motif):
    target = _canon(MOTIF_EDGES[motif])
    for p in itertools.permutations(range(4)):
        if _canon((p[a], p[b]) for a, b in edges) == target:
            return True
    return False


def _motif_csr(j):
    a, b = zip(*MOTIF_EDGES[j])
    return synth.csr_from_edges(4, a, b)


def _load_eq1():
    rows = []
    with open(__file__.replace("test_oracle_exact.py", "golden/eq1_matrix.txt")) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([int(x) for x in line.split()])
    return np.array(rows)


def test_eq1_matrix_from_motif_graphs():
    """Eq. 1: A[i][j] = copies of motif i inside motif j, recounted by
    enumerating edge subsets of each motif graph up to isomorphism."""
    A = _load_eq1()
    assert A.shape == (6, 6)
    for j in range(1, 7):
        ej = MOTIF_EDGES[j]
        for i in range(1, 7):
            ni = len(MOTIF_EDGES[i])
            copies = sum(1 for sub in itertools.combinations(ej, ni) if _isomorphic(sub, i))
            assert copies == A[i - 1, j - 1], (i, j)


@pytest.mark.parametrize("counter", [oracle.exact_brute, oracle.exact_formula])
def test_each_motif_graph_is_its_own_class(counter):
    for j in range(1, 7):
        off, col = _motif_csr(j)
        C, T = counter(off, col)
        want = [0] * 7
        want[j] = 1
        assert C == want, (j, C)
        assert T == {1: 0, 2: 0, 3: 1, 4: 0, 5: 2, 6: 4}[j]


def _closed_forms():
    out = []
    for n in range(4, 10):  # K_n: only 4-cliques, C(n,4) of them
        out.append((f"K{n}", synth.complete(n), [0, 0, 0, 0, 0, 0, math.comb(n, 4)], math.comb(n, 3)))
    for n in range(5, 13):  # C_n, n > 4: n 3-paths
        out.append((f"C{n}", synth.cycle(n), [0, 0, n, 0, 0, 0, 0], 0))
    out.append(("C4", synth.cycle(4), [0, 0, 0, 0, 1, 0, 0], 0))
    for n in range(3, 12):  # K_{1,n}: C(n,3) 3-stars
        out.append((f"S{n}", synth.star(n), [0, math.comb(n, 3), 0, 0, 0, 0, 0], 0))
    for n in range(4, 12):  # P_n: n - 3 3-paths
        out.append((f"P{n}", synth.path(n), [0, 0, n - 3, 0, 0, 0, 0], 0))
    for n in range(2, 9):  # K_{2,n}
        out.append((f"K2,{n}", synth.complete_bipartite(2, n),
                    [0, 2 * math.comb(n, 3), 0, 0, math.comb(n, 2), 0, 0], 0))
    out.append(("K3,3", synth.complete_bipartite(3, 3), [0, 6, 0, 0, 9, 0, 0], 0))
    out.append(("empty", synth.empty(7), [0] * 7, 0))
    return out


@pytest.mark.parametrize("name,graph,want,tri", _closed_forms(), ids=[c[0] for c in _closed_forms()])
@pytest.mark.parametrize("counter", [oracle.exact_brute, oracle.exact_formula])
def test_closed_forms(counter, name, graph, want, tri):
    C, T = counter(*graph)
    assert C == want
    assert T == tri


def _connected_4sets(off, col):
    n = off.size - 1
    nbr = [set(col[off[v]:off[v + 1]].tolist()) for v in range(n)]
    total = 0
    for s in itertools.combinations(range(n), 4):
        seen = {s[0]}
        stack = [s[0]]
        while stack:
            x = stack.pop()
            for y in s:
                if y not in seen and y in nbr[x]:
                    seen.add(y)
                    stack.append(y)
        total += len(seen) == 4
    return total


def test_brute_equals_formula_on_random_graphs():
    for seed in range(120):
        rng = np.random.default_rng(seed)
        n = int(rng.integers(4, 28))
        p = float(rng.uniform(0.05, 0.9))
        off, col = synth.gnp(n, p, seed)
        assert oracle.exact_brute(off, col) == oracle.exact_formula(off, col), seed


def test_counts_sum_to_connected_4_subsets():
    for seed in range(25):
        rng = np.random.default_rng(1000 + seed)
        n = int(rng.integers(4, 13))
        off, col = synth.gnp(n, float(rng.uniform(0.1, 0.8)), 1000 + seed)
        C, _ = oracle.exact_brute(off, col)
        assert sum(C[1:]) == _connected_4sets(off, col)


def test_formula_counter_is_label_invariant():
    off, col = synth.erdos_renyi(300, 3000, 5)
    rng = np.random.default_rng(3)
    perm = rng.permutation(300)
    assert oracle.exact_formula(off, col) == oracle.exact_formula(*synth.permute(off, col, perm))


def test_formula_matches_brute_on_denser_medium_graph():
    off, col = synth.chung_lu(120, 900, 2.3, 40.0, 7)
    assert oracle.exact_brute(off, col) == oracle.exact_formula(off, col)


def test_rejects_invalid_input():
    off, col = synth.complete(5)
    bad = col.copy()
    bad[0], bad[1] = bad[1], bad[0]
    with pytest.raises(oracle.OracleError):
        oracle.exact_formula(off, bad)
