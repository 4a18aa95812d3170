"""GPU exact counter (pm_exact_counts) against the oracle's exact counts.

Induced counts C_1..C_6 and the triangle count must equal the oracle's
formula counter exactly, and the subgraph counts N must equal A C with A the
matrix of Eq. 1 (tests/golden/eq1_matrix.txt), on small structured graphs,
random graphs, power-law graphs, and the Chung-Lu 1e6/1e7 workload.
"""
import os
import sys
import time

import numpy as np
import pytest

import oracle
from paper_1411_4942_amd import pathsamp as ps
from paper_1411_4942_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

A = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "eq1_matrix.txt"), dtype=np.int64).astype(object)


def _say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def _dev(off, col):
    return (torch.from_numpy(np.ascontiguousarray(off, np.int64)).cuda(),
            torch.from_numpy(np.ascontiguousarray(col, np.int32)).cuda())


def _graphs():
    gs = [
        ("K8", synth.complete(8)), ("C10", synth.cycle(10)), ("star9", synth.star(9)),
        ("K3,3", synth.complete_bipartite(3, 3)), ("K2,30", synth.complete_bipartite(2, 30)),
        ("P7", synth.path(7)), ("empty6", synth.empty(6)),
    ]
    for seed in range(12):
        rng = np.random.default_rng(seed)
        n = int(rng.integers(5, 80))
        m = int(rng.integers(n - 1, min(n * (n - 1) // 2, 6 * n) + 1))
        gs.append((f"gnm{seed}", synth.erdos_renyi(n, m, 100 + seed)))
    gs.append(("er_2000_20000", synth.erdos_renyi(2000, 20000, 1)))
    gs.append(("chunglu_50k_500k", synth.chung_lu(50000, 500000, 2.3, 1000.0, 9)))
    gs.append(("rmat_s14", synth.rmat(14, 16, seed=2)))
    # dense: forward rows of every 4-clique class (up to 64, 256, 1024 members)
    gs.append(("er_dense_400", synth.erdos_renyi(400, 40000, 3)))
    gs.append(("cliques_300_70_40", _disjoint([synth.complete(300), synth.complete(70), synth.complete(40),
                                               synth.erdos_renyi(500, 3000, 4)])))
    return gs


def _disjoint(parts):
    """Disjoint union of CSR graphs (vertex ids shifted)."""
    offs, cols, base, top = [np.zeros(1, np.int64)], [], 0, 0
    for off, col in parts:
        offs.append(off[1:].astype(np.int64) + top)
        cols.append(col.astype(np.int64) + base)
        base += off.size - 1
        top += int(off[-1])
    return np.concatenate(offs), np.concatenate(cols).astype(np.int32)


GRAPHS = _graphs()


def _check(name, off, col, got):
    C, T = oracle.exact_formula(off, col)
    assert got["C"][1:] == [int(c) for c in C[1:]], name
    assert got["triangles"] == int(T), name
    N = A.dot(np.array([int(c) for c in C[1:]], dtype=object))
    assert got["N"][1:] == [int(x) for x in N], name


@pytest.mark.parametrize("name,graph", GRAPHS, ids=[g[0] for g in GRAPHS])
def test_exact_counts_equal_oracle(name, graph):
    _say("exact", name)
    off, col = graph
    g = ps.Graph(*_dev(off, col))
    got = g.exact()
    g.destroy()
    _check(name, off, col, got)


@pytest.mark.parametrize("n", [1100, 2800])
def test_exact_counts_complete_closed_form(n):
    """K_n: C(n, 4) 4-cliques and nothing else.  Its lowest vertices have up
    to n - 1 forward neighbours, past the LDS classes of the clique counter:
    for n = 1100 the members and their hash still fit in LDS beside rows in
    global memory; for n = 2800 they do not, and members are found by binary
    search in global memory."""
    _say(f"exact K{n}")
    off, col = synth.complete(n)
    g = ps.Graph(*_dev(off, col))
    got = g.exact()
    g.destroy()
    assert got["C"][1:] == [0, 0, 0, 0, 0, n * (n - 1) * (n - 2) * (n - 3) // 24]
    assert got["triangles"] == n * (n - 1) * (n - 2) // 6


@pytest.mark.parametrize("m", [60000, 70000])
def test_exact_counts_k2m_closed_form(m):
    """K_{2,m}: the higher hub's m lower neighbours (the leaves) all pair it
    with the other hub, so that pair's wedge count is m: just below 2^16
    (m = 60000, the 4-cycle counter's 16-bit mode) or above it (m = 70000,
    its 32-bit mode).  Induced counts: 2 C(m, 3) 3-stars and C(m, 2)
    4-cycles, nothing else."""
    _say(f"exact K2,{m}")
    off, col = synth.complete_bipartite(2, m)
    g = ps.Graph(*_dev(off, col))
    got = g.exact()
    g.destroy()
    assert got["C"][1:] == [2 * (m * (m - 1) * (m - 2) // 6), 0, 0, m * (m - 1) // 2, 0, 0]
    assert got["triangles"] == 0


def test_exact_counts_chunglu_1e6_1e7():
    _say("exact chung-lu 1e6/1e7")
    off_d, col_d = synth.chung_lu_torch(1_000_000, 10_000_000, 2.3, 5000.0, 1, device="cuda")
    g = ps.Graph(off_d, col_d)
    t0 = time.time()
    got = g.exact()
    _say("exact on device", f"{time.time() - t0:.2f}s")
    g.destroy()
    _check("chunglu_1e6_1e7", off_d.cpu().numpy(), col_d.cpu().numpy(), got)
