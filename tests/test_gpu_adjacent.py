"""The adjacency test of the samplers, queried directly (pm_adjacent).

Every search mode (row hash, per-lane and wave-cooperative sorted-row
search) must answer "are a and b adjacent?" exactly as the oracle's
relabelled CSR does: on every edge of the graph, on random non-adjacent
pairs, and on pairs inside hub rows built window by window (rows longer
than one LDS window of the row-hash build), rows of every small length and
rows on both sides of each build class bound.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1411_4942_amd import pathsamp as ps
from paper_1411_4942_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

MODES = [ps.SEARCH_HASH, ps.SEARCH_LANE, ps.SEARCH_WAVE]


def _say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def _graphs():
    return [
        ("K9", synth.complete(9)),
        ("star_100000", synth.star(100_000)),  # one row of 1e5: several build windows
        ("hub_classes", synth.hubs([1, 2, 1023, 1024, 1025, 4096, 4097, 8192, 8193, 16384, 16385, 32769, 70001],
                                   90_000, 120_000, 9)),
        ("every_small_degree", synth.hubs(list(range(1, 301)), 3000, 4000, 17)),
        ("rmat_s14", synth.rmat(14, 16, seed=5)),
        ("chunglu_20k", synth.chung_lu(20000, 150000, 2.2, 800.0, 5)),
    ]


GRAPHS = _graphs()


@pytest.mark.parametrize("name,graph", GRAPHS, ids=[g[0] for g in GRAPHS])
def test_adjacency_matches_oracle_csr(name, graph):
    _say("adjacent", name)
    off, col = graph
    og = oracle.Graph(off, col)
    n = og.n
    deg = np.diff(og.off)
    row = np.repeat(np.arange(n, dtype=np.int64), deg)
    keys = np.sort(row * n + og.col.astype(np.int64))  # relabelled (a, b) of every slot
    rng = np.random.default_rng(11)
    # every slot as a pair (both orders appear), random pairs, and pairs
    # within the largest rows' neighbourhoods (mostly non-adjacent hubs)
    a = [row, rng.integers(0, n, 200_000)]
    b = [og.col.astype(np.int64), rng.integers(0, n, 200_000)]
    top = np.argsort(deg)[-50:]
    pa, pb = np.meshgrid(top, top)
    a.append(pa.ravel())
    b.append(pb.ravel())
    a = np.concatenate(a)
    b = np.concatenate(b)
    keep = a != b
    a, b = a[keep], b[keep]
    want = np.isin(a * n + b, keys)
    assert want.any() and (name == "K9" or not want.all())  # K9: every pair is an edge
    g = ps.Graph(torch.from_numpy(np.ascontiguousarray(off, np.int64)).cuda(),
                 torch.from_numpy(np.ascontiguousarray(col, np.int32)).cuda())
    ta = torch.from_numpy(a.astype(np.int32)).cuda()
    tb = torch.from_numpy(b.astype(np.int32)).cuda()
    for mode in MODES:
        got = g.adjacent(ta, tb, mode).cpu().numpy().astype(bool)
        bad = np.flatnonzero(got != want)
        assert bad.size == 0, (name, mode, bad[:5], a[bad[:5]], b[bad[:5]])
    g.destroy()


def test_adjacent_argument_errors():
    off, col = synth.complete(5)
    g = ps.Graph(torch.from_numpy(off).cuda(), torch.from_numpy(col).cuda())
    t = torch.zeros(4, dtype=torch.int32, device="cuda")
    with pytest.raises(ps.PathSampError) as e:
        g.adjacent(t, t + 1, mode=7)
    assert e.value.status == ps.PM_EINVAL
    empty = torch.zeros(0, dtype=torch.int32, device="cuda")
    assert g.adjacent(empty, empty).numel() == 0
    g.destroy()
