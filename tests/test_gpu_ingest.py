"""GPU parity of the edge-list ingest (pm_csr_from_edges, pm_graph_from_edges).

The CSR must equal the oracle's clean-up of the same pairs exactly; a graph
prepared straight from the edges must equal one prepared from that CSR, at
small sizes and on the benchmark's raw R-MAT scale-22 draws (2.6e8 pairs),
where an independent torch construction stands in for the oracle.
"""
import sys

import numpy as np
import pytest

from oracle import ingest
from paper_1411_4942_amd import pathsamp as ps
from paper_1411_4942_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def _lists():
    out = []
    rng = np.random.default_rng(5)
    for i in range(12):
        n = int(rng.integers(1, 5000))
        e = int(rng.integers(0, 40000))
        src = rng.integers(0, n, e).astype(np.int32)
        dst = rng.integers(0, n, e).astype(np.int32)
        if i % 3 == 0 and e:  # many repeats, both directions
            src = np.concatenate([src, dst, src])
            dst = np.concatenate([dst, src[: len(dst)], dst])
        out.append((f"random{i}", n, src, dst))
    k = np.arange(30, dtype=np.int32)
    out.append(("loops_only", 30, k, k))
    out.append(("empty", 7, np.zeros(0, np.int32), np.zeros(0, np.int32)))
    out.append(("isolated_tail", 100, np.array([0, 1, 2], np.int32), np.array([1, 2, 0], np.int32)))
    out.append(("one_vertex", 1, np.zeros(3, np.int32), np.zeros(3, np.int32)))
    out.append(("rmat_s12_raw", 1 << 12, *[t.cpu().numpy().astype(np.int32)
                                          for t in synth.rmat_edges_torch(12, 16, seed=3, device="cpu")]))
    return out


LISTS = _lists()


@pytest.mark.parametrize("name,n,src,dst", LISTS, ids=[x[0] for x in LISTS])
def test_csr_from_edges_equals_oracle(name, n, src, dst):
    _say("ingest", name)
    want_off, want_col = ingest.csr_from_edges(n, src, dst)
    for dev in (True, False):
        s = torch.from_numpy(src).cuda() if dev else src
        d = torch.from_numpy(dst).cuda() if dev else dst
        off, col = ps.csr_from_edges(n, s, d)
        assert np.array_equal(off.cpu().numpy(), want_off), (name, dev)
        assert np.array_equal(col.cpu().numpy(), want_col), (name, dev)


def test_graph_from_edges_equals_graph_from_csr():
    _say("graph_from_edges")
    n, src, dst = LISTS[1][1:]
    off, col = ingest.csr_from_edges(n, src, dst)
    a = ps.Graph.from_edges(n, torch.from_numpy(src).cuda(), torch.from_numpy(dst).cuda())
    b = ps.Graph(torch.from_numpy(off).cuda(), torch.from_numpy(col).cuda())
    assert a.info() == b.info()
    ea, eb = a.export(), b.export()
    for key in ea:
        assert np.array_equal(ea[key], eb[key]), key
    assert a.count(50_000, 50_000, seed=4) == b.count(50_000, 50_000, seed=4)
    a.destroy()
    b.destroy()


def test_errors():
    src = torch.tensor([0, 1, 5], dtype=torch.int32, device="cuda")
    dst = torch.tensor([1, 2, 0], dtype=torch.int32, device="cuda")
    with pytest.raises(ps.PathSampError) as e:
        ps.csr_from_edges(5, src, dst)  # 5 is not a vertex of a 5-vertex graph
    assert e.value.status == ps.PM_EGRAPH
    view, keep = ps._edge_view(3, np.array([0, 1], np.int32), np.array([1, 2], np.int32))
    off = torch.empty(4, dtype=torch.int64, device="cuda")
    col = torch.empty(3, dtype=torch.int32, device="cuda")
    slots = ps.ctypes.c_int64()
    st = ps.lib().pm_csr_from_edges(ps.ctypes.byref(view), off.data_ptr(), col.data_ptr(), 3, ps.ctypes.byref(slots),
                                    None)
    assert st == ps.PM_EINVAL  # needs 4 slots
    with pytest.raises(ps.PathSampError) as e:
        ps.Graph.from_edges(-1, np.zeros(0, np.int32), np.zeros(0, np.int32))
    assert e.value.status == ps.PM_EINVAL


def test_rmat22_raw_draws_full_size():
    """The benchmark graph's 1.3e8 raw draws: the ingest equals the torch
    construction (unique of min/max pairs, both directions, sorted) that
    builds the benchmark's CSR."""
    _say("ingest rmat22")
    u, v = synth.rmat_edges_torch(22, 31.0, seed=1, device="cuda")
    n = 1 << 22
    src, dst = u.to(torch.int32), v.to(torch.int32)
    del u, v
    off, col = ps.csr_from_edges(n, src, dst)
    want_off, want_col = synth._csr_from_edges_torch(n, src.long(), dst.long())
    assert torch.equal(off, want_off)
    assert torch.equal(col, want_col)
