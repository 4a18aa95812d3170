"""GPU parity of the alias-table edge draw (pm_graph_build_alias,
pm_count_alias) against the oracle's alias mode (oracle/alias.c).

* tables: both samplers' (K, alias) bit-exact on graphs spanning many merge
  tiles and a ragged tail (up to R-MAT scale 18, 2m ~ 7.6e6), plus the exact
  mass identity on the largest (mod 2^64 over every slot);
* tallies: bit-exact against the oracle's alias samplers for several seeds,
  sample counts and first ids;
* R-MAT scale 22 (the benchmark graph): alias estimates agree with the main
  draw's within the two 99% bars, all six motifs;
* degenerate and error cases: a zero-weight sampler has no table and zero
  tallies; counting or exporting without tables is PM_EINVAL; a second build
  is a no-op.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1411_4942_amd import pathsamp as ps
from paper_1411_4942_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def _dev(off, col):
    return (torch.from_numpy(np.ascontiguousarray(off, np.int64)).cuda(),
            torch.from_numpy(np.ascontiguousarray(col, np.int32)).cuda())


GRAPHS = [
    ("K6", lambda: synth.complete(6)),
    ("K3,3", lambda: synth.complete_bipartite(3, 3)),
    ("C9", lambda: synth.cycle(9)),
    ("gnm7", lambda: synth.erdos_renyi(30, 90, 7)),
    ("chunglu_3k", lambda: synth.chung_lu(3000, 20000, 2.2, 300.0, 3)),
    ("rmat_s12", lambda: synth.rmat(12, 16, seed=2)),
    ("er_tiles", lambda: synth.erdos_renyi(9000, 70000, 4)),
    ("hub_classes", lambda: synth.hubs([16, 17, 64, 65, 128, 129, 256, 257, 1024, 1025, 4096, 4097, 8192, 8193, 16384,
                                        16385, 32768, 32769, 70001], 100000, 150000, 9)),
]


@pytest.mark.parametrize("name,make", GRAPHS, ids=[g[0] for g in GRAPHS])
def test_alias_tables_and_tallies_bit_exact(name, make):
    _say("alias tables+tallies", name)
    off, col = make()
    og = oracle.Graph(off, col)
    g = ps.Graph(*_dev(off, col))
    g.build_alias()
    for centered, R in ((False, og.R_tau), (True, og.R_lam)):
        if R == 0:
            continue
        K, A = g.alias_export(centered)
        oK, oA = og.alias_table(centered)
        assert np.array_equal(K, oK), (name, centered)
        assert np.array_equal(A, oA), (name, centered)
    for seed, kp, kc, fp, fc in [(1, 20000, 20000, 0, 0), (0xDEADBEEFCAFEF00D, 777, 1234, 5, 2 ** 33 + 7)]:
        got = g.count_alias(kp, kc, seed=seed, first_path=fp, first_cent=fc)
        assert got["tally_path"] == og.sample_path_alias(seed, kp, fp).tolist(), (name, seed)
        assert got["tally_cent"] == og.sample_centered_alias(seed, kc, fc).tolist(), (name, seed)
    g.destroy()


def test_alias_tables_rmat18():
    """Many merge tiles (2m ~ 7.6e6 / 4096 per tile): tables bit-exact, the
    exact mass identity mod 2^64, and sampled tallies bit-exact."""
    _say("alias rmat s18")
    off, col = synth.rmat(18, 16, seed=3)
    og = oracle.Graph(off, col)
    g = ps.Graph(*_dev(off, col))
    g.build_alias()
    N = og.slots
    for centered, R in ((False, og.R_tau), (True, og.R_lam)):
        K, A = g.alias_export(centered)
        oK, oA = og.alias_table(centered)
        assert np.array_equal(K, oK) and np.array_equal(A, oA), centered
        w = og.weights(centered)
        # slot s owns N w_s: its own kept part plus R - K_b of every bucket aliasing it (mod 2^64)
        give = np.where(K < np.uint64(R), np.uint64(R) - K, np.uint64(0))
        order = np.argsort(A, kind="stable")
        a_sorted = A[order]
        starts = np.flatnonzero(np.r_[True, a_sorted[1:] != a_sorted[:-1]])
        recv = np.zeros(N, np.uint64)
        recv[a_sorted[starts]] = np.add.reduceat(give[order], starts)
        with np.errstate(over="ignore"):
            assert np.array_equal(K + recv, w * np.uint64(N)), centered  # a full bucket gives nothing
    got = g.count_alias(30000, 30000, seed=5)
    assert got["tally_path"] == og.sample_path_alias(5, 30000).tolist()
    assert got["tally_cent"] == og.sample_centered_alias(5, 30000).tolist()
    g.destroy()


def test_alias_degenerate_and_errors():
    _say("alias degenerate")
    off, col = synth.path(8)  # W > 0, Lambda = 0: no 3-path of a path graph is centered
    og = oracle.Graph(off, col)
    assert og.R_lam == 0 and og.R_tau > 0
    g = ps.Graph(*_dev(off, col))
    with pytest.raises(ps.PathSampError) as e:
        g.count_alias(100, 100)
    assert e.value.status == ps.PM_EINVAL
    with pytest.raises(ps.PathSampError):
        g.alias_export(False)
    bytes0 = g.info()["device_bytes"]
    g.build_alias()
    assert g.info()["device_bytes"] == bytes0 + 32 * og.slots  # one table: tau only
    g.build_alias()  # no-op
    assert g.info()["device_bytes"] == bytes0 + 32 * og.slots
    with pytest.raises(ps.PathSampError):
        g.alias_export(True)
    got = g.count_alias(5000, 5000, seed=2)
    assert got["tally_path"] == og.sample_path_alias(2, 5000).tolist()
    assert got["tally_cent"] == [0] * ps.NUM_TALLIES
    g.destroy()


def test_alias_full_size_agrees_with_main_draw():
    """R-MAT scale 22 (the benchmark graph): both draws estimate the same
    counts; each motif's two estimates lie within the sum of their 99% bar
    half-widths."""
    _say("alias full size rmat s22")
    off, col = synth.rmat_torch(22, 31.0, seed=1)
    g = ps.Graph(off, col)
    del off, col
    g.build_alias()
    k = 10_000_000
    a = g.count_alias(k, k, seed=1)
    m = g.count(k, k, seed=1)
    for i in range(1, 7):
        half = (a["hi"][i] - a["lo"][i]) / 2 + (m["hi"][i] - m["lo"][i]) / 2
        assert abs(a["est"][i] - m["est"][i]) <= half, (i, a["est"][i], m["est"][i], half)
    g.destroy()
    torch.cuda.empty_cache()


def test_alias_draw_order_does_not_change_tallies():
    """Draw-ordered alias sampling (ids sorted by their bucket) gives the
    id-order tallies: against the oracle above the threshold, on against off."""
    _say("alias draw order")
    off, col = synth.chung_lu(20000, 150000, 2.2, 800.0, 5)
    og = oracle.Graph(off, col)
    g = ps.Graph(*_dev(off, col))
    g.build_alias()
    k = (1 << 20) + 4321
    try:
        ps.set_draw_order(True, 1 << 20)
        a = g.count_alias(k, k, seed=4, first_path=11, first_cent=2 ** 34)
        ps.set_draw_order(False)
        b = g.count_alias(k, k, seed=4, first_path=11, first_cent=2 ** 34)
    finally:
        ps.set_draw_order(True, 0)
    assert a["tally_path"] == b["tally_path"] and a["tally_cent"] == b["tally_cent"]
    assert a["tally_path"] == og.sample_path_alias(4, k, 11).tolist()
    assert a["tally_cent"] == og.sample_centered_alias(4, k, 2 ** 34).tolist()
    g.destroy()
