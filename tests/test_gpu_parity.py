"""GPU parity: the HIP path against the oracle, element by element.

Prepared arrays (relabelled CSR, rank, tau/lambda prefixes, W, Lambda, N_1)
and per-pattern sample tallies must be bit-exact; estimates within 1e-12
relative, bars within 1e-9 (both computed on the host from identical
integers).  Inputs are seeded synthetic graphs; every case prints its name
before touching the GPU.
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import finalize as ofin
from paper_1411_4942_amd import pathsamp as ps
from paper_1411_4942_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def _dev(off, col):
    return (torch.from_numpy(np.ascontiguousarray(off, np.int64)).cuda(),
            torch.from_numpy(np.ascontiguousarray(col, np.int32)).cuda())


def _graphs():
    gs = [
        ("K6", synth.complete(6)),
        ("K12", synth.complete(12)),
        ("C9", synth.cycle(9)),
        ("C4", synth.cycle(4)),
        ("star7", synth.star(7)),
        ("K3,3", synth.complete_bipartite(3, 3)),
        ("K2,40", synth.complete_bipartite(2, 40)),
        ("P8", synth.path(8)),
        ("matching", synth.csr_from_edges(12, [0, 2, 4, 6], [1, 3, 5, 7])),
        ("empty5", synth.empty(5)),
        ("single_vertex", synth.empty(1)),
    ]
    for seed in range(40):
        rng = np.random.default_rng(seed)
        n = int(rng.integers(5, 40))
        m = int(rng.integers(n - 1, min(n * (n - 1) // 2, 4 * n) + 1))
        gs.append((f"gnm{seed}", synth.erdos_renyi(n, m, seed)))
    gs.append(("chunglu_3k", synth.chung_lu(3000, 20000, 2.2, 300.0, 3)))
    gs.append(("rmat_s12", synth.rmat(12, 16, seed=2)))
    gs.append(("er_tiles", synth.erdos_renyi(9000, 70000, 4)))  # > several scan/radix tiles, ragged tail
    # rows on both sides of every row-build size-class bound (16 .. 32768) and
    # above it (the global hub sort)
    gs.append(("hub_classes", synth.hubs([16, 17, 64, 65, 128, 129, 256, 257, 1024, 1025, 4096, 4097, 8192, 8193, 16384,
                                          16385, 32768, 32769, 70001], 100000, 150000, 9)))
    # rows of every length from 1 to 300: each padding of the lane, wave and
    # register networks (classes up to 16, 64, 128 and 256) and the first
    # block sizes above them
    gs.append(("every_small_degree", synth.hubs(list(range(1, 301)), 3000, 4000, 17)))
    return gs


GRAPHS = _graphs()


def _check_prep(name, off, col):
    og = oracle.Graph(off, col)
    g = ps.Graph(*_dev(off, col))
    info = g.info()
    ex = g.export()
    assert info["n"] == og.n and 2 * info["m"] == og.slots, name
    assert np.array_equal(ex["off"], og.off), name
    assert np.array_equal(ex["col"], og.col), name
    assert np.array_equal(ex["rank"], og.rank), name
    assert np.array_equal(ex["p_tau"], og.p_tau), name
    assert np.array_equal(ex["p_lam"], og.p_lam), name
    assert info["W"] * 2 == og.R_tau and info["Lambda"] * 2 == og.R_lam and info["N1"] == og.N1, name
    deg = np.diff(off)
    assert info["dmax"] == (int(deg.max()) if deg.size else 0)
    assert info["isolated"] == int((deg == 0).sum())
    return og, g


@pytest.mark.parametrize("name,graph", GRAPHS, ids=[g[0] for g in GRAPHS])
def test_prep_and_tallies_bit_exact(name, graph):
    _say("prep+tallies", name)
    off, col = graph
    og, g = _check_prep(name, off, col)
    try:
        # every way of running the adjacency tests (the row hash is the
        # default)
        for mode in (ps.SEARCH_HASH, ps.SEARCH_LANE, ps.SEARCH_WAVE):
            ps.set_search_mode(mode)
            for seed, kp, kc, fp, fc in [(1, 20000, 20000, 0, 0), (0xDEADBEEFCAFEF00D, 777, 1234, 5, 2 ** 33 + 7)]:
                got = g.count(kp, kc, seed=seed, first_path=fp, first_cent=fc)
                assert got["tally_path"] == og.sample_path(seed, kp, fp).tolist(), (name, seed, mode)
                assert got["tally_cent"] == og.sample_centered(seed, kc, fc).tolist(), (name, seed, mode)
                want = ofin.finalize(got["tally_path"], got["tally_cent"], og.R_tau, og.R_lam, og.N1, kp, kc)
                for i in range(1, 7):
                    assert got["est"][i] == pytest.approx(want["est"][i], rel=1e-12, abs=1e-9)
                    assert got["est_basic"][i] == pytest.approx(want["est_basic"][i], rel=1e-12, abs=1e-9)
    finally:
        ps.set_search_mode(ps.SEARCH_HASH)
    with pytest.raises(ps.PathSampError):
        ps.set_search_mode(3)
    g.destroy()


def test_enumeration_exactness_on_device():
    """With k = R (whole range of r realised by many ids) the sampled tallies
    are multinomial, but the GPU and oracle still agree id by id."""
    off, col = synth.complete(7)
    og = oracle.Graph(off, col)
    g = ps.Graph(*_dev(off, col))
    got = g.count(100000, 100000, seed=3)
    assert got["tally_path"][0] + got["tally_path"][6] == 100000
    assert got["tally_path"] == og.sample_path(3, 100000).tolist()


def test_config1_er_2000_20000():
    """ER G(2000, 20000), k = 1e5 per sampler, Philox seed 1, in the launch
    configuration the benchmark uses (pm_count)."""
    _say("config1")
    off, col = synth.erdos_renyi(2000, 20000, 1)
    og, g = _check_prep("config1", off, col)
    got = g.count(100_000, 100_000, seed=1)
    tp = og.sample_path(1, 100_000).tolist()
    tc = og.sample_centered(1, 100_000).tolist()
    assert got["tally_path"] == tp and got["tally_cent"] == tc
    want = ofin.finalize(tp, tc, og.R_tau, og.R_lam, og.N1, 100_000, 100_000)
    for i in range(1, 7):
        assert got["est"][i] == pytest.approx(want["est"][i], rel=1e-12, abs=1e-9)
        for key in ("lo", "hi"):
            assert got[key][i] == pytest.approx(want[key][i], rel=1e-9, abs=1e-6)
    C, _ = oracle.exact_formula(off, col)
    for i in (1, 2):
        assert abs(got["est"][i] - C[i]) <= 0.01 * C[i]
    for i in range(1, 7):
        assert got["lo"][i] - 1e-6 <= C[i] <= got["hi"][i] + 1e-6


def test_count_motifs_one_shot_host_and_device_inputs():
    off, col = synth.erdos_renyi(2000, 20000, 1)
    a = ps.count_motifs(off, col, k=50_000, seed=9)       # host buffers
    b = ps.count_motifs(*_dev(off, col), k=50_000, seed=9)  # device buffers
    assert a == b
    og = oracle.Graph(off, col)
    assert a["tally_path"] == og.sample_path(9, 50_000).tolist()
    assert a["tally_cent"] == og.sample_centered(9, 50_000).tolist()


def test_id_ranges_concatenate_on_device():
    off, col = synth.chung_lu(5000, 40000, 2.3, 200.0, 11)
    g = ps.Graph(*_dev(off, col))
    full = g.count(300_000, 300_000, seed=5)
    a = g.count(100_000, 50_000, seed=5)
    b = g.count(200_000, 250_000, seed=5, first_path=100_000, first_cent=50_000)
    assert full["tally_path"] == [x + y for x, y in zip(a["tally_path"], b["tally_path"])]
    assert full["tally_cent"] == [x + y for x, y in zip(a["tally_cent"], b["tally_cent"])]


def test_sample_async_into_tensor():
    off, col = synth.erdos_renyi(500, 3000, 2)
    og = oracle.Graph(off, col)
    g = ps.Graph(*_dev(off, col))
    t = torch.full((16,), 12345, dtype=torch.int64, device="cuda")
    g.sample_async(t, 4000, 3000, seed=77)
    torch.cuda.synchronize()
    got = t.cpu().numpy().astype(np.uint64)
    assert got[:8].tolist() == og.sample_path(77, 4000).tolist()
    assert got[8:].tolist() == og.sample_centered(77, 3000).tolist()


def test_philox_device_matches_oracle():
    rng = np.random.default_rng(99)
    rows = rng.integers(0, 2 ** 32, size=(512, 6), dtype=np.uint64).astype(np.uint32)
    got = ps.philox_device(rows)
    for r, o in zip(rows, got):
        assert o.tolist() == oracle.philox4x32_10(r[:4], r[4:]).tolist()


def _bad_graphs():
    off, col = synth.complete(5)
    out = []
    c = col.copy()
    c[0], c[1] = c[1], c[0]
    out.append(("unsorted", off, c, ps.PM_EGRAPH))
    c = col.copy()
    c[1] = c[0]
    out.append(("duplicate", off, c, ps.PM_EGRAPH))
    c = col.copy()
    c[0] = 0
    out.append(("self_loop", off, c, ps.PM_EGRAPH))
    c = col.copy()
    c[-1] = 77
    out.append(("out_of_range", off, c, ps.PM_EGRAPH))
    c = col.copy()
    c[-1] = -3
    out.append(("negative", off, c, ps.PM_EGRAPH))
    out.append(("asymmetric", np.array([0, 1, 2, 3], np.int64), np.array([1, 2, 1], np.int32), ps.PM_EGRAPH))
    # a directed 3-cycle: in-degree equals out-degree everywhere, still not symmetric
    out.append(("directed_cycle", np.array([0, 1, 2, 3], np.int64), np.array([1, 2, 0], np.int32), ps.PM_EGRAPH))
    o = off.copy()
    o[2] = o[3] + 1
    out.append(("offsets_decrease", o, col, ps.PM_EGRAPH))
    o = off.copy()
    o[0] = 1
    out.append(("offsets_not_zero", o, col, ps.PM_EGRAPH))
    return out


@pytest.mark.parametrize("name,off,col,status", _bad_graphs(), ids=[b[0] for b in _bad_graphs()])
def test_invalid_graphs_are_rejected(name, off, col, status):
    _say("invalid", name)
    assert oracle.validate(off, col) != oracle.OK
    with pytest.raises(ps.PathSampError) as e:
        ps.Graph(*_dev(off, col))
    assert e.value.status == status


def _run_starts(d):
    """Input positions inside a row of degree d where the row kernel takes a
    slot's predecessor from somewhere other than the register or lane just
    below.  Up to 16 one lane holds the whole row; up to 256 slot e is
    register e % I of lane e // I (I = 1, 2 or 4 keys per lane), so lane
    starts; above, wave w of a W-wave block owns slots [w per, (w + 1) per),
    per = ceil(d / 64W) 64, item i of it the 64 slots from w per + 64 i, so
    item and run starts.  Above 32768 the row is sorted in chunks of 32768
    slots, so chunk starts.  Plus the last slot."""
    bounds = [16, 64, 128, 256, 1024, 4096, 8192, 16384, 32768]
    waves = [0, 0, 0, 0, 1, 4, 8, 16, 16]  # lane and wave networks, then a block per row
    pos = {1, 2, 3, 4, 5, 64, 128, d - 1}
    if d > 32768:
        return sorted(pos | set(range(32768, d, 32768)) | {32769})
    W = next(w for b, w in zip(bounds, waves) if d <= b)
    if W:
        per = -(-d // (64 * W)) * 64
        runs = [w * per for w in range(1, W) if w * per < d]
        pos |= set(runs[:1] + runs[-1:]) | {r + 64 for r in runs[-1:]}
    return sorted(j for j in pos if 1 <= j < d)


def test_row_checks_in_every_size_class():
    """Planted input errors in rows of every size class are reported: an
    unsorted pair and a repeated column at each place where the row kernel
    gets a slot's predecessor from another item, wave or the run before, a
    self-loop, an out-of-range and a negative column."""
    degrees = [10, 50, 100, 200, 700, 3000, 6000, 12000, 20000, 40000]
    off, col = synth.hubs(degrees, 45000, 30000, 13)
    n = len(off) - 1
    g = ps.Graph(*_dev(off, col))  # the clean graph builds
    g.destroy()
    texts = {"order": "not strictly ascending", "loop": "self-loop", "range": "not a vertex id"}
    for u, d in enumerate(degrees):
        a = int(off[u])
        plants = []
        for j in _run_starts(d):
            c = col.copy()
            c[a + j - 1], c[a + j] = c[a + j], c[a + j - 1]
            plants.append(("swap", j, c, "order"))
            c = col.copy()
            c[a + j] = c[a + j - 1]
            plants.append(("repeat", j, c, "order"))
        c = col.copy()
        c[a + d // 2] = u
        plants.append(("loop", d // 2, c, "loop"))
        c = col.copy()
        c[a + d - 1] = n + 3
        plants.append(("range", d - 1, c, "range"))
        c = col.copy()
        c[a] = -3
        plants.append(("negative", 0, c, "range"))
        for kind, j, c, want in plants:
            _say("row check", d, kind, j)
            assert oracle.validate(off, c) != oracle.OK
            with pytest.raises(ps.PathSampError) as e:
                ps.Graph(*_dev(off, c))
            assert e.value.status == ps.PM_EGRAPH, (d, kind, j)
            assert texts[want] in str(e.value), (d, kind, j, str(e.value))


def test_argument_errors():
    off, col = synth.complete(5)
    g = ps.Graph(*_dev(off, col))
    with pytest.raises(ps.PathSampError) as e:
        g.count(0, 0)
    assert e.value.status == ps.PM_EINVAL
    with pytest.raises(ps.PathSampError) as e:
        g.count(10, 10, delta=0.0)
    assert e.value.status == ps.PM_EINVAL
    with pytest.raises(ps.PathSampError) as e:
        ps.count_motifs(off, col, k=0)
    assert e.value.status == ps.PM_EINVAL


def test_n1_overflow_is_reported():
    leaves = 5_300_000
    off, col = synth.star(leaves)
    with pytest.raises(ps.PathSampError) as e:
        ps.Graph(*_dev(off, col))
    assert e.value.status == ps.PM_EOVERFLOW


def test_zero_weight_samplers_are_exact_zero():
    for name, (off, col) in [("star", synth.star(30)), ("matching", synth.csr_from_edges(6, [0, 2], [1, 3])),
                             ("path", synth.path(30))]:
        _say("zero-weight", name)
        og = oracle.Graph(off, col)
        r = ps.count_motifs(off, col, k=1000, seed=1)
        C, _ = oracle.exact_formula(off, col)
        if og.R_tau == 0:
            assert r["tally_path"] == [0] * 8
            assert r["est"][2:4] == [0.0, 0.0]
            assert r["est"][1] == C[1]
        if og.R_lam == 0:
            assert r["tally_cent"] == [0] * 8
            assert r["est"][4:] == [0.0, 0.0, 0.0]


@pytest.mark.parametrize("shape", [(1, 1), (1, 8), (2, 8), (2, 64), (4, 3), (4, 16)])
def test_sampler_launch_shape_does_not_change_tallies(shape):
    """Samples are a function of (seed, tag, id) only: every launch shape of
    the sampling kernels gives the oracle's tallies."""
    _say("shape", shape)
    off, col = synth.chung_lu(20000, 150000, 2.2, 800.0, 5)
    og = oracle.Graph(off, col)
    g = ps.Graph(*_dev(off, col))
    try:
        ps.set_sampler_shape(*shape)
        got = g.count(123_457, 98_765, seed=2024, first_path=17, first_cent=5)
    finally:
        ps.set_sampler_shape(1, 4)
    assert got["tally_path"] == og.sample_path(2024, 123_457, 17).tolist()
    assert got["tally_cent"] == og.sample_centered(2024, 98_765, 5).tolist()
    with pytest.raises(ps.PathSampError):
        ps.set_sampler_shape(3, 8)


def test_cached_device_memory_reuse_across_streams():
    """Graphs created and destroyed repeatedly on two streams reuse cached
    device blocks; every count stays equal to the oracle's."""
    _say("allocator reuse")
    off1, col1 = synth.chung_lu(6000, 50000, 2.3, 300.0, 21)
    off2, col2 = synth.erdos_renyi(3000, 30000, 22)
    o1, o2 = oracle.Graph(off1, col1), oracle.Graph(off2, col2)
    want1 = (o1.sample_path(3, 50_000).tolist(), o1.sample_centered(3, 50_000).tolist())
    want2 = (o2.sample_path(4, 50_000).tolist(), o2.sample_centered(4, 50_000).tolist())
    d1, d2 = _dev(off1, col1), _dev(off2, col2)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    for it in range(4):
        with torch.cuda.stream(s1):
            g1 = ps.Graph(*d1, stream=s1)
            r1 = g1.count(50_000, 50_000, seed=3, stream=s1)
        with torch.cuda.stream(s2):
            g2 = ps.Graph(*d2, stream=s2)
            r2 = g2.count(50_000, 50_000, seed=4, stream=s2)
        assert (r1["tally_path"], r1["tally_cent"]) == want1, it
        assert (r2["tally_path"], r2["tally_cent"]) == want2, it
        g1.destroy()
        g2.destroy()
        if it == 2:
            torch.cuda.synchronize()
            ps.release_cached_memory()


def test_draw_order_does_not_change_tallies():
    """Draw-ordered sampling (large k) gives the id-order tallies exactly:
    against the oracle above the threshold, and on against off across
    several sort chunks."""
    _say("draw order")
    off, col = synth.chung_lu(20000, 150000, 2.2, 800.0, 5)
    og = oracle.Graph(off, col)
    g = ps.Graph(*_dev(off, col))
    k = (1 << 20) + 12345
    try:
        ps.set_draw_order(True, 1 << 20)
        a = g.count(k, k, seed=3, first_path=7, first_cent=2 ** 33)
        assert a["tally_path"] == og.sample_path(3, k, 7).tolist()
        assert a["tally_cent"] == og.sample_centered(3, k, 2 ** 33).tolist()
        # one sampler draw-ordered, the other below the threshold (the two are
        # then launched in turn instead of with their sorts side by side)
        mixed = g.count(k, 5000, seed=3, first_path=7, first_cent=2 ** 33)
        assert mixed["tally_path"] == a["tally_path"]
        assert mixed["tally_cent"] == og.sample_centered(3, 5000, 2 ** 33).tolist()
        for mode in (ps.SEARCH_LANE, ps.SEARCH_WAVE):  # the sorted-row searches over draw-ordered ids
            ps.set_search_mode(mode)
            a2 = g.count(k, k, seed=3, first_path=7, first_cent=2 ** 33)
            assert a2["tally_path"] == a["tally_path"] and a2["tally_cent"] == a["tally_cent"], mode
        ps.set_search_mode(ps.SEARCH_HASH)
        k2 = (1 << 24) * 2 + 777  # three sort chunks, the last one ragged
        on = g.count(k2, k2, seed=9)
        ps.set_draw_order(False)
        b = g.count(k, k, seed=3, first_path=7, first_cent=2 ** 33)
        off_ = g.count(k2, k2, seed=9)
    finally:
        ps.set_draw_order(True, 0)
        ps.set_search_mode(ps.SEARCH_HASH)
    assert a["tally_path"] == b["tally_path"] and a["tally_cent"] == b["tally_cent"]
    assert on["tally_path"] == off_["tally_path"] and on["tally_cent"] == off_["tally_cent"]
    g.destroy()


def test_profile_select_restricts_recording():
    """With a selection only the named scopes are timed; with none, every
    scope of a graph build and a count is."""
    off, col = synth.chung_lu(3000, 20000, 2.2, 300.0, 3)
    try:
        ps.profile_select(["sample_path", "degrees"])
        ps.profile_enable(True)
        g = ps.Graph(*_dev(off, col))
        g.count(5000, 5000, seed=1)
        g.destroy()
        got = ps.profile_read()
        assert set(got) == {"sample_path", "degrees"}, got
        assert got["sample_path"][0] == 1 and got["degrees"][0] == 1
        ps.profile_select(None)
        ps.profile_enable(True)  # clears the totals
        g = ps.Graph(*_dev(off, col))
        g.count(5000, 5000, seed=1)
        g.destroy()
        got = ps.profile_read()
        assert {"sample_path", "sample_centered", "degrees", "build_rows", "reverse_sort.scatter"} <= set(got), got
    finally:
        ps.profile_enable(False)
        ps.profile_select(None)


def test_large_asymmetric_graph_is_rejected():
    """A directed random graph (rows sorted, no loops, no repeats, but not
    symmetric) spanning many tiles and prefix segments: the build reports the
    asymmetry; the inconsistent weights it leaves fill no guide table."""
    rng = np.random.default_rng(21)
    n, m = 50_000, 400_000
    u = rng.integers(0, n, size=m)
    v = rng.integers(0, n, size=m)
    keep = u != v
    key = np.unique(u[keep].astype(np.int64) * n + v[keep])
    src, dst = key // n, key % n
    off = np.zeros(n + 1, np.int64)
    np.add.at(off, src + 1, 1)
    off = np.cumsum(off)
    col = dst.astype(np.int32)
    _say("large asymmetric", len(col))
    assert oracle.validate(off, col) != oracle.OK
    with pytest.raises(ps.PathSampError) as e:
        ps.Graph(*_dev(off, col))
    assert e.value.status == ps.PM_EGRAPH
    assert "not symmetric" in str(e.value)
