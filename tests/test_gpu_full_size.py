"""GPU parity at the full workload sizes, in the launch configuration the
benchmark times (Graph create + pm_count with the default sampler shape).

* Chung-Lu n = 1e6, m = 1e7, exponent 2.3, weight cap 5000, generator seed 1,
  k = 2e6 + 2e6, Philox seed 1: every prepared array and both tallies
  bit-exact against the oracle run on the same CSR.
* R-MAT scale 22 (0.57, 0.19, 0.19, 0.05), edge factor 31, seed 1, k = 1e7 +
  1e7, Philox seed 1 (the benchmark's graph): the oracle's own preparation is
  too slow here, so the device's prepared arrays are checked against their
  definitions (degree order, edge multiset, sorted rows, every tau, lambda at
  sampled slots, N_1), and the oracle's samplers then run on those checked
  arrays over every id of the full-size launch.
"""
import ctypes
import sys
import time

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


def test_chunglu_1e6_1e7_bit_exact():
    t0 = time.time()
    _say("chung-lu 1e6/1e7: generate")
    off_d, col_d = synth.chung_lu_torch(1_000_000, 10_000_000, 2.3, 5000.0, 1, device="cuda")
    off, col = off_d.cpu().numpy(), col_d.cpu().numpy()
    assert off[-1] == 20_000_000
    _say("chung-lu: device prep + count", f"{time.time() - t0:.1f}s")
    g = ps.Graph(off_d, col_d)
    k = 2_000_000
    got = g.count(k, k, seed=1)
    ex = g.export()
    info = g.info()
    g.destroy()
    _say("chung-lu: oracle", f"{time.time() - t0:.1f}s")
    og = oracle.Graph(off, col)
    assert np.array_equal(ex["off"], og.off)
    assert np.array_equal(ex["rank"], og.rank)
    assert np.array_equal(ex["col"], og.col)
    assert np.array_equal(ex["p_tau"], og.p_tau)
    assert np.array_equal(ex["p_lam"], og.p_lam)
    assert (2 * info["W"], 2 * info["Lambda"], info["N1"]) == (og.R_tau, og.R_lam, og.N1)
    tp = og.sample_path(1, k).tolist()
    tc = og.sample_centered(1, k).tolist()
    assert got["tally_path"] == tp
    assert got["tally_cent"] == tc
    want = ofin.finalize(tp, tc, og.R_tau, og.R_lam, og.N1, k, k)
    for i in range(1, 7):
        assert got["est"][i] == pytest.approx(want["est"][i], rel=1e-12, abs=1e-9)
        for key in ("lo", "hi"):
            assert got[key][i] == pytest.approx(want[key][i], rel=1e-9, abs=1e-6)
    _say("chung-lu: done", f"{time.time() - t0:.1f}s")


def _oracle_on_arrays(off, col, p_tau, p_lam, N1):
    """The oracle's graph struct over already-checked prepared arrays (its
    samplers only read off, col and the prefixes)."""
    g = oracle._Graph()
    g.n = off.size - 1
    g.slots = col.size
    g.off = off.ctypes.data_as(type(g.off))
    g.col = col.ctypes.data_as(type(g.col))
    g.rank = ctypes.cast(None, type(g.rank))
    g.p_tau = p_tau.ctypes.data_as(type(g.p_tau))
    g.p_lam = p_lam.ctypes.data_as(type(g.p_lam))
    g.R_tau = int(p_tau[-1])
    g.R_lam = int(p_lam[-1])
    g.N1 = N1
    g._keep = (off, col, p_tau, p_lam)  # the struct points into these
    return g


def _oracle_tally(g, centered, seed, first, k):
    lib = oracle._load()
    t = (ctypes.c_uint64 * 8)()
    fn = lib.or_sample_centered if centered else lib.or_sample_path
    fn(ctypes.byref(g), ctypes.c_uint64(seed), ctypes.c_uint64(first), ctypes.c_uint64(k), t)
    return [int(x) for x in t]


def _parallel_oracle_tally(g, centered, seed, k, windows=64, workers=16):
    """Tallies of ids [0, k) as a sum over id windows, each window one
    single-threaded oracle call (ctypes releases the interpreter lock, so the
    windows run side by side)."""
    from concurrent.futures import ThreadPoolExecutor

    step = (k + windows - 1) // windows
    parts = [(f, min(step, k - f)) for f in range(0, k, step)]
    with ThreadPoolExecutor(max_workers=workers) as ex:
        outs = list(ex.map(lambda fw: _oracle_tally(g, centered, seed, fw[0], fw[1]), parts))
    return [sum(t[c] for t in outs) for c in range(8)]


def test_rmat22_checked_prep_and_full_tallies():
    t0 = time.time()
    _say("rmat22: generate")
    off_d, col_d = synth.rmat_torch(22, 31.0, seed=1, device="cuda")
    n = off_d.numel() - 1
    k = 10_000_000
    _say("rmat22: device prep + count", f"{time.time() - t0:.1f}s")
    g = ps.Graph(off_d, col_d)
    full = g.count(k, k, seed=1)
    ex = g.export()
    info = g.info()
    g.destroy()
    slots = int(off_d[-1].item())
    deg_in_d = off_d[1:] - off_d[:-1]
    # input edges relabelled, sorted on the device (a check, not the product path)
    rank_d = torch.from_numpy(ex["rank"].astype(np.int64)).cuda()
    src_d = torch.repeat_interleave(torch.arange(n, device="cuda"), deg_in_d)
    key_in = torch.sort((rank_d[src_d] << 32) | rank_d[col_d.long()]).values.cpu().numpy()
    deg_in = deg_in_d.cpu().numpy()
    del off_d, col_d, rank_d, src_d, deg_in_d
    torch.cuda.empty_cache()
    _say("rmat22: checks on", slots, "slots", f"{time.time() - t0:.1f}s")

    # degree order: rank is the stable order of (degree, input id)
    order = np.argsort(deg_in, kind="stable")
    assert np.array_equal(ex["rank"][order], np.arange(n, dtype=np.int32))
    off = ex["off"]
    assert off[0] == 0 and np.array_equal(np.diff(off), deg_in[order])
    deg = np.diff(off)
    col = ex["col"]
    row = np.repeat(np.arange(n, dtype=np.int64), deg)
    # rows strictly ascending, and the edge multiset is the input's, relabelled
    same_row = row[1:] == row[:-1]
    assert np.all(col[1:][same_row] > col[:-1][same_row])
    del same_row
    key_out = (row << 32) | col.astype(np.int64)
    assert np.array_equal(key_in, key_out)
    del key_in
    _say("rmat22: relabel checked", f"{time.time() - t0:.1f}s")

    # every tau; lambda at sampled slots; N_1
    tau = (deg[row].astype(np.uint64) - 1) * (deg[col].astype(np.uint64) - 1)
    p_tau = ex["p_tau"]
    assert p_tau[0] == tau[0] and np.array_equal(np.diff(p_tau), tau[1:])
    assert int(p_tau[-1]) == 2 * info["W"]
    del tau
    rng = np.random.default_rng(22)
    s = np.unique(np.concatenate([rng.integers(0, slots, 200_000), [0, slots - 1]]))
    u = row[s]
    v = col[s].astype(np.int64)
    j = s - off[u]
    r = np.searchsorted(key_out, (v << 32) | u)  # slot of (v, u)
    assert np.array_equal(key_out[r], (v << 32) | u)
    lam = (deg[u] - 1 - j).astype(np.uint64) * (deg[v] - 1 - (r - off[v])).astype(np.uint64)
    p_lam = ex["p_lam"]
    prev = np.where(s > 0, p_lam[np.maximum(s - 1, 0)], 0).astype(np.uint64)
    assert np.array_equal(p_lam[s] - prev, lam)
    assert np.all(p_lam[1:] >= p_lam[:-1])
    assert int(p_lam[-1]) == 2 * info["Lambda"]
    N1 = sum(int(d) * (int(d) - 1) * (int(d) - 2) // 6 for d in deg[deg >= 3])
    assert N1 == info["N1"]
    del row, key_out
    _say("rmat22: weights checked", f"{time.time() - t0:.1f}s")

    # the oracle's samplers on the checked arrays, over every id of the launch
    og = _oracle_on_arrays(np.ascontiguousarray(off), np.ascontiguousarray(col), np.ascontiguousarray(p_tau),
                           np.ascontiguousarray(p_lam), N1)
    tp = _parallel_oracle_tally(og, False, 1, k)
    assert full["tally_path"] == tp
    _say("rmat22: 3-path tallies equal", f"{time.time() - t0:.1f}s")
    tc = _parallel_oracle_tally(og, True, 1, k)
    assert full["tally_cent"] == tc
    want = ofin.finalize(tp, tc, 2 * info["W"], 2 * info["Lambda"], N1, k, k)
    for i in range(1, 7):
        assert full["est"][i] == pytest.approx(want["est"][i], rel=1e-12, abs=1e-9)
    _say("rmat22: done", f"{time.time() - t0:.1f}s")
