"""GPU parity at the full workload sizes, in the launch configuration the
benchmark times (Graph create + pm_count with the default sampler shape).

* Chung-Lu n = 1e6, m = 1e7, exponent 2.3, weight cap 5000, generator seed 1,
  k = 2e6 + 2e6, Philox seed 1: every prepared array and both tallies
  bit-exact against the oracle run on the same CSR.
* R-MAT scale 22 (0.57, 0.19, 0.19, 0.05), edge factor 31, seed 1, k = 1e7 +
  1e7, Philox seed 1 (the benchmark's graph): the oracle prepares the same
  input CSR itself (relabel, tau and lambda prefixes of Sections 3 and 4,
  N_1; about a minute on one core), every exported array must equal its
  own, and its own samplers then run over every id of the full-size launch
  (id windows on host threads; tallies are sums over ids).  Nothing the
  device produced is an input of the oracle.
"""
import sys
import time

import numpy as np
import pytest

import oracle
import oracle_windows
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


@pytest.mark.timeout(1200)
def test_rmat22_oracle_prep_and_full_tallies():
    t0 = time.time()
    _say("rmat22: generate")
    off_d, col_d = synth.rmat_torch(22, 31.0, seed=1, device="cuda")
    k = 10_000_000
    _say("rmat22: device prep + count", f"{time.time() - t0:.1f}s")
    g = ps.Graph(off_d, col_d)
    full = g.count(k, k, seed=1)
    ex = g.export()
    info = g.info()
    g.destroy()
    off, col = off_d.cpu().numpy(), col_d.cpu().numpy()
    del off_d, col_d
    torch.cuda.empty_cache()
    assert off[-1] == 242_921_518

    _say("rmat22: oracle preparation of", int(off[-1]), "slots", f"{time.time() - t0:.1f}s")
    og = oracle.Graph(off, col)
    del off, col
    _say("rmat22: compare prepared arrays", f"{time.time() - t0:.1f}s")
    assert np.array_equal(ex["rank"], og.rank)
    assert np.array_equal(ex["off"], og.off)
    assert np.array_equal(ex["col"], og.col)
    assert np.array_equal(ex["p_tau"], og.p_tau)
    assert np.array_equal(ex["p_lam"], og.p_lam)
    assert (2 * info["W"], 2 * info["Lambda"], info["N1"]) == (og.R_tau, og.R_lam, og.N1)
    assert info["n"] == og.n and 2 * info["m"] == og.slots
    del ex

    _say("rmat22: oracle 3-path sampler over", k, "ids", f"{time.time() - t0:.1f}s")
    tp = oracle_windows.tally(og._g, False, 1, k)
    assert full["tally_path"] == tp
    _say("rmat22: oracle centered sampler over", k, "ids", f"{time.time() - t0:.1f}s")
    tc = oracle_windows.tally(og._g, True, 1, k)
    assert full["tally_cent"] == tc
    want = ofin.finalize(tp, tc, og.R_tau, og.R_lam, og.N1, k, k)
    for i in range(1, 7):
        assert full["est"][i] == pytest.approx(want["est"][i], rel=1e-12, abs=1e-9)
        for key in ("lo", "hi"):
            assert full[key][i] == pytest.approx(want[key][i], rel=1e-9, abs=1e-6)
    _say("rmat22: done", f"{time.time() - t0:.1f}s")
