"""GPU parity of the batched path (pm_batch_*, pm_count_batch).

Each graph's tallies from one persistent, graph-captured launch must equal
the oracle's for the same (seed, sampler, id range), bit for bit, whatever
the tile size and launch shape; replays of the captured graph, with eager
work and synchronisations between them, must all give the same result.
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


def _mix():
    """Graphs of very different sizes, including ones with W = 0 or Lambda = 0."""
    gs = [
        ("K7", synth.complete(7)),
        ("C9", synth.cycle(9)),          # Lambda = 0
        ("star6", synth.star(6)),        # W = 0
        ("empty4", synth.empty(4)),      # W = Lambda = 0
        ("K2,30", synth.complete_bipartite(2, 30)),
        ("chunglu_2k", synth.chung_lu(2000, 12000, 2.2, 150.0, 5)),
        ("rmat_s11", synth.rmat(11, 12, seed=3)),
    ]
    for s in range(9):
        gs.append((f"er{s}", synth.erdos_renyi(60 + 37 * s, 200 + 150 * s, 100 + s)))
    return gs


MIX = _mix()


def _params(i):
    rng = np.random.default_rng(1000 + i)
    return dict(k_path=int(rng.integers(1, 40000)), k_cent=int(rng.integers(1, 40000)),
                seed=int(rng.integers(0, 2 ** 63)), first_path=int(rng.integers(0, 2 ** 40)),
                first_cent=int(rng.integers(0, 2 ** 40)), delta=0.01)


@pytest.fixture(scope="module")
def prepared():
    _say("batch: prepare", len(MIX), "graphs")
    ogs = [oracle.Graph(off, col) for _, (off, col) in MIX]
    gs = [ps.Graph(*_dev(off, col)) for _, (off, col) in MIX]
    yield ogs, gs
    for g in gs:
        g.destroy()


def _expected(og, p):
    tp = og.sample_path(p["seed"], p["k_path"], p["first_path"]).tolist() if og.R_tau else [0] * 8
    tc = og.sample_centered(p["seed"], p["k_cent"], p["first_cent"]).tolist() if og.R_lam else [0] * 8
    return tp, tc


def _check(results, ogs, params, where):
    for i, (r, og, p) in enumerate(zip(results, ogs, params)):
        tp, tc = _expected(og, p)
        assert r["tally_path"] == tp, (where, MIX[i][0])
        assert r["tally_cent"] == tc, (where, MIX[i][0])
        want = ofin.finalize(tp, tc, og.R_tau, og.R_lam, og.N1, p["k_path"], p["k_cent"])
        for c in range(1, 7):
            assert r["est"][c] == pytest.approx(want["est"][c], rel=1e-12, abs=1e-9), (where, MIX[i][0], c)


@pytest.mark.parametrize("tune", [(64, 1), (1024, 2), (4096, 8), (16384, 4)])
def test_batch_tallies_match_oracle(prepared, tune):
    _say("batch tune", tune)
    ogs, gs = prepared
    params = [_params(i) for i in range(len(gs))]
    b = ps.Batch(gs, params, tune=tune)
    assert b.tune() == tune
    _check(b.run(), ogs, params, f"tune {tune}")
    b.destroy()


def test_batch_equals_solo_counts(prepared):
    _say("batch vs solo")
    ogs, gs = prepared
    params = [_params(50 + i) for i in range(len(gs))]
    got = ps.count_batch(gs, params, tune=(2048, 4))
    for g, p, r in zip(gs, params, got):
        solo = g.count(p["k_path"], p["k_cent"], seed=p["seed"], first_path=p["first_path"],
                       first_cent=p["first_cent"])
        assert r == solo


def test_batch_replays_with_eager_work_between(prepared):
    """The captured graph replayed several times, with the program's own
    eager work and synchronisations between replays: every replay agrees."""
    _say("batch replays")
    ogs, gs = prepared
    params = [_params(200 + i) for i in range(len(gs))]
    b = ps.Batch(gs, params, tune=(1024, 4))
    first = b.run()
    _check(first, ogs, params, "replay 0")
    x = torch.randn(1 << 20, device="cuda")
    for rep in range(1, 5):
        y = (x * rep).sum()             # eager work on torch's stream
        gs[rep].count(1000, 1000, seed=rep)  # and on the library's solo path
        torch.cuda.synchronize()
        assert torch.isfinite(y)
        assert b.run() == first, f"replay {rep}"
    b.destroy()


def test_batch_set_params_without_recapture(prepared):
    _say("batch set_params")
    ogs, gs = prepared
    params = [_params(300 + i) for i in range(len(gs))]
    b = ps.Batch(gs, params, tune=(1024, 2))
    _check(b.run(), ogs, params, "initial")
    smaller = [dict(p, k_path=max(1, p["k_path"] // 3), k_cent=max(1, p["k_cent"] // 5),
                    seed=p["seed"] ^ 0x5555) for p in params]
    b.set_params(smaller)
    _check(b.run(), ogs, smaller, "smaller")
    _check(b.run(), ogs, smaller, "smaller again")
    bigger = [dict(p, k_path=p["k_path"] * 4) for p in params]
    with pytest.raises(ps.PathSampError) as e:
        b.set_params(bigger)
    assert e.value.status == ps.PM_EINVAL
    _check(b.run(), ogs, smaller, "after rejected set_params")  # unchanged
    b.destroy()


def test_batch_autotune_picks_a_candidate(prepared):
    _say("batch autotune")
    ogs, gs = prepared
    params = [_params(400 + i) for i in range(len(gs))]
    b = ps.Batch(gs, params)
    t = b.tune()
    assert t[0] in (1024, 4096, 16384) and t[1] in (2, 4, 8)
    _check(b.run(), ogs, params, "autotuned")
    b.destroy()


def test_batch_single_graph_many_tiles():
    """One graph, a budget of several thousand tiles with a ragged last tile."""
    _say("batch single graph")
    off, col = synth.erdos_renyi(3000, 25000, 8)
    og = oracle.Graph(off, col)
    g = ps.Graph(*_dev(off, col))
    p = dict(k_path=1_000_003, k_cent=999_999, seed=17, first_path=0, first_cent=0, delta=0.01)
    (r,) = ps.count_batch([g], [p], tune=(256, 8))
    assert r["tally_path"] == og.sample_path(17, 1_000_003).tolist()
    assert r["tally_cent"] == og.sample_centered(17, 999_999).tolist()
    g.destroy()


def test_batch_argument_errors(prepared):
    _, gs = prepared
    with pytest.raises(ps.PathSampError) as e:
        ps.count_batch(gs[:1], [dict(k_path=0, k_cent=0)])
    assert e.value.status == ps.PM_EINVAL
    with pytest.raises(ps.PathSampError) as e:
        ps.count_batch(gs[:1], [dict(k_path=10, delta=1.5)])
    assert e.value.status == ps.PM_EINVAL
    with pytest.raises(ps.PathSampError) as e:
        ps.count_batch(gs[:1], [dict(k_path=10)], tune=(16, 4))
    assert e.value.status == ps.PM_EINVAL
    with pytest.raises(ps.PathSampError) as e:
        ps.count_batch(gs[:1], [dict(k_path=10)], tune=(1024, 65))
    assert e.value.status == ps.PM_EINVAL
    with pytest.raises(ps.PathSampError) as e:
        ps.count_batch([], [])
    assert e.value.status == ps.PM_EINVAL
