"""GPU tests of the served mode (pm_server_*).

Every finished request must be bit-for-bit the one-shot count with its final
budgets (and so the oracle's tallies for the same seed and id range), alone
or mixed with other requests, through graph evictions and re-preparations,
whatever step cut its ids.  Sized budgets must be the sizing rule applied to
the request's own pilot.
"""
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


def _dev(off, col):
    return (torch.from_numpy(np.ascontiguousarray(off, np.int64)).cuda(),
            torch.from_numpy(np.ascontiguousarray(col, np.int32)).cuda())


POOL = [
    ("er_a", synth.erdos_renyi(1500, 9000, 21)),
    ("chunglu", synth.chung_lu(4000, 30000, 2.3, 300.0, 22)),
    ("rmat_s11", synth.rmat(11, 16, seed=23)),
    ("K8", synth.complete(8)),
    ("C12", synth.cycle(12)),        # Lambda = 0
    ("star9", synth.star(9)),        # W = Lambda = 0
    ("er_b", synth.erdos_renyi(700, 5000, 24)),
]


@pytest.fixture(scope="module")
def pool():
    _say("server pool")
    dev = [_dev(o, c) for _, (o, c) in POOL]
    solo = [ps.Graph(o, c) for o, c in dev]
    og = [oracle.Graph(o, c) for _, (o, c) in POOL]
    yield dev, solo, og
    for g in solo:
        g.destroy()


def _solo(g, k_path, k_cent, seed):
    return g.count(k_path, k_cent, seed=seed)


def test_fixed_budgets_equal_one_shot_counts(pool):
    _say("server fixed budgets")
    dev, solo, og = pool
    srv = ps.Server(step_samples=1 << 16, samples_per_tile=1024)
    gids = [srv.add_graph(o, c) for o, c in dev]
    rng = np.random.default_rng(3)
    reqs = []
    for r in range(24):
        gi = int(rng.integers(0, len(gids)))
        kp, kc = int(rng.integers(1, 300000)), int(rng.integers(0, 300000))
        seed = int(rng.integers(0, 2 ** 63))
        reqs.append((gi, kp, kc, seed, srv.submit(gids[gi], k_path=kp, k_cent=kc, seed=seed)))
    for gi, kp, kc, seed, t in reqs:
        res, st = srv.wait(t)
        assert res == _solo(solo[gi], kp, kc, seed), POOL[gi][0]
        assert st["k_path"] == kp and st["k_cent"] == kc
        if og[gi].R_tau:
            assert res["tally_path"] == og[gi].sample_path(seed, kp).tolist()
    s = srv.stats()
    assert s["requests_done"] == 24 and s["steps"] >= 1
    srv.destroy()


def test_sized_requests_use_their_pilot(pool):
    _say("server sized")
    dev, solo, og = pool
    k0, kmax = 4096, 400_000
    srv = ps.Server(k_pilot=k0, k_max=kmax, step_samples=1 << 17, samples_per_tile=512)
    gids = [srv.add_graph(o, c) for o, c in dev]
    tickets = []
    for gi in range(len(gids)):
        for seed in (5, 6):
            tickets.append((gi, seed, 0.05, srv.submit(gids[gi], rel_err=0.05, delta=0.01, seed=seed)))
    for gi, seed, eps, t in tickets:
        res, st = srv.wait(t)
        pilot = _solo(solo[gi], k0, k0, seed)
        kp, kc, capped, unseen = ps.samples_for_request(pilot["tally_path"], pilot["tally_cent"], k0, pilot["W"],
                                                        pilot["Lambda"], pilot["N1"], 0, eps, 0.01, kmax)
        assert (st["k_path"], st["k_cent"]) == (kp, kc), POOL[gi][0]
        assert st["capped_mask"] == capped and st["unseen_mask"] == unseen
        assert res == _solo(solo[gi], kp, kc, seed), POOL[gi][0]
        if og[gi].R_lam:
            assert res["tally_cent"] == og[gi].sample_centered(seed, kc).tolist()
    srv.destroy()


def test_same_result_alone_and_in_the_mix(pool):
    """A request run on an idle server and the same request submitted while
    many others run (arriving mid-stream, admitted between steps) give the
    same tallies, estimates and bars."""
    _say("server alone vs mix")
    dev, solo, og = pool
    srv = ps.Server(k_pilot=8192, k_max=2_000_000, step_samples=1 << 18, samples_per_tile=2048, max_active=6)
    gids = [srv.add_graph(o, c) for o, c in dev]
    probe = dict(graph=gids[1], rel_err=0.02, delta=0.01, seed=99)
    alone, st_alone = srv.wait(srv.submit(**probe))
    rng = np.random.default_rng(11)
    others = []
    for r in range(30):
        gi = int(rng.integers(0, len(gids)))
        others.append(srv.submit(gids[gi], rel_err=float(rng.choice([0.02, 0.05])), seed=1000 + r))
        if r == 12:
            t_probe = srv.submit(**probe)
        time.sleep(0.002)
    mixed, st_mixed = srv.wait(t_probe)
    for t in others:
        srv.wait(t)
    assert mixed == alone
    assert (st_mixed["k_path"], st_mixed["k_cent"]) == (st_alone["k_path"], st_alone["k_cent"])
    assert srv.stats()["requests_done"] == 32
    srv.destroy()


def test_admission_by_hbm_budget_evicts_and_reprepares(pool):
    _say("server hbm budget")
    dev, solo, og = pool
    sizes = [g.info()["device_bytes"] for g in solo[:3]]
    budget = max(sizes) + min(sizes) // 2  # one of the three big graphs at a time, roughly
    srv = ps.Server(hbm_budget=budget, max_active=4, step_samples=1 << 16, samples_per_tile=1024)
    gids = [srv.add_graph(o, c) for o, c in dev[:3]]
    order = [0, 1, 2, 0, 2, 1, 1, 0]
    ts = [(gi, srv.submit(gids[gi], k_path=50_000, k_cent=40_000, seed=7 + j)) for j, gi in enumerate(order)]
    for j, (gi, t) in enumerate(ts):
        res, st = srv.wait(t)
        assert res == _solo(solo[gi], 50_000, 40_000, 7 + j)
    s = srv.stats()
    assert s["evictions"] >= 1 and s["preparations"] >= 4
    assert s["resident_bytes"] <= budget
    srv.destroy()


def test_graph_larger_than_budget_is_refused(pool):
    _say("server too large")
    dev, solo, og = pool
    srv = ps.Server(hbm_budget=1 << 16)
    gid = srv.add_graph(*dev[1])
    t = srv.submit(gid, k_path=1000, k_cent=1000)
    with pytest.raises(ps.PathSampError) as e:
        srv.wait(t)
    assert e.value.status == ps.PM_ENOMEM
    with pytest.raises(ps.PathSampError) as e:
        srv.preload(gid)
    assert e.value.status == ps.PM_ENOMEM
    srv.destroy()


def test_invalid_graph_fails_only_its_requests(pool):
    _say("server invalid graph")
    dev, solo, og = pool
    off, col = synth.complete(5)
    bad = col.copy()
    bad[0], bad[1] = bad[1], bad[0]
    srv = ps.Server()
    g_bad = srv.add_graph(*_dev(off, bad))
    g_ok = srv.add_graph(*dev[0])
    t1 = srv.submit(g_bad, k_path=100, k_cent=100)
    t2 = srv.submit(g_ok, k_path=1000, k_cent=1000, seed=3)
    t3 = srv.submit(g_bad, rel_err=0.1)
    with pytest.raises(ps.PathSampError) as e:
        srv.wait(t1)
    assert e.value.status == ps.PM_EGRAPH
    res, _ = srv.wait(t2)
    assert res == _solo(solo[0], 1000, 1000, 3)
    with pytest.raises(ps.PathSampError) as e:
        srv.wait(t3)
    assert e.value.status == ps.PM_EGRAPH
    srv.destroy()


def test_cancel_timeout_and_shutdown(pool):
    _say("server cancel")
    dev, solo, og = pool
    srv = ps.Server(step_samples=1 << 20, max_active=1)
    gid = srv.add_graph(*dev[1])
    big = srv.submit(gid, k_path=4_000_000_000, k_cent=4_000_000_000)  # seconds of work
    queued = srv.submit(gid, k_path=1000, k_cent=1000, seed=2)  # waits for the only slot
    with pytest.raises(ps.PathSampError) as e:
        srv.wait(queued, timeout_ms=1)
    assert e.value.status == ps.PM_EBUSY
    srv.cancel(big)
    with pytest.raises(ps.PathSampError) as e:
        srv.wait(big)
    assert e.value.status == ps.PM_ECANCELED
    res, _ = srv.wait(queued)
    assert res == _solo(solo[1], 1000, 1000, 2)
    pending = [srv.submit(gid, k_path=2_000_000_000, k_cent=1) for _ in range(3)]
    assert pending
    srv.destroy()  # cancels what is left and returns


def test_zero_weight_and_argument_errors(pool):
    _say("server zero weight")
    dev, solo, og = pool
    srv = ps.Server()
    g_star = srv.add_graph(*dev[5])
    g_cyc = srv.add_graph(*dev[4])
    res, st = srv.wait(srv.submit(g_star, rel_err=0.01))
    assert res["tally_path"] == [0] * 8 and res["tally_cent"] == [0] * 8
    assert res["est"][1] == float(og[5].N1) and st["steps"] == 0
    res, st = srv.wait(srv.submit(g_cyc, rel_err=0.01, seed=4))
    assert res == _solo(solo[4], st["k_path"], st["k_cent"], 4)
    assert res["est"][2] == 12.0
    for bad in (dict(graph=77), dict(graph=g_star, rel_err=0.0), dict(graph=g_star, delta=1.0),
                dict(graph=g_star, motif_mask=1)):
        with pytest.raises(ps.PathSampError) as e:
            srv.submit(**bad)
        assert e.value.status == ps.PM_EINVAL
    with pytest.raises(ps.PathSampError):
        ps.Server(samples_per_tile=8)
    srv.destroy()
