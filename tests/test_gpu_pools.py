"""Oracle parity of the batched and served modes at their benchmark sizes.

* Batched: the 256 Chung-Lu graphs of the batched benchmark (n log-uniform
  in [1e3, 2e5], m log-uniform in [5e3, 2e6], exponent uniform in [2.1, 2.8];
  graph g: generator seed 1000+g, Philox seed 1+g), k = 2e5 per sampler each,
  in one autotuned, graph-captured persistent launch.  Every graph's W,
  Lambda, N_1 and both tally vectors equal the oracle's own preparation and
  samplers on the same CSR (graphs prepared and sampled on host threads).
* Served: requests for all six motifs at 1% relative error and 99%
  confidence on the two largest graphs of the served pool (R-MAT and
  Chung-Lu, m near 5e7), submitted together with requests on smaller pool
  graphs so that they share steps.  For each large-graph request the oracle
  runs the pilot (ids [0, 65536) per sampler), sizes both samplers with its
  own sizing rule (Corollary 5.3 inverted), and its tallies over the final id
  ranges must equal the served result bit for bit.
"""
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
import oracle_windows
from oracle import finalize as ofin
from paper_1411_4942_amd import pathsamp as ps
from paper_1411_4942_amd import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.mark.timeout(1200)
def test_batched_256_chunglu_vs_oracle():
    t0 = time.time()
    specs = workloads.batched_specs(256)
    k = 200_000
    _say("batched 256: generate", f"{time.time() - t0:.1f}s")
    csrs = [workloads.build(sp) for sp in specs]
    graphs = [ps.Graph(o, c) for o, c in csrs]
    infos = [g.info() for g in graphs]
    host = [(o.cpu().numpy(), c.cpu().numpy()) for o, c in csrs]
    del csrs
    params = [dict(k_path=k, k_cent=k, seed=sp["philox_seed"]) for sp in specs]
    _say("batched 256: autotuned batch run", f"{time.time() - t0:.1f}s")
    b = ps.Batch(graphs, params)
    got = b.run()
    assert b.run() == got  # a second replay of the captured launch
    tune = b.tune()
    b.destroy()
    for g in graphs:
        g.destroy()
    _say("batched 256: tune", tune, "oracle on", oracle_windows.workers(), "threads", f"{time.time() - t0:.1f}s")

    def expect(i):
        off, col = host[i]
        og = oracle.Graph(off, col)
        seed = specs[i]["philox_seed"]
        tp = og.sample_path(seed, k).tolist() if og.R_tau else [0] * 8
        tc = og.sample_centered(seed, k).tolist() if og.R_lam else [0] * 8
        return og.R_tau, og.R_lam, og.N1, tp, tc

    with ThreadPoolExecutor(max_workers=oracle_windows.workers()) as ex:
        want = list(ex.map(expect, range(len(specs))))
    zero = 0
    for i, (info, r, (R_tau, R_lam, N1, tp, tc)) in enumerate(zip(infos, got, want)):
        assert (2 * info["W"], 2 * info["Lambda"], info["N1"]) == (R_tau, R_lam, N1), i
        assert r["tally_path"] == tp, i
        assert r["tally_cent"] == tc, i
        zero += (R_tau == 0) + (R_lam == 0)
        fin = ofin.finalize(tp, tc, R_tau, R_lam, N1, k, k)
        for c in range(1, 7):
            assert r["est"][c] == pytest.approx(fin["est"][c], rel=1e-12, abs=1e-9), (i, c)
    _say("batched 256: all equal;", zero, "zero-weight samplers", f"{time.time() - t0:.1f}s")


def _largest(specs, kind):
    cands = [i for i, sp in enumerate(specs) if sp["kind"] == kind]
    size = (lambda i: specs[i]["m_target"]) if kind == "rmat" else (lambda i: specs[i]["m"])
    return max(cands, key=size)


@pytest.mark.timeout(1200)
def test_served_largest_pool_graphs_vs_oracle():
    t0 = time.time()
    specs = workloads.served_specs(64)
    big = [_largest(specs, "rmat"), _largest(specs, "chung_lu")]
    small = [i for i in range(6) if i not in big]  # smaller pool graphs that share the steps
    ids = big + small
    _say("served: generate pool graphs", ids, f"{time.time() - t0:.1f}s")
    csrs = {i: workloads.build(specs[i]) for i in ids}
    k_max = 2_000_000_000
    k0 = 65_536
    srv = ps.Server(k_max=k_max, k_pilot=k0)
    gid = {i: srv.add_graph(*csrs[i]) for i in ids}
    for i in ids:
        srv.preload(gid[i])
    rng = np.random.default_rng(5)
    reqs = []
    for rep in range(2):
        for i in big:
            reqs.append((i, 20_000 + 10 * i + rep))
    for i in small:
        reqs.append((i, 30_000 + i))
    order = rng.permutation(len(reqs))
    tickets = {}
    for j in order:
        i, seed = reqs[j]
        tickets[j] = srv.submit(gid[i], rel_err=0.01, delta=0.01, seed=seed)
    results = {j: srv.wait(t) for j, t in tickets.items()}
    srv.destroy()
    _say("served: requests done", f"{time.time() - t0:.1f}s")

    host = {i: (csrs[i][0].cpu().numpy(), csrs[i][1].cpu().numpy()) for i in big}
    del csrs
    torch.cuda.empty_cache()
    _say("served: oracle preparation of the two largest graphs",
         [int(host[i][0][-1]) for i in big], "slots", f"{time.time() - t0:.1f}s")
    with ThreadPoolExecutor(max_workers=2) as ex:
        ogs = dict(zip(big, ex.map(lambda i: oracle.Graph(*host[i]), big)))
    del host
    with ThreadPoolExecutor(max_workers=oracle_windows.workers()) as pool:
        for j, (i, seed) in enumerate(reqs):
            if i not in big:
                continue
            og = ogs[i]
            res, st = results[j]
            # the oracle's pilot and its own sizing rule (Corollary 5.3 inverted)
            pp = oracle_windows.tally(og._g, False, seed, k0, pool=pool) if og.R_tau else [0] * 8
            pc = oracle_windows.tally(og._g, True, seed, k0, pool=pool) if og.R_lam else [0] * 8
            sized = ofin.samples_for_request(pp, pc, k0, og.R_tau // 2, og.R_lam // 2, og.N1, 0x7E, 0.01, 0.01,
                                             k_max)
            kp, kc = sized[0], sized[1]
            assert (st["k_path"], st["k_cent"]) == (kp, kc), (i, seed)
            _say("served: graph", i, "seed", seed, "k", kp, kc, f"{time.time() - t0:.1f}s")
            tp = oracle_windows.tally(og._g, False, seed, kp, pool=pool) if og.R_tau else [0] * 8
            tc = oracle_windows.tally(og._g, True, seed, kc, pool=pool) if og.R_lam else [0] * 8
            assert res["tally_path"] == tp, (i, seed)
            assert res["tally_cent"] == tc, (i, seed)
            fin = ofin.finalize(tp, tc, og.R_tau, og.R_lam, og.N1, kp, kc, 0.01)
            for c in range(1, 7):
                assert res["est"][c] == pytest.approx(fin["est"][c], rel=1e-12, abs=1e-9), (i, c)
    _say("served: done", f"{time.time() - t0:.1f}s")
