#!/usr/bin/env python3
"""Benchmark: the sampling stage of 3-path sampling on one MI355X.

Workload: R-MAT scale 22 (a, b, c, d) = (0.57, 0.19, 0.19, 0.05),
symmetrised and deduplicated (about 1.2e8 undirected edges), k = 1e7 samples
per sampler, Philox seed 1.  The graph is prepared once (validation,
degree-order relabel, tau/lambda prefix sums, N_1, guide tables) and stays
resident, as in serving.  One timed step = pm_count on the prepared graph:
both samplers (per-sample randomness, edge draw, neighbour picks, adjacency
tests, tallies) and the host finalize with 99% error bars.
value = samples per step (2k) / step time.  Preparation and the whole job
(prepare + count + release) are measured separately and reported beside it.

Prints one JSON line.  --gpus above 1 is not supported (one GPU per box).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic bytes one sample must read at minimum (words, no search probes):
# guide pair 8, P[s-1] and P[s] 16, src[s] and col[s] 8, both rows' offsets 32,
# the two picks 8, three adjacency tests at (two offsets 16 + the hit word 4) 60
BYTES_PER_SAMPLE = 132


def source_hash() -> str:
    """Hash of the HIP library sources: counters taken on other sources are stale."""
    import glob
    import hashlib

    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_1411_4942_amd", "csrc", "*"))):
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic():
    """Per-dispatch HBM bytes measured with rocprofv3 counters (profiles/traffic.json),
    or None when the library sources changed since they were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    return t if t.get("source_hash") == source_hash() else None


def rev_pass_bytes(n: int) -> float:
    """Algorithmic bytes per element of one reverse-sort scatter launch,
    averaged over its passes (8-bit digits over the bits of n - 1)."""
    bits = max(int(n - 1).bit_length(), 1)
    passes = (bits + 7) // 8
    if passes == 1:
        return 8.0  # key read, value written
    per = [12.0] + [16.0] * (passes - 2) + [12.0]
    return sum(per) / passes


def roofline_for(name, kern, alg_entry, traffic, copy_gbs=None):
    alg_bytes, symbol = alg_entry
    achieved = alg_bytes / (kern["avg_ms"] * 1e-3) / 1e9
    tr = hit = None
    if traffic:
        cands = [v for key, v in traffic["kernels"].items() if key.startswith(symbol + "@")]
        if cands:
            best = max(cands, key=lambda v: v["fetch_bytes"])
            tr = best["fetch_bytes"] + best["write_bytes"]
            if best.get("tcc_hit") is not None and best.get("tcc_miss"):
                hit = best["tcc_hit"] / (best["tcc_hit"] + best["tcc_miss"])
    return {"bound": "hbm", "kernel": name, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": tr, "algorithmic_bytes": alg_bytes,
            "measured_copy_gbs": copy_gbs, "frac_of_copy": achieved / copy_gbs if copy_gbs else None,
            "avg_launch_ms": kern["avg_ms"], "launches_timed": kern.get("launches"),
            "traffic_over_algorithmic": (tr / alg_bytes) if tr else None,
            "traffic_gbs": (tr / (kern["avg_ms"] * 1e-3) / 1e9) if tr else None,
            "tcc_hit_rate": hit}


COPY_BYTES = 1 << 30


def measure_copy(stream, reps: int = 5) -> float:
    """Measured streaming ceiling: the library's copy kernel over 1 GiB
    (read + write bytes / average launch time, HIP events on its stream)."""
    import torch

    from paper_1411_4942_amd import pathsamp as ps

    a = torch.empty(COPY_BYTES // 4, dtype=torch.int32, device="cuda").fill_(1)
    b = torch.empty_like(a)
    ps.device_copy(b, a, stream=stream)
    ps.profile_enable(True)
    for _ in range(reps):
        ps.device_copy(b, a, stream=stream)
    torch.cuda.synchronize()
    n, ms = ps.profile_read()["stream_copy"]
    ps.profile_enable(False)
    del a, b
    return 2 * COPY_BYTES / (ms / n * 1e-3) / 1e9


def measure_gather(stream, count: int = 1 << 28, reps: int = 3) -> float:
    """Measured random-access ceiling: independent 4-byte loads at random
    positions of a 2 GiB table (loads per second; each touches its own line)."""
    import torch

    from paper_1411_4942_amd import pathsamp as ps

    t = torch.empty(COPY_BYTES * 2 // 4, dtype=torch.int32, device="cuda").fill_(3)
    ps.device_gather(t, count, seed=7, stream=stream)
    ps.profile_enable(True)
    for r in range(reps):
        ps.device_gather(t, count, seed=11 + r, stream=stream)
    torch.cuda.synchronize()
    n, ms = ps.profile_read()["random_gather"]
    ps.profile_enable(False)
    del t
    return count / (ms / n * 1e-3)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_graph(scale: int, edge_factor: float, seed: int):
    import torch

    from paper_1411_4942_amd import synth

    t0 = time.perf_counter()
    off, col = synth.rmat_torch(scale, edge_factor, seed=seed, device="cuda")
    torch.cuda.synchronize()
    log(f"[bench] R-MAT scale {scale} ef {edge_factor}: n={off.numel() - 1} 2m={col.numel()} "
        f"({time.perf_counter() - t0:.1f}s)")
    return off, col


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform

    return platform.processor() or "unknown"


def cpu_baseline(off, col, k_sample: int, seed: int, gpu_tallies) -> dict:
    """The oracle (single thread, the calling thread pinned to one core) on the
    benchmark's own CSR: its preparation timed once, then each sampler over
    the first k_sample ids (a bounded sample of the k ids a step draws),
    whose tallies must equal the GPU's over the same ids."""
    import oracle

    core = sorted(os.sched_getaffinity(0))[0]
    saved = os.sched_getaffinity(0)
    os.sched_setaffinity(0, {core})  # this thread only (Linux): the oracle runs in it
    try:
        t0 = time.perf_counter()
        g = oracle.Graph(off, col)
        t1 = time.perf_counter()
        tp = g.sample_path(seed, k_sample).tolist()
        t2 = time.perf_counter()
        tc = g.sample_centered(seed, k_sample).tolist()
        t3 = time.perf_counter()
    finally:
        os.sched_setaffinity(0, saved)
    # second figure, not the oracle's own: the same single-threaded oracle
    # calls over id windows on every host thread (tallies are sums over ids)
    from concurrent.futures import ThreadPoolExecutor

    threads = len(saved)
    windows = 4 * threads
    step = (k_sample + windows - 1) // windows
    parts = [(f, min(step, k_sample - f)) for f in range(0, k_sample, step)]
    t4 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        outs = list(ex.map(lambda fw: (g.sample_path(seed, fw[1], fw[0]), g.sample_centered(seed, fw[1], fw[0])),
                           parts))
    t5 = time.perf_counter()
    tp_all = [int(sum(int(o[0][c]) for o in outs)) for c in range(8)]
    tc_all = [int(sum(int(o[1][c]) for o in outs)) for c in range(8)]
    return {
        "value": 2 * k_sample / (t3 - t1),
        "unit": "samples/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"the benchmark graph itself (R-MAT scale 22, 2m={int(off[-1])}), oracle preparation once, "
                  f"then ids [0, {k_sample}) of each sampler (of the {{k}} per step), Philox seed {seed}, "
                  f"one thread pinned to core {core}",
        "cpu_model": cpu_model(),
        "nproc": os.cpu_count(),
        "prep_s": t1 - t0,
        "path_samples_per_s": k_sample / (t2 - t1),
        "centered_samples_per_s": k_sample / (t3 - t2),
        "bit_exact_vs_gpu": tp == gpu_tallies[0] and tc == gpu_tallies[1],
        "all_threads": {"kind": "not the oracle: its samplers over id windows on every host thread",
                        "threads": threads, "samples_per_s": 2 * k_sample / (t5 - t4),
                        "same_tallies": tp_all == tp and tc_all == tc},
    }


def _graph_seconds(fn):
    import torch

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, time.perf_counter() - t0


def batched_leg(count: int, k: int, replays: int) -> dict:
    """Many Chung-Lu graphs in one captured persistent launch, against the
    same work as sequential pm_count calls and as one plain launch."""
    import torch

    from paper_1411_4942_amd import pathsamp as ps
    from paper_1411_4942_amd import workloads

    specs = workloads.batched_specs(count)
    t0 = time.perf_counter()
    csrs = []
    for i, sp in enumerate(specs):
        csrs.append(workloads.build(sp))
        if (i + 1) % 64 == 0:
            log(f"[bench] batched: generated {i + 1}/{count} graphs ({time.perf_counter() - t0:.1f}s)")
    graphs, prep_s = _graph_seconds(lambda: [ps.Graph(o, c) for o, c in csrs])
    infos = [g.info() for g in graphs]
    params = [dict(k_path=k, k_cent=k, seed=sp["philox_seed"]) for sp in specs]
    drawn = sum((k if i["W"] else 0) + (k if i["Lambda"] else 0) for i in infos)

    batch, create_s = _graph_seconds(lambda: ps.Batch(graphs, params))
    res = batch.run()  # warm replay
    times = []
    for _ in range(replays):
        r2, dt = _graph_seconds(batch.run)
        times.append(dt)
        assert r2 == res
    t_batch = min(times)
    log(f"[bench] batched: tune {batch.tune()}, replay {1e3 * t_batch:.2f} ms")

    def sequential():
        return [g.count(p["k_path"], p["k_cent"], seed=p["seed"]) for g, p in zip(graphs, params)]

    seq = sequential()
    seq, t_seq = _graph_seconds(sequential)
    big = max(range(count), key=lambda i: infos[i]["m"])
    half = drawn // 2
    graphs[big].count(half, half, seed=1)
    _, t_plain = _graph_seconds(lambda: graphs[big].count(half, half, seed=1))
    out = {
        "workload": f"{count} Chung-Lu graphs, n log-uniform [1e3,2e5], m log-uniform [5e3,2e6], "
                    f"gamma U[2.1,2.8], k={k} per sampler each, Philox seed 1+g",
        "graphs": count,
        "sum_m": int(sum(i["m"] for i in infos)),
        "zero_W": int(sum(1 for i in infos if i["W"] == 0)),
        "zero_Lambda": int(sum(1 for i in infos if i["Lambda"] == 0)),
        "samples_drawn": int(drawn),
        "tune": list(batch.tune()),
        "autotune_and_capture_s": create_s,
        "prep_s": prep_s,
        "batched_ms": 1e3 * t_batch,
        "batched_samples_per_s": drawn / t_batch,
        "sequential_ms": 1e3 * t_seq,
        "sequential_samples_per_s": drawn / t_seq,
        "plain_one_graph_ms": 1e3 * t_plain,
        "plain_one_graph_samples_per_s": 2 * half / t_plain,
        "plain_graph_m": int(infos[big]["m"]),
        "bit_exact_vs_sequential": res == seq,
    }
    batch.destroy()
    for g in graphs:
        g.destroy()
    del csrs
    torch.cuda.empty_cache()
    ps.release_cached_memory()
    return out


def ingest_leg(scale: int, edge_factor: float, seed: int, k: int, want: dict, reps: int = 3) -> dict:
    """End to end from the raw pair list: the R-MAT draws (loops and repeats
    included) through pm_graph_from_edges and pm_count."""
    import torch

    from paper_1411_4942_amd import pathsamp as ps
    from paper_1411_4942_amd import synth

    u, v = synth.rmat_edges_torch(scale, edge_factor, seed=seed, device="cuda")
    src, dst = u.to(torch.int32), v.to(torch.int32)
    del u, v
    n = 1 << scale
    stream = torch.cuda.current_stream()

    def once():
        g = ps.Graph.from_edges(n, src, dst, stream=stream)
        r = g.count(k, k, seed=1, stream=stream)
        g.destroy()
        return r

    res = once()
    ps.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        res = once()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ps.profile_read()
    ps.profile_enable(False)
    ms = 1e3 * (t1 - t0) / reps
    out = {
        "workload": f"raw R-MAT scale {scale} draws ({src.numel()} pairs, loops and repeats included) -> "
                    f"CSR on the device -> prepare -> k={k} per sampler",
        "pairs": int(src.numel()),
        "ingest_ms": prof["ingest_total"][1] / prof["ingest_total"][0],
        "end_to_end_ms": ms,
        "end_to_end_samples_per_s": 2 * k / (ms * 1e-3),
        "same_tallies_as_csr_input": res["tally_path"] == want["tally_path"] and res["tally_cent"] == want["tally_cent"],
    }
    del src, dst
    torch.cuda.empty_cache()
    return out


def alias_leg(off, col, k: int, stream, reps: int = 3) -> dict:
    """The alias-table edge draw on the benchmark graph: table build time and
    a whole count (both samplers) against the main draw's (guide table and
    search)."""
    import torch

    from paper_1411_4942_amd import pathsamp as ps

    g = ps.Graph(off, col, stream=stream)
    g.build_alias(stream=stream)  # first build: allocations warmed
    g.destroy()
    g = ps.Graph(off, col, stream=stream)
    ps.profile_enable(True)
    g.build_alias(stream=stream)
    for _ in range(reps):
        a = g.count_alias(k, k, seed=1, stream=stream)
        m = g.count(k, k, seed=1, stream=stream)
    prof = ps.profile_read()
    ps.profile_enable(False)

    def avg(name):
        n, ms = prof[name]
        return ms / n

    # whole calls (both samplers: key draws, sorts, sampling kernels), timed
    # on the host without the per-kernel events, one draw after the other
    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t0) / reps

    alias_ms = timed(lambda: g.count_alias(k, k, seed=1, stream=stream))
    main_ms = timed(lambda: g.count(k, k, seed=1, stream=stream))
    g.destroy()
    build_ms = avg("alias_build")
    saved_per_sample = (main_ms - alias_ms) / (2 * k)
    return {
        "workload": f"the benchmark graph; k={k} per sampler, Philox seed 1, {reps} runs each",
        "table_build_ms": build_ms,
        "table_bytes": 2 * 32 * int(off[-1].item()),  # two tables, 32 bytes per slot
        "alias_sampling_ms": alias_ms,
        "main_sampling_ms": main_ms,
        "alias_samples_per_s": 2 * k / (alias_ms * 1e-3),
        "main_samples_per_s": 2 * k / (main_ms * 1e-3),
        "breakeven_samples": (build_ms / saved_per_sample) if saved_per_sample > 0 else None,
        "kernels_ms": {n: avg(n) for n in prof if n.startswith("alias") or n.startswith("sample_")},
        "estimates_within_bars": all(
            abs(a["est"][i] - m["est"][i]) <= (a["hi"][i] - a["lo"][i]) / 2 + (m["hi"][i] - m["lo"][i]) / 2
            for i in range(1, 7)),
    }


def accuracy_leg(ks=(2500, 5000, 10000, 20000, 35000), seeds: int = 50) -> dict:
    """The paper's accuracy experiments (Section 6) on synthetic stand-ins:
    exact counts from pm_exact_counts, then `seeds` runs per k (batched, Philox
    seeds 1000 k + s): mean relative error of each motif's estimate, the
    fraction of runs whose 99% bars hold the exact count, and at the largest k
    the centered estimator's error against Algorithm 2's basic one."""
    import numpy as np
    import torch

    from paper_1411_4942_amd import pathsamp as ps
    from paper_1411_4942_amd import synth

    graphs = [("Chung-Lu n=1e6, m=1e7, gamma 2.3, w_max 5000, seed 1",
               lambda: synth.chung_lu_torch(1_000_000, 10_000_000, 2.3, 5000.0, 1, device="cuda")),
              ("R-MAT scale 16 (0.57, 0.19, 0.19, 0.05), edge factor 16, seed 1",
               lambda: synth.rmat_torch(16, 16.0, seed=1))]
    out = []
    for name, make in graphs:
        off, col = make()
        g = ps.Graph(off, col)
        del off, col
        C = g.exact()["C"]
        per_k = []
        for k in ks:
            params = [ps.make_params(k, k, seed=1000 * k + s) for s in range(seeds)]
            runs = ps.count_batch([g] * seeds, params)
            per_k.append({
                "k": k,
                "mean_rel_err": [float(np.mean([abs(r["est"][i] - C[i]) / C[i] for r in runs])) if C[i] else None
                                 for i in range(1, 7)],
                "bar_coverage": [float(np.mean([r["lo"][i] - 1e-6 <= C[i] <= r["hi"][i] + 1e-6 for r in runs]))
                                 for i in range(1, 7)],
            })
        last = runs
        out.append({
            "graph": name,
            "exact_counts": C[1:],
            "runs_per_k": seeds,
            "by_k": per_k,
            "centered_vs_basic_rel_err_k35000": [
                (float(np.mean([abs(r["est"][i] - C[i]) / C[i] for r in last])),
                 float(np.mean([abs(r["est_basic"][i] - C[i]) / C[i] for r in last]))) if C[i] else None
                for i in (4, 5, 6)],
        })
        g.destroy()
        torch.cuda.empty_cache()
    return {"graphs": out, "delta": 0.01}


def exact_leg(k: int = 2_000_000) -> dict:
    """Sampling against exact enumeration on Chung-Lu n = 1e6, m = 1e7
    (exponent 2.3, weight cap 5000, seed 1): times and the estimates' error."""
    import torch

    from paper_1411_4942_amd import pathsamp as ps
    from paper_1411_4942_amd import synth

    off, col = synth.chung_lu_torch(1_000_000, 10_000_000, 2.3, 5000.0, 1, device="cuda")
    g = ps.Graph(off, col)
    g.exact()
    res = g.count(k, k, seed=1)
    t_ex = t_sa = 1e30
    for _ in range(3):
        ex, dt = _graph_seconds(g.exact)
        t_ex = min(t_ex, dt)
        res, dt = _graph_seconds(lambda: g.count(k, k, seed=1))
        t_sa = min(t_sa, dt)
    g.destroy()
    del off, col
    torch.cuda.empty_cache()
    C = ex["C"]
    return {
        "workload": f"Chung-Lu n=1e6, m=1e7, gamma 2.3, w_max 5000, seed 1; k={k} per sampler, Philox seed 1",
        "exact_ms": 1e3 * t_ex,
        "sampling_ms": 1e3 * t_sa,
        "exact_over_sampling": t_ex / t_sa,
        "exact_counts": C[1:],
        "rel_err": [abs(res["est"][i] - C[i]) / C[i] if C[i] else None for i in range(1, 7)],
        "inside_99pct_bars": [res["lo"][i] <= C[i] <= res["hi"][i] for i in range(1, 7)],
    }


def exact_headline_leg(off, col, res, step_ms: float, stream) -> dict:
    """Exact counts of the benchmark graph itself (the enumeration of
    Section 6 against sampling, as in the paper's speedup figure) and the
    benchmark estimates' error against them."""
    from paper_1411_4942_amd import pathsamp as ps

    g = ps.Graph(off, col, stream=stream)
    ps.profile_enable(True)
    ex, dt = _graph_seconds(lambda: g.exact(stream=stream))
    prof = ps.profile_read()
    ps.profile_enable(False)
    g.destroy()
    C = ex["C"]
    return {
        "workload": "the benchmark graph (R-MAT scale 22); estimates from one benchmark step (k = 1e7 per sampler)",
        "exact_ms": 1e3 * dt,
        "exact_kernels_ms": {n: v[1] / v[0] for n, v in prof.items() if n.startswith("exact")},
        "sampling_step_ms": step_ms,
        "exact_over_sampling": 1e3 * dt / step_ms,
        "exact_counts": C[1:],
        "triangles": ex["triangles"],
        "rel_err": [abs(res["est"][i] - C[i]) / C[i] if C[i] else None for i in range(1, 7)],
        "inside_99pct_bars": [res["lo"][i] <= C[i] <= res["hi"][i] for i in range(1, 7)],
    }


def served_leg(count: int, n_sat: int, n_open: int, loads, rel_err: float, delta: float, k_max: int,
               plain_check: int) -> dict:
    """A pool of resident graphs behind the request server: closed-loop
    saturation, then Poisson arrivals at fractions of it."""
    import numpy as np
    import torch

    from paper_1411_4942_amd import pathsamp as ps
    from paper_1411_4942_amd import workloads

    specs = workloads.served_specs(count)
    t0 = time.perf_counter()
    csrs = []
    for i, sp in enumerate(specs):
        csrs.append(workloads.build(sp))
        if (i + 1) % 16 == 0:
            log(f"[bench] served: generated {i + 1}/{count} graphs ({time.perf_counter() - t0:.1f}s)")
    srv = ps.Server(k_max=k_max)
    gids = [srv.add_graph(o, c) for o, c in csrs]
    _, prep_s = _graph_seconds(lambda: [srv.preload(g) for g in gids])
    st0 = srv.stats()
    log(f"[bench] served: {count} graphs resident, {st0['resident_bytes'] / 2 ** 30:.1f} GiB, prep {prep_s:.1f}s")
    rng = np.random.Generator(np.random.PCG64(1))
    seed_ctr = [10_000]

    def one_request():
        seed_ctr[0] += 1
        return dict(graph=int(gids[int(rng.integers(0, count))]), rel_err=rel_err, delta=delta, seed=seed_ctr[0])

    def run(reqs, arrivals):
        """Submit at the given offsets (s), wait for all; (records, wall s, samples)."""
        s_before = srv.stats()["samples"]
        start = time.perf_counter()
        tickets = []
        for rq, at in zip(reqs, arrivals):
            now = time.perf_counter() - start
            if at > now:
                time.sleep(at - now)
            tickets.append(srv.submit(**rq))
        recs = []
        for rq, t in zip(reqs, tickets):
            res, st = srv.wait(t)
            recs.append((rq, res, st))
        wall = time.perf_counter() - start
        return recs, wall, srv.stats()["samples"] - s_before

    sat_reqs = [one_request() for _ in range(n_sat)]
    recs, wall, samples = run(sat_reqs, [0.0] * n_sat)
    sat_rps = n_sat / wall
    log(f"[bench] served: saturation {sat_rps:.2f} req/s, {samples / wall:.3e} samples/s")
    out = {
        "workload": f"{count} resident graphs (R-MAT + Chung-Lu, m log-uniform [1e4,5e7]), requests for all six "
                    f"motifs at rel_err {rel_err}, delta {delta}, k from Corollary 5.3 on a 65536-id pilot, "
                    f"k_max {k_max:.0e}",
        "graphs": count,
        "resident_gib": st0["resident_bytes"] / 2 ** 30,
        "sum_m": int(sum(int(c.numel()) // 2 for _, c in csrs)),
        "prep_s": prep_s,
        "saturation": {"requests": n_sat, "req_per_s": sat_rps, "samples_per_s": samples / wall,
                       "p50_ms": float(np.percentile([r[2]["latency_ms"] for r in recs], 50)),
                       "p99_ms": float(np.percentile([r[2]["latency_ms"] for r in recs], 99))},
        "capped_requests": int(sum(1 for r in recs if r[2]["capped_mask"])),
        "mean_k_per_sampler": float(np.mean([(r[2]["k_path"] + r[2]["k_cent"]) / 2 for r in recs])),
        "open_loop": [],
    }
    # the same requests one at a time through pm_count on a freshly prepared graph
    if plain_check > 0:
        t_plain = 0.0
        drawn = 0
        same = True
        for rq, res, st in recs[:plain_check]:
            o, c = csrs[gids.index(rq["graph"])]
            g = ps.Graph(o, c)
            r2, dt = _graph_seconds(lambda: g.count(st["k_path"], st["k_cent"], seed=rq["seed"], delta=rq["delta"]))
            t_plain += dt
            drawn += (st["k_path"] if r2["W"] else 0) + (st["k_cent"] if r2["Lambda"] else 0)
            same &= r2 == res
            g.destroy()
        out["plain_sequential"] = {"requests": plain_check, "samples_per_s": drawn / t_plain,
                                   "bit_exact_vs_served": same}
    for frac in loads:
        qps = frac * sat_rps
        gaps = rng.exponential(1.0 / qps, size=n_open)
        arrivals = np.cumsum(gaps) - gaps[0]
        reqs = [one_request() for _ in range(n_open)]
        recs, wall, samples = run(reqs, arrivals.tolist())
        lat = [r[2]["latency_ms"] for r in recs]
        out["open_loop"].append({"load": frac, "qps": qps, "requests": n_open, "req_per_s": n_open / wall,
                                 "samples_per_s": samples / wall, "p50_ms": float(np.percentile(lat, 50)),
                                 "p99_ms": float(np.percentile(lat, 99)),
                                 "mean_queued_ms": float(np.mean([r[2]["queued_ms"] for r in recs]))})
        log(f"[bench] served: load {frac:.2f}: p50 {out['open_loop'][-1]['p50_ms']:.0f} ms, "
            f"p99 {out['open_loop'][-1]['p99_ms']:.0f} ms")
    st = srv.stats()
    out["server_steps"] = st["steps"]
    out["server_busy_ms"] = st["busy_ms"]
    srv.destroy()
    del csrs
    torch.cuda.empty_cache()
    ps.release_cached_memory()
    return out


# The paper's own figure for context (Table 3, Section 6): orkut, 2.24e8
# edges, k = 200K per sampler, 16.24 s end to end including reading the edge
# list, C code on a 2 x 2.4 GHz Xeon with 6 cores.  Not the same metric.
PAPER_CONTEXT = {
    "source": "Table 3 and Section 6: 3-path sampling time, end to end including reading the edge list",
    "graph": "orkut (SNAP), 3.07e6 vertices, 2.24e8 edges",
    "k_per_sampler": 200_000,
    "seconds": 16.24,
    "machine": "2 x 2.4 GHz Intel Xeon, 6 cores, 64 GB (C implementation)",
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--scale", type=int, default=22)
    ap.add_argument("--edge-factor", type=float, default=31.0)
    ap.add_argument("--k", type=int, default=10_000_000)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--whole-steps", type=int, default=5)
    ap.add_argument("--cpu-k", type=int, default=1_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-ingest", action="store_true")
    ap.add_argument("--no-exact", action="store_true")
    ap.add_argument("--no-alias", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--batch-graphs", type=int, default=256)
    ap.add_argument("--batch-k", type=int, default=200_000)
    ap.add_argument("--served-graphs", type=int, default=64)
    ap.add_argument("--served-sat", type=int, default=4000)
    ap.add_argument("--served-open", type=int, default=3000)
    ap.add_argument("--served-loads", type=str, default="0.25,0.5,0.75,0.9")
    ap.add_argument("--served-kmax", type=float, default=2e9)
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the multi-GPU sharding of the path is "
              "designed, not built.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1411_4942_amd import pathsamp as ps

    torch.cuda.set_device(0)
    ps.lib()
    off, col = make_graph(args.scale, args.edge_factor, args.seed)
    stream = torch.cuda.current_stream()
    k = args.k

    # the prepared graph stays resident; a step samples it
    g = ps.Graph(off, col, stream=stream)
    info = g.info()
    slots = 2 * info["m"]

    def step():
        return g.count(k, k, seed=1, stream=stream)

    for i in range(args.warmup):
        t0 = time.perf_counter()
        res = step()
        log(f"[bench] warmup {i}: {1e3 * (time.perf_counter() - t0):.2f} ms")

    # per-kernel breakdown of a step: separate steps with every scope timed
    ps.profile_enable(True)
    for i in range(2):
        step()
    torch.cuda.synchronize()
    kernels = {name: {"launches": n, "avg_ms": ms / n, "ms_per_step": ms / 2}
               for name, (n, ms) in ps.profile_read().items()}
    ps.profile_enable(False)
    samp = "sample_path.sorted" if "sample_path.sorted" in kernels else "sample_path"
    cent = "sample_centered.sorted" if "sample_centered.sorted" in kernels else "sample_centered"
    alg_samp = {
        # the sampling kernels (row-hash adjacency tests, the default search
        # mode 2): algorithmic bytes per sample x samples per launch
        "sample_path.sorted": (BYTES_PER_SAMPLE * k, "pm::k_sample_sorted<false, 2>"),
        "sample_centered.sorted": (BYTES_PER_SAMPLE * k, "pm::k_sample_sorted<true, 2>"),
        "sample_path": (BYTES_PER_SAMPLE * k, "pm::k_sample<false, 1, 2>"),
        "sample_centered": (BYTES_PER_SAMPLE * k, "pm::k_sample<true, 1, 2>"),
    }

    # the timed region: K steps; HIP events only around the 3-path sampling
    # kernel (the step's dominant kernel) on the stream it runs on
    ps.profile_select([samp])
    ps.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        res = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    live = {name: {"launches": n, "avg_ms": ms / n, "ms_per_step": ms / args.steps}
            for name, (n, ms) in ps.profile_read().items()}
    ps.profile_enable(False)
    ps.profile_select(None)
    ms_per_step = 1e3 * (t1 - t0) / args.steps
    value = 2 * k / ((t1 - t0) / args.steps)
    log(f"[bench] {args.steps} steps: {ms_per_step:.3f} ms/step, {value:.4e} samples/s")

    # the whole job per graph: prepare + count + release (the preparation
    # kernels' breakdown from the same steps)
    def whole():
        h = ps.Graph(off, col, stream=stream)
        r = h.count(k, k, seed=1, stream=stream)
        h.destroy()
        return r

    whole()
    # timed without the per-kernel events (each timed scope adds two event
    # records between kernels); the breakdown comes from separate steps
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for _ in range(args.whole_steps):
        rw = whole()
    torch.cuda.synchronize()
    w1 = time.perf_counter()
    assert rw["tally_path"] == res["tally_path"] and rw["tally_cent"] == res["tally_cent"]
    whole_ms = 1e3 * (w1 - w0) / args.whole_steps
    prof_steps = 2
    ps.profile_enable(True)
    for _ in range(prof_steps):
        whole()
    torch.cuda.synchronize()
    prep_kernels = {name: {"launches": n, "avg_ms": ms / n, "ms_per_step": ms / prof_steps}
                    for name, (n, ms) in ps.profile_read().items()}
    ps.profile_enable(False)
    # the preparation alone: its outer scope only, no events between its kernels
    ps.profile_select(["prep_total"])
    ps.profile_enable(True)
    for _ in range(args.whole_steps):
        whole()
    torch.cuda.synchronize()
    prep_n, prep_total_ms = ps.profile_read()["prep_total"]
    ps.profile_enable(False)
    ps.profile_select(None)
    prep_ms = prep_total_ms / prep_n
    log(f"[bench] whole job: {whole_ms:.2f} ms/step (prepare {prep_ms:.2f} ms)")

    copy_gbs = measure_copy(stream)
    gather_per_s = measure_gather(stream)
    traffic = load_traffic()
    roofline = roofline_for(samp, live[samp], alg_samp[samp], traffic, copy_gbs)
    # line-granular view: fetched 128-byte lines per sample against the
    # measured random-load ceiling (one line per independent random load)
    roofline["random_loads_per_s_ceiling"] = gather_per_s
    if roofline["traffic"]:
        lines = roofline["traffic"] / 128.0 / k
        roofline["lines_per_sample"] = lines
        roofline["lines_per_s"] = lines * k / (live[samp]["avg_ms"] * 1e-3)
        roofline["frac_of_random_ceiling"] = roofline["lines_per_s"] / gather_per_s
    roofline_cent = roofline_for(cent, kernels[cent], alg_samp[cent], traffic, copy_gbs)

    prep_alg = {
        # per launch, averaged over the passes: the first reads no value (the
        # payload is the position: key 4 read, key 4 + value 4 written), the
        # middle ones read and write key + value (16), the last writes no key
        # (key 4 + value 4 read, value 4 written)
        "reverse_sort.scatter": (rev_pass_bytes(info["n"]) * slots, "pm::radix_scatter"),
        "reverse_sort.histogram": (4 * slots, "pm::radix_histogram"),
        # per slot: input column 4, its rank 4, column 4 and edge 8 written
        "build_rows": (20 * slots, "pm::k_rows_block"),
        # per slot: edge 8 + rev 4, both rows' 32-bit offset pairs 16, both
        # segment prefixes written 16, the slot record written 16
        "weights.reduce": (60 * slots, "pm::k_weights_reduce"),
        # per slot: its column read 4, two row-hash entries written 8
        "rowhash": (12 * slots, "pm::k_rowhash_small"),
        # per slot: both segment prefixes read 16, guide entries 2 (2m/4 buckets of 4 bytes per table)
        "weights.guide": (18 * slots, "pm::k_guide_fill"),
    }
    multi = {"build_rows", "rowhash"}  # scopes over several kernels: reported, never the dominant kernel
    cand = {n: v for n, v in prep_kernels.items() if n in prep_alg and n not in multi}
    prep_dom = max(cand, key=lambda n: cand[n]["ms_per_step"])
    roofline_prep = roofline_for(prep_dom, prep_kernels[prep_dom], prep_alg[prep_dom], traffic, copy_gbs)
    # the bytes of a multi-kernel scope are those of the whole preparation
    # (the row hash is built in two calls): time it per preparation
    def scope_ms(n):
        return prep_kernels[n]["ms_per_step"] if n in multi else prep_kernels[n]["avg_ms"]

    roofline_prep_all = {n: {"achieved_gbs": prep_alg[n][0] / (scope_ms(n) * 1e-3) / 1e9,
                             "frac": prep_alg[n][0] / (scope_ms(n) * 1e-3) / 1e9 / HBM_PEAK_GBS,
                             "ms_per_step": prep_kernels[n]["ms_per_step"]}
                         for n in prep_alg if n in prep_kernels}
    samp_ms = [kernels[n]["avg_ms"] for n in ("sample_path", "sample_centered") if n in kernels]

    out = {
        "metric": "3-path samples/s on R-MAT 120M edges",
        "value": value,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {
            "workload": f"R-MAT scale {args.scale} (0.57,0.19,0.19,0.05), edge factor {args.edge_factor}, "
                        f"symmetrised+dedup, prepared once and resident; step = pm_count: k={k} 3-path + {k} "
                        f"centered samples (Philox seed 1) + host finalize",
            "n": info["n"], "m": info["m"], "dmax": info["dmax"], "isolated": info["isolated"],
            "W": info["W"], "Lambda": info["Lambda"], "N1": info["N1"],
            "samples_per_step": 2 * k,
            "parallelism": "single GPU",
        },
        "roofline": roofline,
        "roofline_centered": roofline_cent,
        "roofline_prep": roofline_prep,
        "roofline_prep_by_kernel": roofline_prep_all,
        "prep_ms": prep_ms,
        "whole_job": {"what": "pm_graph_create from the device-resident CSR (all checks) + pm_count + "
                              "pm_graph_destroy, per step",
                      "ms_per_step": whole_ms, "samples_per_s": 2 * k / (whole_ms * 1e-3),
                      "steps": args.whole_steps},
        # every scope of a step, from two profiled steps outside the timed region
        "kernels": kernels,
        "prep_kernels": prep_kernels,
        "sampling_kernels_samples_per_s": 2 * k / (sum(samp_ms) * 1e-3),
        "estimates": res["est"][1:],
        "rel_bar_halfwidth": [((h - l) / 2 / e if e else None) for e, l, h in zip(res["est"][1:], res["lo"][1:], res["hi"][1:])],
        "paper_context": dict(PAPER_CONTEXT),
    }
    # the paper's end-to-end figure next to ours at its k (prepare + 2 x 200K samples)
    kp = PAPER_CONTEXT["k_per_sampler"]
    h = ps.Graph(off, col, stream=stream)
    h.count(kp, kp, seed=1, stream=stream)
    h.destroy()
    torch.cuda.synchronize()
    c0 = time.perf_counter()
    h = ps.Graph(off, col, stream=stream)
    h.count(kp, kp, seed=1, stream=stream)
    h.destroy()
    torch.cuda.synchronize()
    out["paper_context"]["this_gpu_prepare_plus_200k_per_sampler_ms"] = 1e3 * (time.perf_counter() - c0)
    out["paper_context"]["this_gpu_graph"] = f"R-MAT scale {args.scale}, {info['m']} edges, CSR already in HBM"

    gpu_cpu_tallies = None
    if not args.no_cpu_baseline:
        r_small = g.count(args.cpu_k, args.cpu_k, seed=1, stream=stream)
        gpu_cpu_tallies = (r_small["tally_path"], r_small["tally_cent"])
    g.destroy()
    if not args.no_ingest:
        log("[bench] ingest leg ...")
        out["ingest"] = ingest_leg(args.scale, args.edge_factor, args.seed, k, res)
        log(f"[bench] ingest: {out['ingest']['ingest_ms']:.2f} ms, end to end {out['ingest']['end_to_end_ms']:.2f} ms")
    if not args.no_alias:
        log("[bench] alias leg ...")
        out["alias"] = alias_leg(off, col, k, stream)
        log(f"[bench] alias: tables {out['alias']['table_build_ms']:.2f} ms, sampling "
            f"{out['alias']['alias_sampling_ms']:.2f} ms vs {out['alias']['main_sampling_ms']:.2f} ms")
    if not args.no_accuracy:
        log("[bench] accuracy leg ...")
        out["accuracy"] = accuracy_leg()
        for gr in out["accuracy"]["graphs"]:
            log(f"[bench] accuracy {gr['graph'][:20]}: k=35000 mean rel err "
                + ", ".join(f"{x:.3f}" if x is not None else "-" for x in gr["by_k"][-1]["mean_rel_err"]))
    if not args.no_exact:
        log("[bench] exact leg ...")
        out["exact"] = exact_leg()
        log(f"[bench] exact: {out['exact']['exact_ms']:.1f} ms vs sampling {out['exact']['sampling_ms']:.2f} ms")
        out["exact_headline"] = exact_headline_leg(off, col, res, ms_per_step, stream)
        log(f"[bench] exact on the benchmark graph: {out['exact_headline']['exact_ms']:.0f} ms, estimates' rel err "
            + ", ".join(f"{x:.2e}" for x in out["exact_headline"]["rel_err"]))
    if not args.no_batched:
        log("[bench] batched leg ...")
        out["batched"] = batched_leg(args.batch_graphs, args.batch_k, replays=5)
    if not args.no_served:
        log("[bench] served leg ...")
        out["served"] = served_leg(args.served_graphs, args.served_sat, args.served_open,
                                   [float(x) for x in args.served_loads.split(",")], 0.01, 0.01,
                                   int(args.served_kmax), plain_check=min(8, args.served_sat))
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle on the benchmark graph) ...")
        off_h, col_h = off.cpu().numpy(), col.cpu().numpy()
        del off, col
        torch.cuda.empty_cache()
        cb = cpu_baseline(off_h, col_h, args.cpu_k, 1, gpu_cpu_tallies)
        cb["sample"] = cb["sample"].replace("{k}", str(k))
        out["cpu_baseline"] = cb
        log(f"[bench] cpu baseline: prep {cb['prep_s']:.1f} s, {cb['value']:.3e} samples/s, "
            f"bit-exact vs GPU: {cb['bit_exact_vs_gpu']}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
