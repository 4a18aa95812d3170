#!/usr/bin/env python3
"""Benchmark: the whole 3-path sampling hot path on one MI355X.

One step = prepare the graph from its device-resident CSR (validation,
degree-order relabel, tau/lambda prefix sums, N_1, guide tables), run both
samplers with k samples each, and finalize estimates with 99% error bars.
Workload: R-MAT scale 22 (a, b, c, d) = (0.57, 0.19, 0.19, 0.05), symmetrised
and deduplicated (about 1.2e8 undirected edges), k = 1e7 samples per sampler,
Philox seed 1.  value = samples per step (2k) / step time.

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


def roofline_for(name, kern, alg_entry, traffic):
    alg_bytes, symbol = alg_entry
    achieved = alg_bytes / (kern["avg_ms"] * 1e-3) / 1e9
    tr = None
    if traffic:
        cands = [v for key, v in traffic["kernels"].items() if key.startswith(symbol)]
        if cands:
            best = max(cands, key=lambda v: v["fetch_bytes"])
            tr = best["fetch_bytes"] + best["write_bytes"]
    return {"bound": "hbm", "kernel": name, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": tr, "algorithmic_bytes": alg_bytes,
            "avg_launch_ms": kern["avg_ms"],
            "traffic_over_algorithmic": (tr / alg_bytes) if tr else None}


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


def cpu_baseline(scale: int, edge_factor: float, k: int, seed: int) -> dict:
    """The oracle (single thread) on a bounded sample of the workload: an
    R-MAT graph of the same family at a smaller scale, k scaled by the same
    factor as the edges, whole job (prep + both samplers)."""
    import oracle
    from paper_1411_4942_amd import synth

    off, col = synth.rmat(scale, edge_factor, seed=seed)
    t0 = time.perf_counter()
    g = oracle.Graph(off, col)
    t1 = time.perf_counter()
    g.sample_path(1, k)
    g.sample_centered(1, k)
    t2 = time.perf_counter()
    return {
        "value": 2 * k / (t2 - t0),
        "unit": "samples/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"R-MAT scale {scale} (same a,b,c,d and edge factor {edge_factor}, 2m={off[-1]}), "
                  f"k={k} per sampler, prep {t1 - t0:.2f}s + sampling {t2 - t1:.2f}s, single thread",
        "sampling_only_samples_per_s": 2 * k / (t2 - t1),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--scale", type=int, default=22)
    ap.add_argument("--edge-factor", type=float, default=31.0)
    ap.add_argument("--k", type=int, default=10_000_000)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--cpu-scale", type=int, default=18)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build runs on single-GPU boxes "
              "(the multi-GPU sharding is described, not built).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1411_4942_amd import pathsamp as ps

    torch.cuda.set_device(0)
    ps.lib()
    off, col = make_graph(args.scale, args.edge_factor, args.seed)
    stream = torch.cuda.current_stream()
    k = args.k

    def step():
        g = ps.Graph(off, col, stream=stream)
        res = g.count(k, k, seed=1, stream=stream)
        info = g.info()
        g.destroy()
        return res, info

    for i in range(args.warmup):
        t0 = time.perf_counter()
        res, info = step()
        log(f"[bench] warmup {i}: {1e3 * (time.perf_counter() - t0):.1f} ms")

    ps.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        res, info = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ps.profile_read()
    ps.profile_enable(False)
    ms_per_step = 1e3 * (t1 - t0) / args.steps
    value = 2 * k / ((t1 - t0) / args.steps)
    log(f"[bench] {args.steps} steps: {ms_per_step:.2f} ms/step")

    # per-kernel averages (HIP events on the launch stream)
    kernels = {name: {"launches": n, "avg_ms": ms / n, "ms_per_step": ms / args.steps}
               for name, (n, ms) in prof.items()}
    slots = 2 * info["m"]
    # algorithmic bytes per launch of the kernels the roofline can name
    alg = {
        "sample_path": (BYTES_PER_SAMPLE * k, "pm::k_sample<false,"),
        "sample_centered": (BYTES_PER_SAMPLE * k, "pm::k_sample<true,"),
        # one pass: read key + value, write key + value (the last pass of the
        # transpose sort writes the interleaved edge array instead of the keys)
        "transpose_sort.scatter": (16 * slots, "pm::radix_scatter"),
        "reverse_sort.scatter": (16 * slots, "pm::radix_scatter"),
    }
    traffic = load_traffic()
    timed = {n: v for n, v in kernels.items() if n in alg}
    dom_name = max(timed, key=lambda n: timed[n]["ms_per_step"])
    roofline = roofline_for(dom_name, kernels[dom_name], alg[dom_name], traffic)
    roofline_sampler = roofline_for("sample_path", kernels["sample_path"], alg["sample_path"], traffic)
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
                        f"symmetrised+dedup; k={k} 3-path + {k} centered samples, Philox seed 1",
            "n": info["n"], "m": info["m"], "dmax": info["dmax"], "isolated": info["isolated"],
            "W": info["W"], "Lambda": info["Lambda"], "N1": info["N1"],
            "samples_per_step": 2 * k,
            "parallelism": "single GPU",
        },
        "roofline": roofline,
        "roofline_sampler": roofline_sampler,
        "kernels": kernels,
        "sampling_samples_per_s": 2 * k / (sum(samp_ms) * 1e-3),
        "estimates": res["est"][1:],
        "rel_bar_halfwidth": [((h - l) / 2 / e if e else None) for e, l, h in zip(res["est"][1:], res["lo"][1:], res["hi"][1:])],
    }
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        kc = max(1, int(k * (2 ** args.cpu_scale) / (2 ** args.scale)))
        out["cpu_baseline"] = cpu_baseline(args.cpu_scale, args.edge_factor, kc, args.seed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
