"""bench.py end to end on a small graph: the JSON line it prints parses and
carries the keys of its contract (the full-size run is the benchmark itself;
this catches a broken report before it)."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_prints_one_json_line():
    print("[test] bench.py on R-MAT scale 14", flush=True)
    cmd = [sys.executable, "-u", os.path.join(ROOT, "bench.py"), "--scale", "14", "--edge-factor", "16",
           "--k", "300000", "--steps", "2", "--warmup", "1", "--whole-steps", "1", "--no-cpu-baseline",
           "--no-batched", "--no-served", "--no-ingest", "--no-exact", "--no-alias", "--no-accuracy"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=240, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-3000:]
    lines = [l for l in r.stdout.splitlines() if l.strip()]
    assert len(lines) == 1, r.stdout[-2000:]
    out = json.loads(lines[0])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
                "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "prep_ms", "whole_job"):
        assert key in out, key
    assert out["n_gpus"] == 1 and out["steps"] == 2 and out["warmup"] == 1
    assert out["value"] > 0 and out["ms_per_step"] > 0 and out["prep_ms"] > 0
    assert out["roofline"]["peak"] > 0 and out["roofline"]["achieved"] > 0
    assert "workload" in out["config"]
