"""Seeded synthetic workloads for the batched and served measurements.

Only graph recipes live here (no step of the method): sizes, generator seeds
and Philox seeds of the many-graph pools, drawn on the device with the torch
generators of :mod:`synth`.
"""
from __future__ import annotations

import math

import numpy as np

from . import synth


def batched_specs(count: int = 256, seed: int = 1):
    """Chung-Lu graphs for the batched run: n log-uniform in [1e3, 2e5],
    m log-uniform in [5e3, 2e6] clamped to n(n-1)/4, degree exponent uniform in
    [2.1, 2.8], weight cap min(n-1, sqrt(2m)); graph g uses generator seed
    1000+g and Philox seed 1+g."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for g in range(count):
        n = int(round(math.exp(rng.uniform(math.log(1e3), math.log(2e5)))))
        m = int(round(math.exp(rng.uniform(math.log(5e3), math.log(2e6)))))
        m = min(m, n * (n - 1) // 4)
        gamma = float(rng.uniform(2.1, 2.8))
        w_max = min(n - 1.0, math.sqrt(2.0 * m))
        out.append(dict(kind="chung_lu", n=n, m=m, gamma=gamma, w_max=w_max, gen_seed=1000 + g, philox_seed=1 + g))
    return out


def served_specs(count: int = 64, seed: int = 1, m_lo: float = 1e4, m_hi: float = 5e7):
    """Pool of the served run: half R-MAT (0.57, 0.19, 0.19, 0.05) with the
    scale chosen so the edge factor lies in [16, 32], half Chung-Lu with
    exponent 2.3, mean degree 20 and weight cap min(n-1, sqrt(2m)); target m
    log-uniform in [m_lo, m_hi]; graph g uses generator seed 5000+g."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for g in range(count):
        m = int(round(math.exp(rng.uniform(math.log(m_lo), math.log(m_hi)))))
        if g % 2 == 0:
            # about 0.9 of the directed draws survive symmetrise + dedup
            scale = max(6, math.ceil(math.log2(m / (32 * 0.9))))
            ef = min(32.0, max(16.0, m / (0.9 * (1 << scale))))
            out.append(dict(kind="rmat", scale=scale, edge_factor=ef, m_target=m, gen_seed=5000 + g))
        else:
            n = max(100, m // 10)
            out.append(dict(kind="chung_lu", n=n, m=m, gamma=2.3, w_max=min(n - 1.0, math.sqrt(2.0 * m)),
                            gen_seed=5000 + g))
    return out


def build(spec: dict, device="cuda"):
    """CSR (int64 offsets, int32 columns) of one spec, on ``device``."""
    if spec["kind"] == "rmat":
        return synth.rmat_torch(spec["scale"], spec["edge_factor"], seed=spec["gen_seed"], device=device)
    return synth.chung_lu_torch(spec["n"], spec["m"], spec["gamma"], spec["w_max"], spec["gen_seed"], device=device)
