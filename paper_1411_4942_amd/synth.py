"""Seeded synthetic graph inputs, as sorted CSR (int64 offsets, int32 columns).

This module only makes inputs: it holds none of the sampling method's
arithmetic, and both the HIP library and the CPU oracle consume what it
produces.  Every generator is deterministic in its seed.

The paper's own workloads are SNAP graphs read as edge lists with direction
ignored and duplicates dropped; heavy-tailed Chung-Lu and R-MAT graphs stand in
for them here, and Erdos-Renyi graphs give the small exact-count case.

numpy generators (PCG64) run anywhere; the ``*_torch`` variants build the
large graphs on a torch device (fast on a GPU; deterministic for a given
device type and seed).
"""
from __future__ import annotations

import math

import numpy as np


# --------------------------------------------------------------------------
# CSR assembly
# --------------------------------------------------------------------------

def csr_from_edges(n: int, u, v):
    """Symmetrise, drop self-loops and duplicates, sort rows.

    Returns (off int64[n+1], col int32[2m]).
    """
    u = np.asarray(u, dtype=np.int64).ravel()
    v = np.asarray(v, dtype=np.int64).ravel()
    keep = u != v
    u, v = u[keep], v[keep]
    a = np.minimum(u, v)
    b = np.maximum(u, v)
    key = np.unique(a * n + b)
    a = key // n
    b = key % n
    src = np.concatenate([a, b])
    dst = np.concatenate([b, a])
    order = np.lexsort((dst, src))
    src, dst = src[order], dst[order]
    off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(src, minlength=n), out=off[1:])
    return off, dst.astype(np.int32)


def num_edges(off) -> int:
    return int(off[-1]) // 2


def edges_of(off, col):
    """Undirected edge list (a < b) of a CSR."""
    off = np.asarray(off)
    n = off.size - 1
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(off))
    col = np.asarray(col, dtype=np.int64)
    keep = src < col
    return src[keep], col[keep]


def permute(off, col, perm):
    """The same graph with vertex v renamed perm[v]."""
    a, b = edges_of(off, col)
    perm = np.asarray(perm, dtype=np.int64)
    return csr_from_edges(off.size - 1, perm[a], perm[b])


# --------------------------------------------------------------------------
# small structured graphs
# --------------------------------------------------------------------------

def complete(n: int):
    a, b = np.triu_indices(n, 1)
    return csr_from_edges(n, a, b)


def cycle(n: int):
    a = np.arange(n)
    return csr_from_edges(n, a, (a + 1) % n)


def path(n: int):
    a = np.arange(n - 1)
    return csr_from_edges(n, a, a + 1)


def star(leaves: int):
    """K_{1,leaves}, hub is vertex 0 (the CSR written out directly)."""
    off = np.empty(leaves + 2, dtype=np.int64)
    off[0] = 0
    off[1:] = np.arange(leaves, 2 * leaves + 1, dtype=np.int64)
    col = np.zeros(2 * leaves, dtype=np.int32)
    col[:leaves] = np.arange(1, leaves + 1, dtype=np.int32)
    return off, col


def complete_bipartite(p: int, q: int):
    a, b = np.meshgrid(np.arange(p), np.arange(p, p + q), indexing="ij")
    return csr_from_edges(p + q, a.ravel(), b.ravel())


def empty(n: int):
    return np.zeros(n + 1, np.int64), np.zeros(0, np.int32)


def gnp(n: int, p: float, seed: int):
    rng = np.random.Generator(np.random.PCG64(seed))
    a, b = np.triu_indices(n, 1)
    keep = rng.random(a.size) < p
    return csr_from_edges(n, a[keep], b[keep])


# --------------------------------------------------------------------------
# random families
# --------------------------------------------------------------------------

def erdos_renyi(n: int, m: int, seed: int):
    """G(n, m): m distinct unordered non-loop pairs, uniformly (PCG64)."""
    if m > n * (n - 1) // 2:
        raise ValueError("too many edges")
    rng = np.random.Generator(np.random.PCG64(seed))
    keys = np.zeros(0, np.int64)
    while keys.size < m:
        need = m - keys.size
        u = rng.integers(0, n, size=2 * need + 16)
        v = rng.integers(0, n, size=2 * need + 16)
        ok = u != v
        a = np.minimum(u[ok], v[ok])
        b = np.maximum(u[ok], v[ok])
        new = a * n + b
        # keep first occurrences in draw order so the top-up is deterministic
        merged = np.concatenate([keys, new])
        _, idx = np.unique(merged, return_index=True)
        keys = merged[np.sort(idx)][:m]
    return csr_from_edges(n, keys // n, keys % n)


def hubs(hub_degrees, n_rest: int, m_rest: int, seed: int):
    """Hubs of exactly the given degrees over n_rest other vertices, plus
    m_rest random pairs among those others (repeats and loops dropped).

    Vertex ids: hubs first (0 .. len(hub_degrees) - 1), in the given order.
    Each hub's neighbours are distinct non-hub vertices, and no other edge
    touches a hub, so hub degrees are exact: graphs whose degree sequence hits
    chosen values (e.g. both sides of a size-class boundary).
    """
    rng = np.random.default_rng(seed)
    h = len(hub_degrees)
    n = h + n_rest
    us, vs = [], []
    for i, d in enumerate(hub_degrees):
        if d > n_rest:
            raise ValueError("hub degree above the number of other vertices")
        nb = rng.choice(n_rest, size=int(d), replace=False) + h
        us.append(np.full(int(d), i, dtype=np.int64))
        vs.append(nb.astype(np.int64))
    us.append(rng.integers(h, n, size=m_rest))
    vs.append(rng.integers(h, n, size=m_rest))
    return csr_from_edges(n, np.concatenate(us), np.concatenate(vs))


def chung_lu_weights(n: int, mean_degree: float, gamma: float, w_max: float):
    """w_i = min(w_max, w_min (1 - (i+1/2)/n)^(-1/(gamma-1))), w_min solved so
    that the mean weight is mean_degree (bisection)."""
    x = (1.0 - (np.arange(n) + 0.5) / n) ** (-1.0 / (gamma - 1.0))

    def mean_for(wmin):
        return float(np.minimum(w_max, wmin * x).mean())

    lo, hi = 1e-9, float(mean_degree)
    while mean_for(hi) < mean_degree:
        hi *= 2.0
    for _ in range(100):
        mid = 0.5 * (lo + hi)
        if mean_for(mid) < mean_degree:
            lo = mid
        else:
            hi = mid
    return np.minimum(w_max, hi * x)


def chung_lu(n: int, m: int, gamma: float, w_max: float, seed: int):
    """Chung-Lu graph with exactly m distinct undirected edges: endpoints
    drawn independently with probability proportional to the weights, loops
    and duplicates dropped, topped up until m edges exist."""
    if m > n * (n - 1) // 4:
        raise ValueError("too many edges for n")
    w = chung_lu_weights(n, 2.0 * m / n, gamma, w_max)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    rng = np.random.Generator(np.random.PCG64(seed))
    keys = np.zeros(0, np.int64)
    rounds = 0
    while keys.size < m:
        need = m - keys.size
        draw = int(need * 1.1) + 64
        u = np.minimum(np.searchsorted(cdf, rng.random(draw), side="right"), n - 1)
        v = np.minimum(np.searchsorted(cdf, rng.random(draw), side="right"), n - 1)
        ok = u != v
        a = np.minimum(u[ok], v[ok])
        b = np.maximum(u[ok], v[ok])
        merged = np.concatenate([keys, a * n + b])
        _, idx = np.unique(merged, return_index=True)
        keys = merged[np.sort(idx)][:m]
        rounds += 1
        if rounds > 1000:
            raise RuntimeError("chung_lu: could not reach m distinct edges")
    return csr_from_edges(n, keys // n, keys % n)


def rmat(scale: int, edge_factor: float, abcd=(0.57, 0.19, 0.19, 0.05), seed: int = 1):
    """R-MAT (Chakrabarti, Zhan, Faloutsos): edge_factor * 2^scale directed
    draws, each bit level picks a quadrant with probabilities (a, b, c, d);
    then symmetrised, loops and duplicates dropped (no noise, no shuffle)."""
    n = 1 << scale
    ne = int(edge_factor * n)
    a, b, c, _ = abcd
    rng = np.random.Generator(np.random.PCG64(seed))
    u = np.zeros(ne, np.int64)
    v = np.zeros(ne, np.int64)
    for level in range(scale):
        r = rng.random(ne)
        ubit = r >= a + b                      # quadrants c, d
        vbit = ((r >= a) & (r < a + b)) | (r >= a + b + c)  # quadrants b, d
        u |= ubit.astype(np.int64) << level
        v |= vbit.astype(np.int64) << level
    return csr_from_edges(n, u, v)


# --------------------------------------------------------------------------
# torch variants for large inputs (built where the tensors live)
# --------------------------------------------------------------------------

def _csr_from_edges_torch(n: int, u, v):
    import torch

    keep = u != v
    u, v = u[keep], v[keep]
    a = torch.minimum(u, v)
    b = torch.maximum(u, v)
    key = torch.unique(a * n + b)  # sorted, distinct
    del a, b, u, v
    a = key // n
    b = key - a * n
    del key
    src = torch.cat([a, b])
    dst = torch.cat([b, a])
    del a, b
    skey = src * n + dst
    del src, dst
    skey, _ = torch.sort(skey)
    src = skey // n
    col = (skey - src * n).to(torch.int32)
    del skey
    counts = torch.bincount(src, minlength=n)
    del src
    off = torch.zeros(n + 1, dtype=torch.int64, device=col.device)
    torch.cumsum(counts, 0, out=off[1:])
    return off, col


def rmat_torch(scale: int, edge_factor: float, abcd=(0.57, 0.19, 0.19, 0.05), seed: int = 1,
               device="cuda", chunk: int = 1 << 25):
    """R-MAT as :func:`rmat`, drawn with torch's generator on ``device``."""
    u, v = rmat_edges_torch(scale, edge_factor, abcd, seed, device, chunk)
    return _csr_from_edges_torch(1 << scale, u, v)


def rmat_edges_torch(scale: int, edge_factor: float, abcd=(0.57, 0.19, 0.19, 0.05), seed: int = 1,
                     device="cuda", chunk: int = 1 << 25):
    """The raw directed R-MAT draws (int64 u, v) behind :func:`rmat_torch`:
    loops and repeats included, not symmetrised."""
    import torch

    n = 1 << scale
    ne = int(edge_factor * n)
    a, b, c, _ = abcd
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    us, vs = [], []
    for start in range(0, ne, chunk):
        cnt = min(chunk, ne - start)
        u = torch.zeros(cnt, dtype=torch.int64, device=device)
        v = torch.zeros(cnt, dtype=torch.int64, device=device)
        for level in range(scale):
            r = torch.rand(cnt, generator=gen, device=device)
            ubit = r >= a + b
            vbit = ((r >= a) & (r < a + b)) | (r >= a + b + c)
            u |= ubit.to(torch.int64) << level
            v |= vbit.to(torch.int64) << level
        us.append(u)
        vs.append(v)
    u = torch.cat(us)
    v = torch.cat(vs)
    del us, vs
    return u, v


def chung_lu_torch(n: int, m: int, gamma: float, w_max: float, seed: int, device="cuda"):
    """Chung-Lu as :func:`chung_lu` (exactly m edges), drawn with torch."""
    import torch

    if m > n * (n - 1) // 4:
        raise ValueError("too many edges for n")
    w = torch.from_numpy(chung_lu_weights(n, 2.0 * m / n, gamma, w_max)).to(device)
    cdf = torch.cumsum(w, 0)
    cdf = cdf / cdf[-1]
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    keys = torch.zeros(0, dtype=torch.int64, device=device)
    rounds = 0
    while keys.numel() < m:
        need = m - keys.numel()
        draw = int(need * 1.1) + 64
        u = torch.searchsorted(cdf, torch.rand(draw, generator=gen, device=device, dtype=torch.float64),
                               right=True).clamp_(max=n - 1)
        v = torch.searchsorted(cdf, torch.rand(draw, generator=gen, device=device, dtype=torch.float64),
                               right=True).clamp_(max=n - 1)
        ok = u != v
        a = torch.minimum(u[ok], v[ok])
        b = torch.maximum(u[ok], v[ok])
        new = a * n + b
        merged = torch.cat([keys, new])
        uniq, inv = torch.unique(merged, return_inverse=True)
        # first occurrence of each key, in draw order
        first = torch.full((uniq.numel(),), merged.numel(), dtype=torch.int64, device=device)
        first.scatter_reduce_(0, inv, torch.arange(merged.numel(), device=device), reduce="amin")
        keys = merged[torch.sort(first).values][:m]
        rounds += 1
        if rounds > 1000:
            raise RuntimeError("chung_lu_torch: could not reach m distinct edges")
    return _csr_from_edges_torch(n, keys // n, keys % n)
