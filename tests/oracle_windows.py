"""Oracle tallies of long id ranges on several host threads.

Tallies are sums over sample ids (each sample depends only on seed, sampler
and id), so the range [first, first + k) splits into windows that the
single-threaded oracle runs side by side: ctypes releases the interpreter
lock during each call.  Test infrastructure only.
"""
import ctypes
import os
from concurrent.futures import ThreadPoolExecutor

import oracle


def workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def window_tally(g, centered: bool, seed: int, first: int, k: int):
    """One oracle call over ids [first, first + k) of the oracle graph struct g."""
    lib = oracle._load()
    t = (ctypes.c_uint64 * 8)()
    fn = lib.or_sample_centered if centered else lib.or_sample_path
    fn(ctypes.byref(g), ctypes.c_uint64(seed), ctypes.c_uint64(first), ctypes.c_uint64(k), t)
    return [int(x) for x in t]


def tally(g, centered: bool, seed: int, k: int, first: int = 0, windows: int = 64, pool=None):
    """Tallies of ids [first, first + k) as a sum over id windows."""
    if k == 0:
        return [0] * 8
    step = max(1, (k + windows - 1) // windows)
    parts = [(first + f, min(step, k - f)) for f in range(0, k, step)]
    if pool is None:
        with ThreadPoolExecutor(max_workers=workers()) as ex:
            outs = list(ex.map(lambda fw: window_tally(g, centered, seed, fw[0], fw[1]), parts))
    else:
        outs = list(pool.map(lambda fw: window_tally(g, centered, seed, fw[0], fw[1]), parts))
    return [sum(t[c] for t in outs) for c in range(8)]
