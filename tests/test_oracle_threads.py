"""The oracle may prepare several graphs on host threads at once (the
full-size GPU tests do): each build must equal the same build run alone.
The degree-order sort and the exact counter's vertex order keep their
comparator state per thread."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle
from paper_1411_4942_amd import synth


def _graphs():
    out = []
    for s in range(12):
        # different sizes and degree profiles, many isolated vertices in some
        out.append(synth.chung_lu(3000 + 4000 * s, 4000 + 3000 * s, 2.1 + 0.05 * s, 80.0 + 20 * s, 700 + s))
    return out


def _build(csr):
    g = oracle.Graph(*csr)
    return g.rank, g.col, g.p_tau, g.p_lam, g.R_lam


def test_concurrent_builds_equal_sequential():
    gs = _graphs()
    alone = [_build(c) for c in gs]
    for _ in range(3):
        with ThreadPoolExecutor(max_workers=8) as ex:
            together = list(ex.map(_build, gs))
        for a, b in zip(alone, together):
            for x, y in zip(a[:4], b[:4]):
                assert np.array_equal(x, y)
            assert a[4] == b[4]


def test_concurrent_exact_counts_equal_sequential():
    gs = _graphs()[:6]
    alone = [oracle.exact_formula(*c) for c in gs]
    with ThreadPoolExecutor(max_workers=6) as ex:
        together = list(ex.map(lambda c: oracle.exact_formula(*c), gs))
    assert alone == together
