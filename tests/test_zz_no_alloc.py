"""pm_count_noalloc, the allocation-free pm_count, against pm_count.

The entry point keeps every device buffer in a fixed per-device array of
the library (tallies and one draw-order sort chunk of 2^22 ids).  Two calls
in a row, through the C ABI: first a budget above the draw-order threshold
spanning several sort chunks with a ragged last one, then a smaller graph
and a smaller budget in id order; each must equal pm_count exactly (and the
second the oracle's tallies), which also shows the tallies left in the array
by the first call are cleared.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1411_4942_amd import pathsamp as ps
from paper_1411_4942_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def _graph(off, col):
    return ps.Graph(torch.from_numpy(np.ascontiguousarray(off, np.int64)).cuda(),
                    torch.from_numpy(np.ascontiguousarray(col, np.int32)).cuda())


def test_noalloc_equals_count_on_two_calls_the_second_smaller():
    # tallies (256 B), then one sort chunk of 2^22 ids: keys (4 B each),
    # bucketed pairs (8 B), sorted ids (4 B), two count tables of 256 tiles
    # x 2048 buckets (4 B), the bucket totals and starts (2048 and 2049
    # words, each slice rounded up to 256 B)
    c = 1 << 22
    assert ps.static_scratch_bytes() == 256 + (4 + 8 + 4) * c + 2 * 4 * 256 * 2048 + 4 * 2048 + 8448
    _say("noalloc: call 1, R-MAT scale 16, k = 2^23 + 777 per sampler (draw order, three sort chunks)")
    g1 = _graph(*synth.rmat(16, 16, seed=4))
    k1 = (1 << 23) + 777
    want1 = g1.count(k1, k1, seed=5, first_path=3, first_cent=2 ** 33)
    got1 = g1.count_noalloc(k1, k1, seed=5, first_path=3, first_cent=2 ** 33)
    assert got1 == want1
    _say("noalloc: call 2, ER G(2000, 20000), k = 50000 / 40000 (id order)")
    off2, col2 = synth.erdos_renyi(2000, 20000, 1)
    g2 = _graph(off2, col2)
    want2 = g2.count(50_000, 40_000, seed=9)
    got2 = g2.count_noalloc(50_000, 40_000, seed=9)
    assert got2 == want2
    og = oracle.Graph(off2, col2)
    assert got2["tally_path"] == og.sample_path(9, 50_000).tolist()
    assert got2["tally_cent"] == og.sample_centered(9, 40_000).tolist()
    g1.destroy()
    g2.destroy()


def test_noalloc_zero_weight_and_errors():
    _say("noalloc: star (W = 0) and argument errors")
    g = _graph(*synth.star(9))
    r = g.count_noalloc(1000, 1000, seed=1)
    assert r["tally_path"] == [0] * 8 and r["tally_cent"] == [0] * 8
    assert r == g.count(1000, 1000, seed=1)
    with pytest.raises(ps.PathSampError) as e:
        g.count_noalloc(0, 0)
    assert e.value.status == ps.PM_EINVAL
    with pytest.raises(ps.PathSampError) as e:
        g.count_noalloc(10, 10, delta=2.0)
    assert e.value.status == ps.PM_EINVAL
    g.destroy()
