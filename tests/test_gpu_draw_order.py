"""pm_draw_order: the order in which a draw-ordered launch runs its samples.

The draw-ordered samplers sort each chunk of sample ids by the top 24 bits
of the sample's first draw r (Algorithm 1 step 2 / Algorithm 3 step 2), with
a two-level counting sort (2048 high-digit buckets, then each bucket by its
low digit).  The order among equal keys is free, so these tests check what
is unique: the ids are a permutation of the chunk, and the keys the oracle
draws for them (oracle.draws, each r computed from scratch on the CPU) are
nondecreasing in that order.  Cases: a graph whose keys are full 24-bit
prefixes of r over a ragged number of tiles, both samplers; small total
weights whose keys are all of r (no low digit; a one-bit low digit); and a
chunk of 2^24 samples over about a thousand buckets, where buckets exceed
the size ordered in LDS and take the counting path with 32-bit counters.
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


def _keys(seed, centered, first, k, R):
    """The draw keys of samples first .. first + k - 1, from the oracle's draws."""
    rbits = int(R - 1).bit_length()
    shift = max(rbits - 24, 0)
    r = oracle.draws(seed, 1 if centered else 0, first, k, R)
    return r >> np.uint64(shift)


def _check_order(g, og, centered, seed, k, first):
    R = og.R_lam if centered else og.R_tau
    ids = g.draw_order(centered, seed, k, first).cpu().numpy().astype(np.int64)
    assert ids.shape == (k,)
    assert ids.min() >= 0 and ids.max() < k
    assert np.array_equal(np.bincount(ids, minlength=k), np.ones(k, np.int64)), "not a permutation of the chunk"
    keys = _keys(seed, centered, first, k, R)[ids]
    assert np.all(keys[1:] >= keys[:-1]), "keys decrease along the order"
    return keys


@pytest.mark.parametrize("centered", [False, True])
def test_rmat_full_keys_ragged_tiles(centered):
    off, col = synth.rmat(12, 8, seed=3)
    og = oracle.Graph(off, col)
    R = og.R_lam if centered else og.R_tau
    assert R - 1 >= 1 << 24  # keys are the top 24 bits of r: both digits in use
    g = _graph(off, col)
    k = 19 * 16384 + 4321  # 20 tiles, the last ragged
    first = 5 if not centered else 2 ** 33 + 7
    _say("draw order: R-MAT 12", "centered" if centered else "3-path", "k", k, "first", first)
    keys = _check_order(g, og, centered, 11, k, first)
    assert len(np.unique(keys >> np.uint64(13))) > 1000  # many buckets filled
    g.destroy()


@pytest.mark.parametrize("k", [1, 2, 3, 16384, 16385])
def test_tiny_and_tile_edge_chunks(k):
    # one sample, two, three; exactly one tile, one tile and one sample
    off, col = synth.rmat(10, 8, seed=5)
    og = oracle.Graph(off, col)
    g = _graph(off, col)
    _say("draw order: R-MAT 10, k", k)
    _check_order(g, og, False, 2, k, 40)
    _check_order(g, og, True, 2, k, 40)
    g.destroy()


@pytest.mark.parametrize("n,k", [(500, 100_000), (1500, 200_003)])
def test_small_weight_keys_are_all_of_r(n, k):
    # a cycle: every slot has weight 1, R = 2n; keys of 10 bits take the
    # buckets alone, keys of 12 bits leave a one-bit low digit
    off, col = synth.cycle(n)
    og = oracle.Graph(off, col)
    assert og.R_tau == 2 * n
    g = _graph(off, col)
    _say("draw order: cycle", n, "k", k)
    keys = _check_order(g, og, False, 3, k, 0)
    assert keys.max() < 2 * n
    g.destroy()


def test_full_chunk_with_buckets_above_the_lds_size():
    # R = 4098: 13-bit keys, 2-bit low digit, 1025 buckets of about 16.4K
    # samples each at k = 2^24 (above the 16384 ordered in LDS)
    off, col = synth.cycle(2049)
    og = oracle.Graph(off, col)
    assert og.R_tau == 4098
    g = _graph(off, col)
    k = 1 << 24
    _say("draw order: cycle 2049, k = 2^24")
    keys = _check_order(g, og, False, 9, k, 1000)
    sizes = np.bincount((keys >> np.uint64(2)).astype(np.int64))
    assert sizes.max() > 16384
    g.destroy()


def test_errors():
    off, col = synth.cycle(50)
    g = _graph(off, col)
    _say("draw order: argument errors")
    for k in (0, (1 << 24) + 1):
        with pytest.raises(ps.PathSampError):
            g.draw_order(False, 1, k)
    g.destroy()
    s = _graph(*synth.star(6))  # W = 0: no 3-path draws
    with pytest.raises(ps.PathSampError):
        s.draw_order(False, 1, 1000)
    s.destroy()


def test_default_threshold_is_2_pow_21():
    # pm_count sorts a sampler's ids from 2^21 samples on (the default of
    # pm_set_draw_order); below, the samples run in id order.  Tallies are
    # the same either way, so the launch is told apart by its timed scopes.
    off, col = synth.rmat(10, 8, seed=5)
    g = _graph(off, col)
    ps.set_draw_order(True, 0)
    runs = {}
    try:
        for k in ((1 << 21) - 1, 1 << 21):
            _say("draw order: default threshold, k", k)
            ps.profile_enable(True)
            r = g.count(k, k, seed=3)
            torch.cuda.synchronize()
            runs[k] = (ps.profile_read(), r)
            ps.profile_enable(False)
    finally:
        ps.profile_enable(False)
    below, at = runs[(1 << 21) - 1][0], runs[1 << 21][0]
    assert "sample_path.sorted" not in below and "draw_sort.keys" not in below
    assert below["sample_path"][0] == 1
    assert at["sample_path.sorted"][0] == 1 and at["sample_centered.sorted"][0] == 1
    assert at["draw_sort.keys"][0] == 2  # one sort per sampler
    g.destroy()
