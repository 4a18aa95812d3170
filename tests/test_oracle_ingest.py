"""The oracle's edge-list clean-up against graphs built independently."""
import numpy as np
import pytest

from oracle import ingest
from paper_1411_4942_amd import synth


def _same(a, b):
    return np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_complete_graph_from_every_ordered_pair_with_loops():
    n = 9
    src, dst = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    src = np.concatenate([src.ravel(), src.ravel()])  # every pair twice, both directions, and loops
    dst = np.concatenate([dst.ravel(), dst.ravel()])
    assert _same(ingest.csr_from_edges(n, src, dst), synth.complete(n))


def test_cycle_star_path_and_isolated_vertices():
    n = 12
    c = np.arange(n)
    assert _same(ingest.csr_from_edges(n, c, (c + 1) % n), synth.cycle(n))
    assert _same(ingest.csr_from_edges(n, (c + 1) % n, c), synth.cycle(n))
    assert _same(ingest.csr_from_edges(8, np.zeros(7, int), np.arange(1, 8)), synth.star(7))
    off, col = ingest.csr_from_edges(10, [0, 1], [1, 0])
    assert off.tolist() == [0, 1, 2] + [2] * 8 and col.tolist() == [1, 0]
    off, col = ingest.csr_from_edges(4, [], [])
    assert off.tolist() == [0] * 5 and col.size == 0


@pytest.mark.parametrize("seed", range(6))
def test_random_lists_match_the_generator_builder(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 300))
    e = int(rng.integers(0, 3000))
    src = rng.integers(0, n, e)
    dst = rng.integers(0, n, e)
    keep = src != dst
    want = synth.csr_from_edges(n, src[keep], dst[keep])
    assert _same(ingest.csr_from_edges(n, src, dst), want)


def test_out_of_range_is_refused():
    with pytest.raises(ValueError):
        ingest.csr_from_edges(3, [0], [3])
