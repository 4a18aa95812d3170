"""Pins for the oracle's estimates and error bars (Algorithms 2 and 4,
Section 5), and for the constants A_{2,i} / B_i against the paper's tables."""
import math
import os

import numpy as np
import pytest
from scipy import special, stats

import oracle
from oracle import finalize
from paper_1411_4942_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def _kl(a, b):
    # independent evaluation of the Bernoulli KL divergence
    return float(special.rel_entr(a, b) + special.rel_entr(1 - a, 1 - b))


@pytest.mark.parametrize("count,k", [(1, 10), (5, 100), (500, 1000), (99, 100), (3, 200000), (123456, 200000)])
@pytest.mark.parametrize("delta", [0.01, 0.05])
def test_chernoff_roots_solve_definition(count, k, delta):
    pl, pu = finalize.chernoff_interval(count, k, delta)
    alpha = count / k
    assert 0 < pl < alpha < pu < 1
    target = math.log(1 / delta) / k
    assert _kl(alpha, pl) == pytest.approx(target, rel=1e-9)
    assert _kl(alpha, pu) == pytest.approx(target, rel=1e-9)


def test_chernoff_edge_outcomes():
    k, delta = 1000, 0.01
    pl, pu = finalize.chernoff_interval(0, k, delta)
    assert pl == 0.0
    assert (1 - pu) ** k == pytest.approx(delta, rel=1e-9)  # P[X = 0 | p_u] = delta
    pl, pu = finalize.chernoff_interval(k, k, delta)
    assert pu == 1.0
    assert pl ** k == pytest.approx(delta, rel=1e-9)


@pytest.mark.parametrize("count,k", [(0, 50), (7, 50), (30, 50), (50, 50), (40, 2000), (1900, 2000)])
def test_corollary_5_3_outside_the_bar(count, k):
    """Corollary 5.3: for p outside [p_l, p_u], Pr[X/k = alpha] <= delta."""
    delta = 0.01
    pl, pu = finalize.chernoff_interval(count, k, delta)
    for p in np.concatenate([np.linspace(0, pl, 20, endpoint=False)[1:], np.linspace(pu, 1, 20)[1:-1]]):
        if p <= 0 or p >= 1:
            continue
        assert stats.binom.pmf(count, k, p) <= delta * (1 + 1e-9)


def test_bars_cover_the_truth():
    rng = np.random.default_rng(5)
    k, delta, trials = 5000, 0.01, 3000
    miss = 0
    for _ in range(trials):
        p = float(rng.uniform(0.001, 0.3))
        x = int(rng.binomial(k, p))
        pl, pu = finalize.chernoff_interval(x, k, delta)
        miss += not (pl <= p <= pu)
    assert miss / trials <= 0.02


def _tables():
    rows = []
    with open(os.path.join(HERE, "golden", "tables_2_3.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                parts = line.split()
                rows.append((parts[0], [float(x) for x in parts[1:]]))
    return rows


@pytest.mark.parametrize("name,vals", _tables(), ids=[r[0] for r in _tables()])
def test_paper_tables_agree_with_the_coefficients(name, vals):
    """W = sum_i A_{2,i} C_i + 3T with 3T >= 0 small (Eq. 1 row 2, Claim 3.1),
    and Lambda >= sum_i B_i C_i (Lemma 4.2, Claim 4.3), on the paper's
    printed numbers (3 significant figures)."""
    W, Lam, *C = vals
    C = [0.0] + C
    paths = sum(finalize.A2[i] * C[i] for i in range(2, 7))
    assert 0.98 <= paths / W <= 1.01
    centered = sum(finalize.B[i] * C[i] for i in (4, 5, 6))
    assert centered / Lam <= 1.01


def test_star_and_cycle_estimates_are_exact():
    off, col = synth.star(20)
    g = oracle.Graph(off, col)
    res = finalize.finalize(g.sample_path(1, 10), g.sample_centered(1, 10), g.R_tau, g.R_lam, g.N1, 10, 10)
    assert res["est"][1] == math.comb(20, 3)
    assert res["lo"][1] == res["hi"][1] == math.comb(20, 3)
    assert res["est"][2:] == [0.0] * 5


def test_config1_estimates_within_one_percent_where_feasible():
    """ER G(2000, 20000), k = 100000 per sampler, Philox seed 1: the 3-star and
    3-path (the motifs Corollary 5.3 can resolve to 1% at this k) within 1%
    of the exact counts; every motif inside its 99% bar."""
    off, col = synth.erdos_renyi(2000, 20000, 1)
    C, T = oracle.exact_formula(off, col)
    res = oracle.count_motifs(off, col, k=100_000, seed=1)
    for i in (1, 2):
        assert abs(res["est"][i] - C[i]) <= 0.01 * C[i], i
    for i in range(1, 7):
        assert res["lo"][i] - 1e-6 <= C[i] <= res["hi"][i] + 1e-6, (i, res["lo"][i], C[i], res["hi"][i])
