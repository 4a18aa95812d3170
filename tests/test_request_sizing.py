"""The served mode's sample sizing (Corollary 5.3 applied to pilot tallies).

The library's host function against the oracle's restatement of the rule,
and the rule against what it promises, checked through the interval
root-finder of Definition 5.2 rather than the closed form: at the sized k the
bar of the pilot's proportion lies inside the relative-error band, one sample
fewer it does not.  Host arithmetic only; no device call.
"""
import math

import numpy as np
import pytest

from oracle import finalize as ofin
from paper_1411_4942_amd import pathsamp as ps

K0 = 65536


def _pilot(rng):
    tp = [0] * 8
    tc = [0] * 8
    p = rng.dirichlet(np.ones(6))
    x = rng.multinomial(K0, p)
    tp[0], tp[2], tp[3], tp[4], tp[5], tp[6] = (int(v) for v in x)
    q = rng.dirichlet(np.ones(5))
    y = rng.multinomial(K0, q)
    tc[0], tc[1], tc[4], tc[5], tc[6] = (int(v) for v in y)
    if rng.random() < 0.3:  # a motif without hits
        i = int(rng.integers(2, 7))
        tp[0] += tp[i]
        tp[i] = 0
    if rng.random() < 0.3:
        i = int(rng.integers(4, 7))
        tc[1] += tc[i]
        tc[i] = 0
    return tp, tc


def _band_ok(alpha, k, eps, delta):
    pl, pu = ofin.chernoff_interval_alpha(alpha, k, delta)
    return pl >= alpha * (1 - eps) and (pu <= alpha * (1 + eps) or alpha * (1 + eps) >= 1.0)


def test_library_matches_oracle_rule():
    rng = np.random.default_rng(7)
    for _ in range(300):
        tp, tc = _pilot(rng)
        W = int(rng.integers(1, 2 ** 50))
        Lam = int(rng.integers(0, 2 ** 45)) if rng.random() < 0.9 else 0
        N1 = int(W * rng.uniform(0.5, 50))
        mask = int(rng.integers(0, 128)) & 0x7E
        eps = float(rng.choice([0.01, 0.05, 0.2]))
        delta = float(rng.choice([0.01, 0.001, 0.1]))
        k_max = int(rng.choice([K0, 10 ** 7, 2 * 10 ** 9]))
        got = ps.samples_for_request(tp, tc, K0, W, Lam, N1, mask, eps, delta, k_max)
        want = ofin.samples_for_request(tp, tc, K0, W, Lam, N1, mask, eps, delta, k_max)
        assert got[2:] == want[2:]
        for a, b in zip(got[:2], want[:2]):
            assert abs(a - b) <= 1 + 1e-12 * b  # one rounding of a log apart at most


@pytest.mark.parametrize("i", [2, 3, 4, 5, 6])
def test_single_motif_k_is_the_smallest_inside_the_band(i):
    rng = np.random.default_rng(100 + i)
    for _ in range(20):
        tp, tc = _pilot(rng)
        t = (tp if i <= 3 else tc)[i]
        if t == 0:
            continue
        eps, delta = 0.01, 0.01
        kp, kc, capped, unseen = ps.samples_for_request(tp, tc, K0, 10 ** 12, 10 ** 11, 10 ** 13, 1 << i, eps,
                                                        delta, 2 ** 62)
        k = kp if i <= 3 else kc
        other = kc if i <= 3 else kp
        assert other == K0 and capped == 0 and unseen == 0
        alpha = t / K0
        if k == K0:
            assert _band_ok(alpha, K0, eps, delta)
            continue
        assert _band_ok(alpha, k, eps, delta)
        assert not _band_ok(alpha, k - 1, eps, delta)


def test_unseen_motif_sized_from_upper_root():
    tp = [1000, 0, K0 - 1000, 0, 0, 0, 0, 0]
    tc = [10, K0 - 10, 0, 0, 0, 0, 0, 0]
    kp, kc, capped, unseen = ps.samples_for_request(tp, tc, K0, 10 ** 9, 10 ** 9, 10 ** 10, 1 << 4, 0.05, 0.01,
                                                    2 ** 62)
    assert unseen == 1 << 4 and capped == 0 and kp == K0
    _, pu = ofin.chernoff_interval(0, K0, 0.01)
    assert _band_ok(pu, kc, 0.05, 0.01) and not _band_ok(pu, kc - 1, 0.05, 0.01)


def test_cap_and_flags():
    tp = [0, 0, K0 - 3, 3, 0, 0, 0, 0]
    tc = [0, K0 - 1, 0, 0, 1, 0, 0, 0]
    kp, kc, capped, unseen = ps.samples_for_request(tp, tc, K0, 10 ** 9, 10 ** 9, 10 ** 12, 0, 0.01, 0.01, 10 ** 7)
    assert kp == 10 ** 7 and kc == 10 ** 7
    assert capped & (1 << 3) and capped & (1 << 4)
    assert unseen == (1 << 5) | (1 << 6)  # motifs 5, 6 on the centered sampler (tp[5], tp[6] are 0 too)


def test_zero_weight_samplers_get_k0():
    kp, kc, capped, unseen = ps.samples_for_request([0] * 8, [0] * 8, K0, 0, 0, 35, 0, 0.01, 0.01, 10 ** 9)
    assert (kp, kc, capped, unseen) == (K0, K0, 0, 0)


def test_three_star_bar_within_its_share():
    """Motif 1 alone: at the sized k, the bar of N_1 - C_3 - 2 C_5 - 4 C_6
    (errors added up, Corollary 5.3 remark) around the pilot estimate is within
    rel_err of it, computed with the interval root-finder."""
    rng = np.random.default_rng(5)
    W = 10 ** 9
    for _ in range(30):
        tp, tc = _pilot(rng)
        est = {j: tp[j] * W / (K0 * ofin.A2[j]) for j in (3, 5, 6)}
        N1 = int((est[3] + 2 * est[5] + 4 * est[6]) * rng.uniform(1.05, 3.0)) + 1
        est1 = N1 - est[3] - 2 * est[5] - 4 * est[6]
        eps = 0.01
        kp, kc, capped, unseen = ps.samples_for_request(tp, tc, K0, W, 0, N1, 1 << 1, eps, 0.01, 2 ** 62)
        assert capped == 0 and kc == K0
        up = dn = 0.0
        for j, c in ((3, 1), (5, 2), (6, 4)):
            if tp[j] == 0:
                continue
            a = tp[j] / K0
            pl, pu = ofin.chernoff_interval_alpha(a, kp, 0.01)
            K = W / ofin.A2[j]
            up += c * K * (pu - a)
            dn += c * K * (a - pl)
        assert up <= eps * est1 * (1 + 1e-9) and dn <= eps * est1 * (1 + 1e-9)


def test_argument_errors():
    with pytest.raises(ps.PathSampError):
        ps.samples_for_request([0] * 8, [0] * 8, 0, 1, 1, 1, 0, 0.01, 0.01, 10)
    with pytest.raises(ps.PathSampError):
        ps.samples_for_request([0] * 8, [0] * 8, K0, 1, 1, 1, 0, 0.0, 0.01, 10 ** 9)
    with pytest.raises(ps.PathSampError):
        ps.samples_for_request([0] * 8, [0] * 8, K0, 1, 1, 1, 0, 0.01, 0.01, K0 - 1)


def test_chernoff_alpha_agrees_with_count_form():
    for c, k in [(1, 7), (500, 1000), (3, 200000)]:
        assert ofin.chernoff_interval(c, k, 0.01) == ofin.chernoff_interval_alpha(c / k, k, 0.01)
    assert math.isclose(ofin.samples_for_error(0.01, 0.01, 0.5), ps.samples_for_error(0.01, 0.01, 0.5), abs_tol=1)
