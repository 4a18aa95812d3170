"""Pins of the oracle's alias-table edge draw (oracle/alias.c), the variant of
the weighted edge pick of Algorithm 1 step 2 and Algorithm 3 step 2.

* exactness: every slot's mass over all buckets is exactly N * w[s], so the
  draw picks s with probability w[s] / R (checked with Python integers, and
  by enumerating every (bucket, coin) pair on tiny tables);
* the table equals the closed form of the sweep (light slot i takes the first
  heavy slot whose cumulative excess reaches the light deficits before i; a
  heavy slot drawn down keeps R + E_h - (first cumulative deficit beyond
  E_h)), written independently here from prefix sums;
* the draw's stream is the stated one (Philox candidates in order, Lemire
  acceptance, b then x then o), composed from the pinned primitives;
* the alias samplers' outcome frequencies match the exact distribution from
  enumerating every r (chi-square at a fixed seed), and their estimates are
  unbiased against exact counts.
"""
import numpy as np
import pytest

import oracle
from oracle import finalize as ofin
from paper_1411_4942_amd import synth


def _weights_cases():
    rng = np.random.default_rng(7)
    cases = [
        np.array([1, 2, 3, 4, 0, 10], np.uint64),
        np.array([5], np.uint64),
        np.array([0, 0, 7, 0], np.uint64),
        np.full(17, 3, np.uint64),                       # all equal: every bucket full
        np.array([1] * 50 + [1000], np.uint64),          # one dominant slot
        np.array([2 ** 60, 3, 2 ** 59, 1, 0], np.uint64),  # N * w beyond 2^64
    ]
    for n in (2, 3, 8, 31, 64, 257):
        cases.append(rng.integers(0, 20, size=n).astype(np.uint64))
        cases.append((rng.pareto(1.2, size=n) * 10).astype(np.uint64))
        cases.append(rng.integers(0, 2 ** 40, size=n).astype(np.uint64))
    return [c for c in cases if int(c.astype(object).sum()) > 0]


def _masses(K, A, R):
    N = len(K)
    got = [0] * N
    for b in range(N):
        got[b] += int(K[b])
        if int(K[b]) < R:
            got[int(A[b])] += R - int(K[b])
    return got


@pytest.mark.parametrize("w", _weights_cases(), ids=lambda w: f"N{len(w)}")
def test_alias_table_is_exact(w):
    K, A = oracle.alias_build(w)
    N = len(w)
    R = int(w.astype(object).sum())
    assert all(0 <= int(k) <= R for k in K)
    assert all(0 <= int(a) < N for a in A)
    assert _masses(K, A, R) == [N * int(x) for x in w]
    for b in range(N):  # an alias only ever names a heavy slot
        if int(K[b]) < R:
            assert N * int(w[int(A[b])]) >= R


@pytest.mark.parametrize("w", [np.array(x, np.uint64) for x in
                               ([1, 2, 3], [0, 4, 1, 1], [3, 3, 3, 1, 0, 2], [7, 0, 0, 0, 1], [1, 1])])
def test_alias_enumeration(w):
    """Every (bucket, coin) pair once: slot s comes up exactly N * w[s] times."""
    K, A = oracle.alias_build(w)
    N, R = len(w), int(w.sum())
    hits = [0] * N
    for b in range(N):
        for x in range(R):
            hits[b if x < int(K[b]) else int(A[b])] += 1
    assert hits == [N * int(v) for v in w]


def _closed_form(w):
    N = len(w)
    R = sum(int(x) for x in w)
    M = [N * int(x) for x in w]
    light = [s for s in range(N) if M[s] < R]
    heavy = [s for s in range(N) if M[s] >= R]
    D = [0]
    for s in light:
        D.append(D[-1] + R - M[s])     # D[i] = deficits of the first i light slots
    E = []
    acc = 0
    for s in heavy:
        acc += M[s] - R
        E.append(acc)                  # E[h] = excess of heavy slots 0..h
    K = [0] * N
    A = [0] * N
    for i, s in enumerate(light):
        h = next(h for h in range(len(heavy)) if D[i] <= E[h])
        K[s], A[s] = M[s], heavy[h]
    for h, s in enumerate(heavy):
        beyond = [d for d in D[1:] if d > E[h]]
        if beyond:
            K[s], A[s] = R + E[h] - beyond[0], heavy[h + 1]
        else:
            K[s], A[s] = R, s
    return K, A


@pytest.mark.parametrize("w", _weights_cases(), ids=lambda w: f"N{len(w)}")
def test_alias_table_closed_form(w):
    K, A = oracle.alias_build(w)
    K2, A2 = _closed_form(w)
    assert [int(x) for x in K] == K2
    assert [int(x) for x in A] == A2


def test_alias_build_rejects_bad_input():
    with pytest.raises(oracle.OracleError):
        oracle.alias_build(np.zeros(4, np.uint64))
    with pytest.raises(oracle.OracleError):
        oracle.alias_build(np.array([2 ** 63, 2 ** 63], np.uint64))


def _stream(seed, tag, sid):
    """Candidate words of one sample, in order."""
    attempt = 0
    while True:
        w = oracle.philox4x32_10([sid & 0xFFFFFFFF, sid >> 32, tag, attempt], [seed & 0xFFFFFFFF, seed >> 32])
        yield int(w[0]) | (int(w[1]) << 32)
        yield int(w[2]) | (int(w[3]) << 32)
        attempt += 1


def _bounded(gen, R):
    for x in gen:
        ok, r = oracle.lemire(x, R, 64)
        if ok:
            return r


@pytest.mark.parametrize("centered", [False, True])
def test_alias_draw_follows_its_stream(centered):
    off, col = synth.chung_lu(300, 1500, 2.3, 60.0, 4)
    g = oracle.Graph(off, col)
    K, A = g.alias_table(centered)
    P = g.p_lam if centered else g.p_tau
    R = g.R_lam if centered else g.R_tau
    for seed, sid in [(1, 0), (1, 1), (0xDEADBEEFCAFEF00D, 2 ** 33 + 5), (7, 123456)]:
        gen = _stream(seed, 3 if centered else 2, sid)
        b = _bounded(gen, g.slots)
        x = _bounded(gen, R)
        s = b if x < int(K[b]) else int(A[b])
        below = int(P[s - 1]) if s else 0
        o = _bounded(gen, int(P[s]) - below)
        assert g.draw_alias(centered, seed, sid) == below + o


@pytest.mark.parametrize("name,graph", [("K6", synth.complete(6)), ("gnm", synth.erdos_renyi(40, 150, 3)),
                                        ("chunglu", synth.chung_lu(120, 500, 2.2, 30.0, 2))])
def test_alias_sampler_frequencies_match_enumeration(name, graph):
    """Outcome counts of 60,000 alias draws against the exact outcome
    distribution (every r once): chi-square below the 0.999 quantile."""
    from scipy.stats import chi2

    g = oracle.Graph(*graph)
    k = 60000
    for got, exact, R in [(g.sample_path_alias(11, k), g.enumerate_path(), g.R_tau),
                          (g.sample_centered_alias(11, k), g.enumerate_centered(), g.R_lam)]:
        cls = [c for c in range(8) if exact[c] > 0]
        exp = np.array([k * int(exact[c]) / R for c in cls])
        obs = np.array([int(got[c]) for c in cls])
        assert int(got.sum()) == k
        assert all(int(got[c]) == 0 for c in range(8) if exact[c] == 0), name
        if len(cls) > 1:
            stat = float(((obs - exp) ** 2 / exp).sum())
            assert stat < chi2.ppf(0.999, len(cls) - 1), (name, stat)


def test_alias_estimates_unbiased():
    off, col = synth.chung_lu(2000, 12000, 2.3, 150.0, 5)
    C, _ = oracle.exact_formula(off, col)
    g = oracle.Graph(off, col)
    k = 40000
    runs = []
    for seed in range(12):
        tp = g.sample_path_alias(seed, k)
        tc = g.sample_centered_alias(seed, k)
        runs.append(ofin.finalize(tp, tc, g.R_tau, g.R_lam, g.N1, k, k)["est"])
    for i in range(1, 7):
        if C[i] == 0:
            continue
        est = np.array([r[i] for r in runs])
        se = est.std(ddof=1) / np.sqrt(len(est))
        assert abs(est.mean() - C[i]) <= 5 * se + 1e-9 * C[i], (i, est.mean(), C[i], se)
