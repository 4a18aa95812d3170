"""Estimates and error bars from sample tallies -- the oracle's host half.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Estimates (exact rational arithmetic, one rounding at the end):
  Algorithm 2:  C^_i = (count_i / k) * W / A_{2,i},  i = 2..6,
                C^_1 = N_1 - C^_3 - 2 C^_5 - 4 C^_6   (Alg. 2's own C^_5, C^_6)
  Algorithm 4:  C^_i = (count_i / k) * Lambda / B_i,  i = 4..6
  Final (end of Section 4): C_1..C_3 from Algorithm 2, C_4..C_6 from Algorithm 4.
A_{2,i} is row 2 of Eq. 1 (3-paths inside motif i); B_i is Lemma 4.2
(centered 3-paths inside motif i).

Error bars (Section 5): with alpha = count_i / k, p_l < alpha < p_u are the two
roots of k D(alpha, p) = ln(1/delta), D the Bernoulli KL divergence of
Theorem 5.1 (Definition 5.2, Corollary 5.3); the bar of C^_i is
[K_i p_l, K_i p_u] with K_i the scaling above.  For the 3-star the errors of
C^_3, 2 C^_5, 4 C^_6 (from Algorithm 2) are added up.
"""
from __future__ import annotations

import math
from fractions import Fraction

# Eq. 1, row 2: number of 3-paths in motif i (i = 1..6)
A2 = {1: 0, 2: 1, 3: 2, 4: 4, 5: 6, 6: 12}
# Lemma 4.2: number of centered 3-paths in motif i
B = {4: 1, 5: 1, 6: 3}


def kl_bernoulli(a: float, b: float) -> float:
    """D(a, b) of Theorem 5.1, with 0 ln 0 = 0 (infinite where b puts no
    mass on an outcome a has)."""
    if (b <= 0.0 and a > 0.0) or (b >= 1.0 and a < 1.0):
        return math.inf
    t1 = 0.0 if a == 0.0 else a * math.log(a / b)
    t2 = 0.0 if a == 1.0 else (1.0 - a) * math.log((1.0 - a) / (1.0 - b))
    return t1 + t2


def chernoff_interval(count: int, k: int, delta: float):
    """(p_l, p_u) of Definition 5.2 for alpha = count / k at x = delta.

    Bisection on each monotone side of p -> D(alpha, p) (unimodality of
    exp(-k D), Section 5).  At alpha = 0 the lower root is 0 and the upper
    root solves k ln(1/(1-p)) = ln(1/delta); symmetrically at alpha = 1.
    """
    if k <= 0:
        raise ValueError("k must be positive")
    if not (0.0 < delta < 1.0):
        raise ValueError("delta must lie in (0, 1)")
    if count == 0:
        return 0.0, 1.0 - delta ** (1.0 / k)
    if count == k:
        return delta ** (1.0 / k), 1.0
    return chernoff_interval_alpha(count / k, k, delta)


def chernoff_interval_alpha(alpha: float, k: int, delta: float):
    """The two roots of k D(alpha, p) = ln(1/delta) for a proportion
    0 < alpha < 1 given as a real number (Definition 5.2)."""
    target = math.log(1.0 / delta) / k

    def solve(lo, hi, increasing):
        # root of D(alpha, p) = target on [lo, hi]; D is monotone there
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            f = kl_bernoulli(alpha, mid) - target
            if (f > 0) == increasing:
                hi = mid
            else:
                lo = mid
            if hi - lo <= 1e-16:
                break
        return 0.5 * (lo + hi)

    # below alpha, D decreases in p; above alpha, D increases in p
    if kl_bernoulli(alpha, 5e-324) <= target:  # pragma: no cover - k tiny
        p_l = 0.0
    else:
        p_l = solve(0.0, alpha, increasing=False)
    if kl_bernoulli(alpha, math.nextafter(1.0, 0.0)) <= target:  # pragma: no cover
        p_u = 1.0
    else:
        p_u = solve(alpha, 1.0, increasing=True)
    return p_l, p_u


def _f(x: Fraction) -> float:
    return float(x)


def finalize(tally_path, tally_cent, R_tau: int, R_lam: int, N1: int, k_path: int, k_cent: int,
             delta: float = 0.01) -> dict:
    """Estimates and bars; index 1..6 is the motif number, index 0 unused."""
    tp = [int(x) for x in tally_path]
    tc = [int(x) for x in tally_cent]
    W = Fraction(int(R_tau), 2)
    Lam = Fraction(int(R_lam), 2)
    est = [0.0] * 7
    lo = [0.0] * 7
    hi = [0.0] * 7
    est_basic = [0.0] * 7
    exact_basic = {}

    # Algorithm 2 (3-path-sampler), estimates for motifs 2..6
    for i in range(2, 7):
        if R_tau == 0 or k_path == 0:
            e = Fraction(0)
        else:
            e = Fraction(tp[i], k_path) * W / A2[i]
        exact_basic[i] = e
        est_basic[i] = _f(e)
    c1 = Fraction(int(N1)) - exact_basic[3] - 2 * exact_basic[5] - 4 * exact_basic[6]
    est_basic[1] = _f(c1)

    # bars of Algorithm 2's counts
    lo_b, hi_b = {}, {}
    for i in range(2, 7):
        if R_tau == 0 or k_path == 0:
            lo_b[i], hi_b[i] = 0.0, 0.0
        else:
            pl, pu = chernoff_interval(tp[i], k_path, delta)
            K = float(W) / A2[i]
            lo_b[i], hi_b[i] = K * pl, K * pu

    for i in (1, 2, 3):
        est[i] = est_basic[i]
    for i in (2, 3):
        lo[i], hi[i] = lo_b[i], hi_b[i]
    lo[1] = float(N1) - (hi_b[3] + 2 * hi_b[5] + 4 * hi_b[6])
    hi[1] = float(N1) - (lo_b[3] + 2 * lo_b[5] + 4 * lo_b[6])

    # Algorithm 4 (centered-sampler), estimates for motifs 4..6
    for i in (4, 5, 6):
        if R_lam == 0 or k_cent == 0:
            est[i], lo[i], hi[i] = 0.0, 0.0, 0.0
            continue
        est[i] = _f(Fraction(tc[i], k_cent) * Lam / B[i])
        pl, pu = chernoff_interval(tc[i], k_cent, delta)
        K = float(Lam) / B[i]
        lo[i], hi[i] = K * pl, K * pu

    return {
        "tally_path": tp,
        "tally_cent": tc,
        "W": int(R_tau) // 2,
        "Lambda": int(R_lam) // 2,
        "N1": int(N1),
        "k_path": int(k_path),
        "k_cent": int(k_cent),
        "est": est,
        "lo": lo,
        "hi": hi,
        "est_basic": est_basic,
    }


def samples_for_error(rel_err: float, delta: float, alpha: float) -> int:
    """Smallest k with k min(D(alpha, alpha(1-e)), D(alpha, alpha(1+e))) >=
    ln(1/delta): the bar of Corollary 5.3 around alpha stays within relative
    error e on both sides (the side above 1 does not bind)."""
    d = kl_bernoulli(alpha, alpha * (1.0 - rel_err))
    if alpha * (1.0 + rel_err) < 1.0:
        d = min(d, kl_bernoulli(alpha, alpha * (1.0 + rel_err)))
    return math.ceil(math.log(1.0 / delta) / d)


def samples_for_request(tally_path, tally_cent, k0: int, W: int, Lambda: int, N1: int, mask: int,
                        rel_err: float, delta: float, k_max: int):
    """Budgets (k_path, k_cent, capped, unseen) of the served mode from pilot
    tallies over k0 ids per sampler.

    Motifs 2, 3 are sized on the 3-path sampler's proportions and 4, 5, 6 on
    the centered sampler's, each at relative error rel_err; a motif without a
    pilot hit takes the upper root p_u of its interval as its proportion.
    Motif 1 is N_1 - C_3 - 2 C_5 - 4 C_6 (Algorithm 2): its allowed error
    rel_err * C^_1 is shared equally by the h terms with a hit, term j sized at
    relative error rel_err C^_1 / (h c_j C^_j) when that is below 1.  Each
    sampler's k is its largest requirement, at least k0, at most k_max."""
    if mask == 0:
        mask = 0x7E
    capped = unseen = 0
    need = [0] * 7
    p_unseen = 1.0 - delta ** (1.0 / k0)

    def size(i, t, eps):
        nonlocal unseen
        if t == 0:
            unseen |= 1 << i
            alpha = p_unseen
        else:
            alpha = t / k0
        if alpha >= 1.0:
            return math.ceil(math.log(1.0 / delta) / kl_bernoulli(1.0, 1.0 - eps))
        return samples_for_error(eps, delta, alpha)

    tp = [int(x) for x in tally_path]
    tc = [int(x) for x in tally_cent]
    if W:
        for i in (2, 3):
            if mask >> i & 1:
                need[i] = size(i, tp[i], rel_err)
        if mask >> 1 & 1:
            terms = ((3, 1.0), (5, 2.0), (6, 4.0))
            est = {j: tp[j] * W / (k0 * A2[j]) for j, _ in terms}
            hits = sum(1 for j, _ in terms if tp[j])
            est1 = N1 - est[3] - 2.0 * est[5] - 4.0 * est[6]
            if not est1 > 0.0:
                capped |= 2
            else:
                for j, c in terms:
                    if tp[j] == 0:
                        continue
                    eps = rel_err * est1 / (hits * c * est[j])
                    if eps < 1.0:
                        need[1] = max(need[1], size(1, tp[j], eps))
    if Lambda:
        for i in (4, 5, 6):
            if mask >> i & 1:
                need[i] = size(i, tc[i], rel_err)
    k = [k0, k0]
    for i in range(1, 7):
        if need[i] > k_max:
            capped |= 1 << i
            need[i] = k_max
        side = 0 if i <= 3 else 1
        k[side] = max(k[side], need[i])
    return k[0], k[1], capped, unseen
