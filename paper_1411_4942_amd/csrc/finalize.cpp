// Host-side estimates (Algorithms 2 and 4) and error bars (Section 5).
//
// Estimates are exact rationals rounded once: every numerator is formed in
// 128-bit integers and divided in long double.
//   Algorithm 2:  C_i = count_i W / (k A_{2,i}),  A_{2,.} = (-, 1, 2, 4, 6, 12)
//                 C_1 = N_1 - C_3 - 2 C_5 - 4 C_6  (Algorithm 2's own values)
//   Algorithm 4:  C_i = count_i Lambda / (k B_i),  B_4 = B_5 = 1, B_6 = 3
//   final (end of Section 4): motifs 1..3 from Algorithm 2, 4..6 from Algorithm 4
// Bars: count_i / k = alpha; p_l < alpha < p_u solve k D(alpha, p) = ln(1/delta)
// (Theorem 5.1, Definition 5.2, Corollary 5.3); bar = [K p_l, K p_u] with K the
// estimate's scaling; the 3-star bar adds up the bars of C_3, 2 C_5, 4 C_6.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <algorithm>
#include <string>

#include "../../include/pathsamp.h"

namespace pm {

void set_error(const std::string &msg);

namespace {

const int kA2[7] = {0, 0, 1, 2, 4, 6, 12};  // 3-paths in motif i (Eq. 1, row 2)
const int kB[7] = {0, 0, 0, 0, 1, 1, 3};    // centered 3-paths in motif i (Lemma 4.2)

typedef unsigned __int128 u128;
typedef __int128 i128;

// D(a, b), the Bernoulli KL divergence of Theorem 5.1 (0 ln 0 = 0)
double kl(double a, double b)
{
    if ((b <= 0.0 && a > 0.0) || (b >= 1.0 && a < 1.0)) return INFINITY;
    double t1 = a == 0.0 ? 0.0 : a * std::log(a / b);
    double t2 = a == 1.0 ? 0.0 : (1.0 - a) * std::log((1.0 - a) / (1.0 - b));
    return t1 + t2;
}

// root of D(alpha, p) = target for p in [lo, hi], D monotone there
double bisect(double alpha, double target, double lo, double hi, bool increasing)
{
    for (int it = 0; it < 200 && hi - lo > 1e-16; ++it) {
        double mid = 0.5 * (lo + hi);
        double f = kl(alpha, mid) - target;
        if ((f > 0) == increasing)
            hi = mid;
        else
            lo = mid;
    }
    return 0.5 * (lo + hi);
}

}  // namespace

pm_status chernoff_interval(uint64_t count, uint64_t k, double delta, double *p_lo, double *p_hi)
{
    if (!p_lo || !p_hi || k == 0 || count > k || !(delta > 0.0 && delta < 1.0)) {
        set_error("chernoff_interval: need k > 0, count <= k, delta in (0,1)");
        return PM_EINVAL;
    }
    const double target = std::log(1.0 / delta) / (double)k;
    if (count == 0) {
        *p_lo = 0.0;
        *p_hi = 1.0 - std::pow(delta, 1.0 / (double)k);
        return PM_OK;
    }
    if (count == k) {
        *p_lo = std::pow(delta, 1.0 / (double)k);
        *p_hi = 1.0;
        return PM_OK;
    }
    const double alpha = (double)count / (double)k;
    *p_lo = kl(alpha, 5e-324) <= target ? 0.0 : bisect(alpha, target, 0.0, alpha, false);
    *p_hi = kl(alpha, std::nextafter(1.0, 0.0)) <= target ? 1.0 : bisect(alpha, target, alpha, 1.0, true);
    return PM_OK;
}

static double ratio(u128 num, u128 den) { return (double)((long double)num / (long double)den); }

pm_status finalize(const uint64_t tp[PM_NUM_TALLIES], const uint64_t tc[PM_NUM_TALLIES], uint64_t W,
                   uint64_t Lambda, uint64_t N1, uint64_t k_path, uint64_t k_cent, double delta, pm_result *out)
{
    if (!tp || !tc || !out || !(delta > 0.0 && delta < 1.0)) {
        set_error("finalize: null argument or delta outside (0,1)");
        return PM_EINVAL;
    }
    pm_result r;
    std::memset(&r, 0, sizeof(r));
    std::memcpy(r.tally_path, tp, sizeof(r.tally_path));
    std::memcpy(r.tally_cent, tc, sizeof(r.tally_cent));
    r.W = W;
    r.Lambda = Lambda;
    r.N1 = N1;
    r.k_path = k_path;
    r.k_cent = k_cent;

    const bool use_path = W != 0 && k_path != 0;
    const bool use_cent = Lambda != 0 && k_cent != 0;
    double lo_b[7] = {0}, hi_b[7] = {0};
    if (use_path) {
        for (int i = 2; i <= 6; ++i) {
            if (tp[i] > k_path) {
                set_error("finalize: a tally exceeds k");
                return PM_EINVAL;
            }
            r.est_basic[i] = ratio((u128)tp[i] * W, (u128)k_path * (u128)kA2[i]);
            double pl, pu;
            chernoff_interval(tp[i], k_path, delta, &pl, &pu);
            const double K = (double)W / kA2[i];
            lo_b[i] = K * pl;
            hi_b[i] = K * pu;
        }
        // C_1 = N_1 - W (3 t_3 + 2 t_5 + 2 t_6) / (6 k), one exact numerator
        const i128 num = (i128)6 * (i128)k_path * (i128)N1 -
                         (i128)W * (i128)(3 * (u128)tp[3] + 2 * (u128)tp[5] + 2 * (u128)tp[6]);
        r.est_basic[1] = (double)((long double)num / (long double)(6 * (u128)k_path));
    } else {
        r.est_basic[1] = (double)N1;
    }
    for (int i = 1; i <= 3; ++i) r.est[i] = r.est_basic[i];
    for (int i = 2; i <= 3; ++i) {
        r.lo[i] = lo_b[i];
        r.hi[i] = hi_b[i];
    }
    r.lo[1] = (double)N1 - (hi_b[3] + 2 * hi_b[5] + 4 * hi_b[6]);
    r.hi[1] = (double)N1 - (lo_b[3] + 2 * lo_b[5] + 4 * lo_b[6]);
    if (use_cent) {
        for (int i = 4; i <= 6; ++i) {
            if (tc[i] > k_cent) {
                set_error("finalize: a tally exceeds k");
                return PM_EINVAL;
            }
            r.est[i] = ratio((u128)tc[i] * Lambda, (u128)k_cent * (u128)kB[i]);
            double pl, pu;
            chernoff_interval(tc[i], k_cent, delta, &pl, &pu);
            const double K = (double)Lambda / kB[i];
            r.lo[i] = K * pl;
            r.hi[i] = K * pu;
        }
    }
    *out = r;
    return PM_OK;
}

pm_status samples_for_error(double rel_err, double delta, double alpha, uint64_t *k_out)
{
    if (!k_out || !(rel_err > 0.0 && rel_err < 1.0) || !(delta > 0.0 && delta < 1.0) ||
        !(alpha > 0.0 && alpha < 1.0)) {
        set_error("samples_for_error: need rel_err, delta, alpha in (0,1)");
        return PM_EINVAL;
    }
    const double up = alpha * (1.0 + rel_err);
    double d = kl(alpha, alpha * (1.0 - rel_err));
    if (up < 1.0) d = std::fmin(d, kl(alpha, up));
    const double k = std::ceil(std::log(1.0 / delta) / d);
    *k_out = (k >= 1.8e19) ? UINT64_MAX : (uint64_t)k;
    return PM_OK;
}

namespace {

// k of pm_samples_for_error, extended to alpha = 1 (only the lower side
// binds: D(1, 1 - e) = ln(1 / (1 - e))) and saturating instead of failing
uint64_t k_for(double rel_err, double delta, double alpha)
{
    if (alpha >= 1.0) {
        const double k = std::ceil(std::log(1.0 / delta) / -std::log1p(-rel_err));
        return k >= 1.8e19 ? UINT64_MAX : (uint64_t)k;
    }
    uint64_t k = UINT64_MAX;
    (void)samples_for_error(rel_err, delta, alpha, &k);
    return k;
}

}  // namespace

pm_status samples_for_request(const uint64_t tp[PM_NUM_TALLIES], const uint64_t tc[PM_NUM_TALLIES], uint64_t k0,
                              uint64_t W, uint64_t Lambda, uint64_t N1, uint32_t mask, double rel_err, double delta,
                              uint64_t k_max, uint64_t *k_path, uint64_t *k_cent, uint32_t *capped, uint32_t *unseen)
{
    if (!tp || !tc || !k_path || !k_cent || !capped || !unseen || k0 == 0 || k_max < k0 ||
        !(rel_err > 0.0 && rel_err < 1.0) || !(delta > 0.0 && delta < 1.0)) {
        set_error("samples_for_request: need k0 > 0, k_max >= k0, rel_err and delta in (0,1)");
        return PM_EINVAL;
    }
    if (mask == 0) mask = 0x7e;
    *capped = 0;
    *unseen = 0;
    uint64_t need[7] = {0};
    // p_u of Definition 5.2 for a proportion observed as 0 in k0 samples
    const double p_unseen = 1.0 - std::pow(delta, 1.0 / (double)k0);
    auto size_one = [&](int i, uint64_t t, double eps) -> uint64_t {
        double alpha = (double)t / (double)k0;
        if (t == 0) {
            alpha = p_unseen;
            *unseen |= 1u << i;
        }
        return k_for(eps, delta, alpha);
    };
    if (W != 0) {
        for (int i = 2; i <= 3; ++i)
            if (mask & (1u << i)) need[i] = size_one(i, tp[i], rel_err);
        if (mask & 2u) {
            // C_1 = N_1 - C_3 - 2 C_5 - 4 C_6 (Algorithm 2's estimates): split
            // the error budget over the terms that had a hit
            const int terms[3] = {3, 5, 6};
            const double coef[3] = {1.0, 2.0, 4.0};
            double est[3];
            int hits = 0;
            for (int j = 0; j < 3; ++j) {
                est[j] = (double)tp[terms[j]] * (double)W / ((double)k0 * kA2[terms[j]]);
                if (tp[terms[j]] != 0) ++hits;
            }
            const double est1 = (double)N1 - est[0] - 2.0 * est[1] - 4.0 * est[2];
            if (!(est1 > 0.0)) {
                *capped |= 2u;  // no relative error can be promised
            } else {
                for (int j = 0; j < 3; ++j) {
                    if (tp[terms[j]] == 0) continue;
                    const double eps = rel_err * est1 / (hits * coef[j] * est[j]);
                    if (eps < 1.0) need[1] = std::max(need[1], size_one(1, tp[terms[j]], eps));
                }
            }
        }
    }
    if (Lambda != 0)
        for (int i = 4; i <= 6; ++i)
            if (mask & (1u << i)) need[i] = size_one(i, tc[i], rel_err);
    uint64_t kp = k0, kc = k0;
    for (int i = 1; i <= 6; ++i) {
        uint64_t &k = i <= 3 ? kp : kc;
        if (need[i] > k_max) {
            *capped |= 1u << i;
            need[i] = k_max;
        }
        k = std::max(k, need[i]);
    }
    *k_path = kp;
    *k_cent = kc;
    return PM_OK;
}

}  // namespace pm
