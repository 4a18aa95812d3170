"""CPU-side checks of the C ABI: the library loads, exports every function
include/pathsamp.h declares, and its host-side finalize agrees with the
oracle's estimates and bars.  No device call is made here."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from oracle import finalize as ofin
from paper_1411_4942_amd import pathsamp as ps

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = []
    for fname in os.listdir(os.path.join(ROOT, "include")):
        if not fname.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fname)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(pm_[a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for must in ("pm_count_motifs", "pm_graph_create", "pm_graph_destroy", "pm_count", "pm_finalize",
                 "pm_samples_for_error", "pm_last_error", "pm_status_string"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(ps.LIB_PATH if os.path.exists(ps.LIB_PATH) else ps.lib()._name)
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding knows every one of them
    assert not [n for n in _declared_functions() if n not in ps._SIGNATURES]


def _random_case(rng):
    k_path = int(rng.integers(1, 10 ** int(rng.integers(1, 8))))
    k_cent = int(rng.integers(1, 10 ** int(rng.integers(1, 8))))
    tp = rng.multinomial(k_path, rng.dirichlet(np.ones(7))).tolist()
    tp = [tp[0], 0] + tp[1:6]
    tp = tp + [0] * (8 - len(tp))
    tp[0] += k_path - sum(tp)
    tc = rng.multinomial(k_cent, rng.dirichlet(np.ones(5))).tolist()
    tc = [tc[0], tc[1], 0, 0, tc[2], tc[3], tc[4], 0]
    W = int(rng.integers(1, 2 ** 62))
    Lam = int(rng.integers(1, W + 1))
    N1 = int(rng.integers(0, 2 ** 63))
    return tp, tc, W, Lam, N1, k_path, k_cent


def test_finalize_matches_oracle():
    rng = np.random.default_rng(7)
    for _ in range(300):
        tp, tc, W, Lam, N1, kp, kc = _random_case(rng)
        delta = float(rng.choice([0.01, 0.05, 0.001]))
        got = ps.finalize(tp, tc, W, Lam, N1, kp, kc, delta)
        want = ofin.finalize(tp, tc, 2 * W, 2 * Lam, N1, kp, kc, delta)
        for key in ("est", "est_basic"):
            for i in range(1, 7):
                assert got[key][i] == pytest.approx(want[key][i], rel=1e-12, abs=1e-6), (key, i)
        for key in ("lo", "hi"):
            for i in range(1, 7):
                scale = max(abs(want[key][i]), 1.0)
                if i == 1:  # difference of large numbers: compare against the parts
                    scale = max(scale, float(W))
                assert abs(got[key][i] - want[key][i]) <= 1e-9 * scale, (key, i, got[key][i], want[key][i])


def test_finalize_zero_weight_samplers():
    got = ps.finalize([0] * 8, [0] * 8, 0, 0, 123, 10, 10)
    assert got["est"] == [0.0, 123.0, 0.0, 0.0, 0.0, 0.0, 0.0]
    assert got["lo"][1] == got["hi"][1] == 123.0


def test_finalize_rejects_bad_arguments():
    with pytest.raises(ps.PathSampError) as e:
        ps.finalize([0] * 8, [0] * 8, 1, 1, 1, 10, 10, delta=1.5)
    assert e.value.status == ps.PM_EINVAL
    with pytest.raises(ps.PathSampError):
        ps.finalize([0, 0, 11, 0, 0, 0, 0, 0], [0] * 8, 5, 5, 1, 10, 10)  # tally > k


def test_chernoff_matches_oracle():
    for count, k in [(0, 10), (10, 10), (1, 1000), (500, 1000), (3, 200000), (199990, 200000)]:
        for delta in (0.01, 0.1):
            got = ps.chernoff_interval(count, k, delta)
            want = ofin.chernoff_interval(count, k, delta)
            assert got[0] == pytest.approx(want[0], rel=1e-9, abs=1e-15)
            assert got[1] == pytest.approx(want[1], rel=1e-9, abs=1e-15)


def test_samples_for_error():
    """k from Corollary 5.3: at that k the bar of a proportion alpha stays within
    the relative error, and one less sample does not guarantee it."""
    for alpha in (0.969, 0.0199, 0.0129, 2.7e-4):
        k = ps.samples_for_error(0.01, 0.01, alpha)
        target = math.log(100.0)
        d_up = ofin.kl_bernoulli(alpha, alpha * 1.01)
        d_dn = ofin.kl_bernoulli(alpha, alpha * 0.99)
        assert k * min(d_up, d_dn) >= target
        assert (k - 1) * min(d_up, d_dn) < target
        # small-alpha approximation 2 ln(1/delta) / (alpha eps^2)
        if alpha < 0.05:
            approx = 2 * target / (alpha * 1e-4)
            assert 0.8 * approx < k < 1.2 * approx
    with pytest.raises(ps.PathSampError):
        ps.samples_for_error(0.0, 0.01, 0.5)


def test_status_strings():
    """Every status code has its name; unknown codes say so (no device call)."""
    L = ps.lib()
    names = {ps.PM_OK: b"PM_OK", ps.PM_EINVAL: b"PM_EINVAL", ps.PM_EGRAPH: b"PM_EGRAPH",
             ps.PM_EOVERFLOW: b"PM_EOVERFLOW", ps.PM_ENOMEM: b"PM_ENOMEM", ps.PM_EDEVICE: b"PM_EDEVICE",
             ps.PM_EBUSY: b"PM_EBUSY", ps.PM_ECANCELED: b"PM_ECANCELED"}
    for code, name in names.items():
        assert L.pm_status_string(code) == name
    assert L.pm_status_string(-99) == b"PM_UNKNOWN"
