"""Plain CPU oracle for 3-path sampling (Jha, Seshadhri, Pinar, arXiv 1411.4942).

TEST INFRASTRUCTURE ONLY.  This package is the checker the HIP library is
compared against, never a fallback for it: only the test suite, the smoke
check and the CPU-baseline leg of the benchmark import it.  It shares no code
with the HIP library.

The sampling steps (Sections 2-4) are single-threaded C in ``oracle.c``;
the exact counters are in ``exact.c``; estimates and error bars (Algorithms
2 and 4, Section 5) are in :mod:`oracle.finalize`.  This module loads the C
half through ctypes and converts numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SOURCES = [os.path.join(_HERE, "oracle.c"), os.path.join(_HERE, "exact.c"), os.path.join(_HERE, "alias.c")]

OK, EINVAL, EGRAPH, EOVERFLOW, ENOMEM = 0, -1, -2, -3, -4
STATUS_NAMES = {OK: "OK", EINVAL: "EINVAL", EGRAPH: "EGRAPH", EOVERFLOW: "EOVERFLOW", ENOMEM: "ENOMEM"}

# tally indices: 0 triangle outcome, 1 centered "not centered" reject,
# 2..6 the motifs of Figure 1 (3-path .. 4-clique)
TRI, OPEN = 0, 1


class OracleError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {STATUS_NAMES.get(status, status)}")
        self.status = status


def build(force: bool = True) -> str:
    """Compile the C half of the oracle with gcc (single-threaded, -O2)."""
    if not force and os.path.exists(_SO):
        return _SO
    tmp = _SO + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared", "-o", tmp] + _SOURCES
    subprocess.run(cmd, check=True)
    os.replace(tmp, _SO)
    return _SO


class _Graph(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("slots", ctypes.c_int64),
        ("off", ctypes.POINTER(ctypes.c_int64)),
        ("col", ctypes.POINTER(ctypes.c_int32)),
        ("rank", ctypes.POINTER(ctypes.c_int32)),
        ("p_tau", ctypes.POINTER(ctypes.c_uint64)),
        ("p_lam", ctypes.POINTER(ctypes.c_uint64)),
        ("R_tau", ctypes.c_uint64),
        ("R_lam", ctypes.c_uint64),
        ("N1", ctypes.c_uint64),
    ]


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        build()
    lib = ctypes.CDLL(_SO)
    P = ctypes.c_void_p
    u64, i64, u32, i32 = ctypes.c_uint64, ctypes.c_int64, ctypes.c_uint32, ctypes.c_int32
    gp = ctypes.POINTER(_Graph)
    sig = {
        "or_validate": (i32, [i64, P, P]),
        "or_graph_build": (i32, [i64, P, P, gp]),
        "or_graph_free": (None, [gp]),
        "or_philox4x32_10": (None, [P, P, P]),
        "or_lemire": (i32, [u64, u64, ctypes.c_int, ctypes.POINTER(u64)]),
        "or_draw": (u64, [u64, u32, u64, u64]),
        "or_draws": (None, [u64, u32, u64, u64, u64, P]),
        "or_decode_path": (None, [gp, u64, P]),
        "or_decode_centered": (None, [gp, u64, P]),
        "or_classify_path": (ctypes.c_int, [gp, P]),
        "or_classify_centered": (ctypes.c_int, [gp, P]),
        "or_sample_path": (None, [gp, u64, u64, u64, P]),
        "or_sample_centered": (None, [gp, u64, u64, u64, P]),
        "or_enumerate_path": (None, [gp, P]),
        "or_enumerate_centered": (None, [gp, P]),
        "or_exact_brute": (i32, [i64, P, P, P, ctypes.POINTER(u64)]),
        "or_exact_formula": (i32, [i64, P, P, P, ctypes.POINTER(u64)]),
        "or_alias_build": (i32, [P, i64, P, P]),
        "or_draw_alias": (u64, [P, P, P, i64, u64, u64, u32, u64]),
        "or_sample_path_alias": (None, [gp, P, P, u64, u64, u64, P]),
        "or_sample_centered_alias": (None, [gp, P, P, u64, u64, u64, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _csr(off, col):
    off = np.ascontiguousarray(off, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    if col.size == 0:
        col = np.zeros(1, dtype=np.int32)[:0]
    return off, col


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p) if a.size else None


def validate(off, col) -> int:
    off, col = _csr(off, col)
    return _load().or_validate(off.size - 1, _ptr(off), _ptr(col) if col.size else _ptr(np.zeros(1, np.int32)))


class Graph:
    """The oracle's prepared graph: relabelled CSR, tau/lambda prefixes, N_1."""

    def __init__(self, off, col):
        lib = _load()
        off, col = _csr(off, col)
        self._g = _Graph()
        colbuf = col if col.size else np.zeros(1, np.int32)
        st = lib.or_graph_build(off.size - 1, _ptr(off), _ptr(colbuf), ctypes.byref(self._g))
        if st != OK:
            raise OracleError(st, "or_graph_build")
        g = self._g
        n, slots = g.n, g.slots
        self.n = int(n)
        self.slots = int(slots)
        self.off = np.ctypeslib.as_array(g.off, shape=(n + 1,)).copy()
        self.col = np.ctypeslib.as_array(g.col, shape=(max(slots, 1),))[:slots].copy()
        self.rank = np.ctypeslib.as_array(g.rank, shape=(max(n, 1),))[:n].copy()
        self.p_tau = np.ctypeslib.as_array(g.p_tau, shape=(max(slots, 1),))[:slots].copy()
        self.p_lam = np.ctypeslib.as_array(g.p_lam, shape=(max(slots, 1),))[:slots].copy()
        self.R_tau = int(g.R_tau)
        self.R_lam = int(g.R_lam)
        self.N1 = int(g.N1)

    @property
    def W(self):
        """Number of 3-paths plus three times the triangles (Section 3)."""
        return self.R_tau // 2

    @property
    def Lam(self):
        """Lambda of Section 4."""
        return self.R_lam // 2

    def __del__(self):
        lib = _lib
        if lib is not None and hasattr(self, "_g"):
            lib.or_graph_free(ctypes.byref(self._g))

    def sample_path(self, seed: int, k: int, first: int = 0) -> np.ndarray:
        t = np.zeros(8, np.uint64)
        _load().or_sample_path(ctypes.byref(self._g), seed, first, k, _ptr(t))
        return t

    def sample_centered(self, seed: int, k: int, first: int = 0) -> np.ndarray:
        t = np.zeros(8, np.uint64)
        _load().or_sample_centered(ctypes.byref(self._g), seed, first, k, _ptr(t))
        return t

    def enumerate_path(self) -> np.ndarray:
        t = np.zeros(8, np.uint64)
        _load().or_enumerate_path(ctypes.byref(self._g), _ptr(t))
        return t

    def enumerate_centered(self) -> np.ndarray:
        t = np.zeros(8, np.uint64)
        _load().or_enumerate_centered(ctypes.byref(self._g), _ptr(t))
        return t

    def decode_path(self, r: int):
        q = np.zeros(4, np.int32)
        _load().or_decode_path(ctypes.byref(self._g), r, _ptr(q))
        return q

    def decode_centered(self, r: int):
        q = np.zeros(4, np.int32)
        _load().or_decode_centered(ctypes.byref(self._g), r, _ptr(q))
        return q

    def classify_path(self, q) -> int:
        q = np.ascontiguousarray(q, np.int32)
        return _load().or_classify_path(ctypes.byref(self._g), _ptr(q))

    def classify_centered(self, q) -> int:
        q = np.ascontiguousarray(q, np.int32)
        return _load().or_classify_centered(ctypes.byref(self._g), _ptr(q))

    def weights(self, centered: bool) -> np.ndarray:
        """tau (or lambda) per slot, from the inclusive prefix."""
        P = self.p_lam if centered else self.p_tau
        return np.diff(P, prepend=np.uint64(0)).astype(np.uint64)

    def alias_table(self, centered: bool):
        """(K, alias) of the sampler's weights (alias.c), built once."""
        key = "_alias_c" if centered else "_alias_p"
        if not hasattr(self, key):
            setattr(self, key, alias_build(self.weights(centered)))
        return getattr(self, key)

    def sample_path_alias(self, seed: int, k: int, first: int = 0) -> np.ndarray:
        t = np.zeros(8, np.uint64)
        if self.R_tau == 0:
            return t
        K, A = self.alias_table(False)
        _load().or_sample_path_alias(ctypes.byref(self._g), _ptr(K), _ptr(A), seed, first, k, _ptr(t))
        return t

    def sample_centered_alias(self, seed: int, k: int, first: int = 0) -> np.ndarray:
        t = np.zeros(8, np.uint64)
        if self.R_lam == 0:
            return t
        K, A = self.alias_table(True)
        _load().or_sample_centered_alias(ctypes.byref(self._g), _ptr(K), _ptr(A), seed, first, k, _ptr(t))
        return t

    def draw_alias(self, centered: bool, seed: int, sample_id: int) -> int:
        """r in [0, R) of one alias draw (tag 3 centered, 2 otherwise)."""
        K, A = self.alias_table(centered)
        P = self.p_lam if centered else self.p_tau
        R = self.R_lam if centered else self.R_tau
        return int(_load().or_draw_alias(_ptr(P), _ptr(K), _ptr(A), self.slots, R, seed, 3 if centered else 2,
                                         sample_id))


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, np.uint32)
    k = np.ascontiguousarray(key, np.uint32)
    out = np.zeros(4, np.uint32)
    _load().or_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def lemire(x: int, R: int, bits: int):
    """(accepted, r) for word x of the given width."""
    r = ctypes.c_uint64(0)
    ok = _load().or_lemire(x, R, bits, ctypes.byref(r))
    return bool(ok), int(r.value)


def draw(seed: int, tag: int, sample_id: int, R: int) -> int:
    return int(_load().or_draw(seed, tag, sample_id, R))


def draws(seed: int, tag: int, first: int, k: int, R: int) -> np.ndarray:
    """uint64[k]: draw(seed, tag, first + i, R) for i < k."""
    out = np.zeros(k, np.uint64)
    _load().or_draws(seed, tag, first, k, R, _ptr(out))
    return out


def alias_build(w):
    """(K uint64[N], alias int64[N]) of weights w (alias.c)."""
    w = np.ascontiguousarray(w, np.uint64)
    K = np.zeros(w.size, np.uint64)
    A = np.zeros(w.size, np.int64)
    st = _load().or_alias_build(_ptr(w), w.size, _ptr(K), _ptr(A))
    if st != OK:
        raise OracleError(st, "or_alias_build")
    return K, A


def exact_brute(off, col):
    """(C[1..6] as a 7-list with C[0]=0, triangles) by the definition."""
    off, col = _csr(off, col)
    C = np.zeros(7, np.uint64)
    T = ctypes.c_uint64(0)
    colbuf = col if col.size else np.zeros(1, np.int32)
    st = _load().or_exact_brute(off.size - 1, _ptr(off), _ptr(colbuf), _ptr(C), ctypes.byref(T))
    if st != OK:
        raise OracleError(st, "or_exact_brute")
    return [int(x) for x in C], int(T.value)


def exact_formula(off, col):
    """(C[1..6] as a 7-list with C[0]=0, triangles) through Eq. 1."""
    off, col = _csr(off, col)
    C = np.zeros(7, np.uint64)
    T = ctypes.c_uint64(0)
    colbuf = col if col.size else np.zeros(1, np.int32)
    st = _load().or_exact_formula(off.size - 1, _ptr(off), _ptr(colbuf), _ptr(C), ctypes.byref(T))
    if st != OK:
        raise OracleError(st, "or_exact_formula")
    return [int(x) for x in C], int(T.value)


def count_motifs(off, col, k: int, seed: int, delta: float = 0.01, k_cent: int | None = None):
    """The whole method on the oracle: both samplers, estimates, error bars."""
    from . import finalize

    g = Graph(off, col)
    kc = k if k_cent is None else k_cent
    tp = g.sample_path(seed, k)
    tc = g.sample_centered(seed, kc)
    res = finalize.finalize(tp, tc, g.R_tau, g.R_lam, g.N1, k, kc, delta)
    res["graph"] = g
    return res
