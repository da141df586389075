"""ctypes front end of the ORBGRAND CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It compiles ``orbgrand_oracle.c`` with the host C
compiler and exposes its functions with numpy arrays.  Nothing here touches the
GPU decoder or its sources.

Paper passages followed by the C code: Algorithm 1 (GRAND driver), Sec. III-A
(hard decision, reliability, permutation), Sec. III-B (logistic weight and the
distinct-part partition classes), Sec. III-C (Build-mountain, Algorithm 2
Landslide), Sec. I (membership of a linear code by a parity-check product),
Sec. IV-A (abandonment).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "orbgrand_oracle.c")
_LIB = os.path.join(_HERE, "liborbgrand_oracle.so")
_lib = None

WIDTH = 16  # ranks stored per pattern row by order_prefix


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, OpenMP); returns the library path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        # no contraction into fused multiply-adds: the FP32 fits run in the
        # order the source writes
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fopenmp", "-shared",
                               "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        i32p = ctypes.POINTER(ctypes.c_int)
        u8p = ctypes.c_void_p
        L.oracle_landslide.restype = ctypes.c_long
        L.oracle_landslide.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, i32p, ctypes.c_long]
        L.oracle_order_prefix.restype = ctypes.c_long
        L.oracle_order_prefix.argtypes = [ctypes.c_int, ctypes.c_long, ctypes.c_int, i32p, i32p]
        L.oracle_decode.restype = ctypes.c_int
        L.oracle_decode.argtypes = [u8p, u8p, ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                                    ctypes.c_long, u8p, u8p, u8p, ctypes.c_int]
        L.oracle_decode_ordered.restype = ctypes.c_int
        L.oracle_decode_ordered.argtypes = [u8p, u8p, ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                                            ctypes.c_long, u8p, u8p, u8p, u8p, ctypes.c_int]
        L.oracle_is_codeword.restype = ctypes.c_int
        L.oracle_is_codeword.argtypes = [u8p, ctypes.c_int, ctypes.c_int, u8p]
        L.oracle_permutation.restype = None
        L.oracle_permutation.argtypes = [u8p, ctypes.c_int, i32p]
        L.oracle_order1_prefix.restype = ctypes.c_long
        L.oracle_order1_prefix.argtypes = [ctypes.c_int, ctypes.c_long, ctypes.c_long, ctypes.c_int, i32p, i32p]
        L.oracle_fit_j0.restype = ctypes.c_long
        L.oracle_fit_j0.argtypes = [u8p, ctypes.c_int]
        L.oracle_decode_1line.restype = ctypes.c_int
        L.oracle_decode_1line.argtypes = [u8p, u8p, ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_long,
                                          u8p, u8p, u8p, u8p, ctypes.c_long, ctypes.c_int]
        lp = ctypes.POINTER(ctypes.c_long)
        L.oracle_order_mline_prefix.restype = ctypes.c_long
        L.oracle_order_mline_prefix.argtypes = [ctypes.c_int, ctypes.c_int, i32p, lp, lp, ctypes.c_long,
                                                ctypes.c_int, i32p, i32p]
        L.oracle_fit_mline.restype = ctypes.c_int
        L.oracle_fit_mline.argtypes = [u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int, i32p, i32p, lp, lp]
        L.oracle_decode_mline.restype = ctypes.c_int
        L.oracle_decode_mline.argtypes = [u8p, u8p, ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_long,
                                          ctypes.c_int, ctypes.c_int, u8p, u8p, u8p, u8p, ctypes.c_int]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def landslide(Wp: int, w: int, np_: int) -> list[tuple[int, ...]]:
    """All partitions u of W' into w non-decreasing parts <= n', Landslide order."""
    L = lib()
    total = L.oracle_landslide(Wp, w, np_, None, 0)
    if total == 0:
        return []
    out = np.zeros((total, w), dtype=np.int32)
    got = L.oracle_landslide(Wp, w, np_, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), total)
    assert got == total
    return [tuple(int(x) for x in row) for row in out]


def order_prefix(n: int, count: int) -> list[tuple[int, ...]]:
    """First `count` basic-ORBGRAND patterns for length n, as 1-based rank tuples."""
    L = lib()
    out = np.zeros((count, WIDTH), dtype=np.int32)
    wout = np.zeros(count, dtype=np.int32)
    got = L.oracle_order_prefix(n, count, WIDTH,
                                out.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                wout.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    if got < 0:
        raise ValueError("pattern wider than the row width")
    return [tuple(int(x) for x in out[g, :wout[g]]) for g in range(got)]


def order_prefix_array(n: int, count: int) -> np.ndarray:
    """First `count` patterns as an int32 [count, 16] array of ranks (zero padded)."""
    L = lib()
    out = np.zeros((count, WIDTH), dtype=np.int32)
    wout = np.zeros(count, dtype=np.int32)
    got = L.oracle_order_prefix(n, count, WIDTH,
                                out.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                wout.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    if got < 0:
        raise ValueError("pattern wider than the row width")
    return out[:got]


def decode(H: np.ndarray, llr: np.ndarray, budget: int, threads: int = 1):
    """Plain ORBGRAND on every row of llr.  Returns (codeword u8[N,n], queries u64[N],
    abandoned u8[N])."""
    H = np.ascontiguousarray(H, dtype=np.uint8)
    m, n = H.shape
    k = n - m
    llr = np.ascontiguousarray(np.atleast_2d(llr), dtype=np.float32)
    N = llr.shape[0]
    assert llr.shape[1] == n
    cw = np.zeros((N, n), dtype=np.uint8)
    q = np.zeros(N, dtype=np.uint64)
    ab = np.zeros(N, dtype=np.uint8)
    rc = lib().oracle_decode(_ptr(H), _ptr(llr), n, k, int(budget), N, _ptr(cw), _ptr(q), _ptr(ab),
                             int(threads))
    if rc != 0:
        raise ValueError("oracle_decode rejected its arguments")
    return cw, q, ab


def decode_ordered(H: np.ndarray, llr: np.ndarray, budget: int, order: np.ndarray, threads: int = 1):
    """Learned-order ORBGRAND: order[N,64] permutes the first 64 batches of 64 patterns."""
    H = np.ascontiguousarray(H, dtype=np.uint8)
    m, n = H.shape
    k = n - m
    llr = np.ascontiguousarray(np.atleast_2d(llr), dtype=np.float32)
    N = llr.shape[0]
    order = np.ascontiguousarray(np.atleast_2d(order), dtype=np.uint8)
    assert order.shape == (N, 64)
    cw = np.zeros((N, n), dtype=np.uint8)
    q = np.zeros(N, dtype=np.uint64)
    ab = np.zeros(N, dtype=np.uint8)
    rc = lib().oracle_decode_ordered(_ptr(H), _ptr(llr), n, k, int(budget), N, _ptr(order),
                                     _ptr(cw), _ptr(q), _ptr(ab), int(threads))
    if rc != 0:
        raise ValueError("oracle_decode_ordered rejected its arguments")
    return cw, q, ab


def is_codeword(H: np.ndarray, x: np.ndarray) -> bool:
    H = np.ascontiguousarray(H, dtype=np.uint8)
    m, n = H.shape
    x = np.ascontiguousarray(x, dtype=np.uint8)
    return bool(lib().oracle_is_codeword(_ptr(H), n, n - m, _ptr(x)))


def permutation(llr: np.ndarray) -> np.ndarray:
    llr = np.ascontiguousarray(llr, dtype=np.float32)
    n = llr.shape[0]
    pi = np.zeros(n, dtype=np.int32)
    lib().oracle_permutation(_ptr(llr), n, pi.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    return pi


# ---------------------------------------------------------------------------
# 1-line ORBGRAND (Sec. III-D/III-E with one segment; readings R10, R11 in the C source)
# ---------------------------------------------------------------------------
NO_FORCE = -(1 << 63)


def order1_prefix(n: int, j0: int, count: int) -> list[tuple[int, ...]]:
    """First `count` patterns of the 1-line order for (n, J0), as rank tuples."""
    L = lib()
    out = np.zeros((count, WIDTH), dtype=np.int32)
    wout = np.zeros(count, dtype=np.int32)
    got = L.oracle_order1_prefix(n, j0, count, WIDTH, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                 wout.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    assert got >= 0, got
    return [tuple(int(x) for x in out[g, :wout[g]]) for g in range(got)]


def order1_prefix_array(n: int, j0: int, count: int) -> np.ndarray:
    """First `count` 1-line patterns as an int32 [count, 16] array of ranks (zero padded)."""
    L = lib()
    out = np.zeros((count, WIDTH), dtype=np.int32)
    wout = np.zeros(count, dtype=np.int32)
    got = L.oracle_order1_prefix(n, j0, count, WIDTH, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                 wout.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    if got < 0:
        raise ValueError("pattern wider than the row width")
    return out[:got]


def fit_j0(llr: np.ndarray) -> int:
    """J0 of one block (1-D float32 LLRs)."""
    x = np.ascontiguousarray(llr, dtype=np.float32)
    return int(lib().oracle_fit_j0(_ptr(x), x.shape[0]))


def decode_1line(H: np.ndarray, llr: np.ndarray, budget: int, threads: int = 1, j0_force: int | None = None):
    """1-line ORBGRAND decode; returns (codewords u8 [N, n], queries u64 [N], abandoned u8 [N], J0 i32 [N])."""
    H = np.ascontiguousarray(H, dtype=np.uint8)
    llr = np.ascontiguousarray(llr, dtype=np.float32)
    N, n = llr.shape
    k = n - H.shape[0]
    cw = np.zeros((N, n), dtype=np.uint8)
    q = np.zeros(N, dtype=np.uint64)
    ab = np.zeros(N, dtype=np.uint8)
    j0 = np.zeros(N, dtype=np.int32)
    rc = lib().oracle_decode_1line(_ptr(H), _ptr(llr), n, k, budget, N, _ptr(cw), _ptr(q), _ptr(ab), _ptr(j0),
                                   NO_FORCE if j0_force is None else int(j0_force), threads)
    assert rc == 0, rc
    return cw, q, ab, j0


# ---------------------------------------------------------------------------
# Full (m-line) ORBGRAND (Sec. III-D, fit of Sec. III-E; readings R12-R15 in the C source)
# ---------------------------------------------------------------------------
MMAX = 8


def order_mline_prefix(n: int, I, J, beta, count: int, width: int = 32) -> list[tuple[int, ...]]:
    """First `count` patterns of the m-line order of the model (I[0..m], J[0..m-1],
    beta[0..m-1]) as 1-based rank tuples."""
    m = len(J)
    Ia = np.ascontiguousarray(I, dtype=np.int32)
    Ja = np.ascontiguousarray(J, dtype=np.int64)
    Ba = np.ascontiguousarray(beta, dtype=np.int64)
    assert Ia.shape[0] == m + 1 and Ba.shape[0] == m
    out = np.zeros((count, width), dtype=np.int32)
    wout = np.zeros(count, dtype=np.int32)
    lp = ctypes.POINTER(ctypes.c_long)
    i32p = ctypes.POINTER(ctypes.c_int)
    got = lib().oracle_order_mline_prefix(n, m, Ia.ctypes.data_as(i32p), Ja.ctypes.data_as(lp),
                                          Ba.ctypes.data_as(lp), count, width, out.ctypes.data_as(i32p),
                                          wout.ctypes.data_as(i32p))
    if got == -2:
        raise ValueError("invalid model")
    if got < 0:
        raise ValueError("pattern wider than the row width")
    return [tuple(int(x) for x in out[g, :wout[g]]) for g in range(got)]


def fit_mline(llr: np.ndarray, mreq: int, jdiv: bool = False):
    """Model of one block (1-D float32 LLRs) with at most mreq segments:
    returns (I, J, beta) as lists, len(J) = len(beta) = m, len(I) = m + 1."""
    x = np.ascontiguousarray(llr, dtype=np.float32)
    m = ctypes.c_int(0)
    I = np.zeros(MMAX + 1, dtype=np.int32)
    J = np.zeros(MMAX, dtype=np.int64)
    B = np.zeros(MMAX, dtype=np.int64)
    lp = ctypes.POINTER(ctypes.c_long)
    i32p = ctypes.POINTER(ctypes.c_int)
    rc = lib().oracle_fit_mline(_ptr(x), x.shape[0], int(mreq), int(bool(jdiv)), ctypes.byref(m),
                                I.ctypes.data_as(i32p), J.ctypes.data_as(lp), B.ctypes.data_as(lp))
    if rc != 0:
        raise ValueError("oracle_fit_mline rejected its arguments")
    mm = m.value
    return [int(v) for v in I[:mm + 1]], [int(v) for v in J[:mm]], [int(v) for v in B[:mm]]


def decode_mline(H: np.ndarray, llr: np.ndarray, budget: int, mreq: int, jdiv: bool = False, threads: int = 1):
    """m-line ORBGRAND decode; returns (codewords u8 [N, n], queries u64 [N], abandoned u8 [N],
    segment counts i32 [N])."""
    H = np.ascontiguousarray(H, dtype=np.uint8)
    llr = np.ascontiguousarray(np.atleast_2d(llr), dtype=np.float32)
    N, n = llr.shape
    k = n - H.shape[0]
    cw = np.zeros((N, n), dtype=np.uint8)
    q = np.zeros(N, dtype=np.uint64)
    ab = np.zeros(N, dtype=np.uint8)
    ms = np.zeros(N, dtype=np.int32)
    rc = lib().oracle_decode_mline(_ptr(H), _ptr(llr), n, k, int(budget), N, int(mreq), int(bool(jdiv)),
                                   _ptr(cw), _ptr(q), _ptr(ab), _ptr(ms), int(threads))
    if rc != 0:
        raise ValueError("oracle_decode_mline rejected its arguments")
    return cw, q, ab, ms
