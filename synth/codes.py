"""Seeded synthetic codes: parity-check matrices and generator bases.

This module builds inputs only; it holds none of the decoder's arithmetic and
is shared by the tests, the oracle legs and the benchmark.

* Random linear codes: H = [P | I_{n-k}] with P i.i.d. Bernoulli(1/2) drawn
  from a seeded numpy PCG64 generator.  The paper evaluates ORBGRAND on random
  linear codes (Sec. IV-A).
* Narrow-sense binary BCH(127, 113), t = 2: GF(2^7) built on the primitive
  polynomial x^7 + x^3 + 1; column i of H is the 7-bit vector of alpha^i
  stacked over the 7-bit vector of alpha^(3i) (zeros alpha and alpha^3).
* Generator basis of ker H by Gaussian elimination over GF(2).
"""
from __future__ import annotations

import numpy as np


def rlc_H(n: int, k: int, seed: int) -> np.ndarray:
    """(n-k) x n parity-check matrix [P | I] with P ~ Bernoulli(1/2)."""
    m = n - k
    rng = np.random.Generator(np.random.PCG64(seed))
    P = rng.integers(0, 2, size=(m, k), dtype=np.uint8)
    return np.concatenate([P, np.eye(m, dtype=np.uint8)], axis=1)


def gf2m_powers(m: int, poly: int) -> np.ndarray:
    """alpha^i for i = 0 .. 2^m - 2 in polynomial basis (bit j = coeff of x^j)."""
    order = (1 << m) - 1
    out = np.zeros(order, dtype=np.int64)
    a = 1
    for i in range(order):
        out[i] = a
        a <<= 1
        if a >> m:
            a ^= poly
    return out


def bch_H(n: int = 127, k: int = 113, poly: int = 0b10001001) -> np.ndarray:
    """Parity-check matrix of the narrow-sense double-error-correcting BCH code of
    length 2^m - 1 (default BCH(127, 113) on x^7 + x^3 + 1)."""
    m = (n + 1).bit_length() - 1
    assert (1 << m) - 1 == n and n - k == 2 * m, "only t = 2 narrow-sense codes"
    pw = gf2m_powers(m, poly)
    H = np.zeros((2 * m, n), dtype=np.uint8)
    for i in range(n):
        a1 = int(pw[i % n])
        a3 = int(pw[(3 * i) % n])
        for r in range(m):
            H[r, i] = (a1 >> r) & 1
            H[m + r, i] = (a3 >> r) & 1
    return H


def gf2_rank(A: np.ndarray) -> int:
    A = (np.array(A, dtype=np.uint8) & 1).copy()
    rows, cols = A.shape
    r = 0
    for c in range(cols):
        piv = None
        for i in range(r, rows):
            if A[i, c]:
                piv = i
                break
        if piv is None:
            continue
        A[[r, piv]] = A[[piv, r]]
        for i in range(rows):
            if i != r and A[i, c]:
                A[i] ^= A[r]
        r += 1
        if r == rows:
            break
    return r


def generator_matrix(H: np.ndarray) -> np.ndarray:
    """A basis of {x : H x = 0 over GF(2)} as the rows of G (dim x n)."""
    A = (np.array(H, dtype=np.uint8) & 1).copy()
    rows, n = A.shape
    pivots = []
    r = 0
    for c in range(n):
        piv = None
        for i in range(r, rows):
            if A[i, c]:
                piv = i
                break
        if piv is None:
            continue
        A[[r, piv]] = A[[piv, r]]
        for i in range(rows):
            if i != r and A[i, c]:
                A[i] ^= A[r]
        pivots.append(c)
        r += 1
        if r == rows:
            break
    free = [c for c in range(n) if c not in pivots]
    G = np.zeros((len(free), n), dtype=np.uint8)
    for j, f in enumerate(free):
        G[j, f] = 1
        for i, p in enumerate(pivots):
            G[j, p] = A[i, f]
    return G


def code(name: str):
    """The codes used by the workloads, by name: returns (H, G)."""
    table = {
        "rlc32_26": lambda: rlc_H(32, 26, seed=3226),
        "bch127_113": lambda: bch_H(127, 113),
        "rlc64_52": lambda: rlc_H(64, 52, seed=6452),
        "rlc128_116": lambda: rlc_H(128, 116, seed=128116),
        "rlc256_240": lambda: rlc_H(256, 240, seed=256240),
        "rlc256_234": lambda: rlc_H(256, 234, seed=256234),
        "rlc128_105": lambda: rlc_H(128, 105, seed=128105),
        "rlc512_490": lambda: rlc_H(512, 490, seed=512490),
    }
    H = table[name]()
    return H, generator_matrix(H)
