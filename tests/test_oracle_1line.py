"""Pins of the 1-line ORBGRAND oracle (the full ORBGRAND of Sec. III-D with one
segment): the order against brute-force sorting of all subsets by the
reliability weight J0 w + W of eq. (W2IJ) (beta = 1), the J0 = 0 reduction to
the basic order and decoder, the fit of eqs. (Q) and (quant) on curves whose J0
is known in closed form, and the decoder against brute force over all
codewords of tiny codes."""
import itertools
import os

import numpy as np
import pytest

from oracle import oracle as O
from synth import channel, codes

THREADS = min(8, os.cpu_count() or 1)


def _brute_1line(n, j0):
    subs = [c for w in range(n + 1) for c in itertools.combinations(range(1, n + 1), w)]
    return sorted(subs, key=lambda s: (j0 * len(s) + sum(s), len(s), s))


@pytest.mark.parametrize("n", [1, 2, 5, 8, 11])
@pytest.mark.parametrize("j0", [-1, 0, 1, 2, 5, 40])
def test_order_equals_brute_force(n, j0):
    assert O.order1_prefix(n, j0, 1 << n) == _brute_1line(n, j0)


def test_j0_zero_is_the_basic_order():
    for n in (8, 30, 127):
        assert O.order1_prefix(n, 0, 5000) == O.order_prefix(n, 5000)


def test_large_j0_takes_hamming_weight_first():
    """J0 above every reachable logistic weight: all single flips by rank, then
    pairs by W then lexicographically, ..."""
    n = 9
    got = O.order1_prefix(n, 1000, 1 << n)
    want = sorted((c for w in range(n + 1) for c in itertools.combinations(range(1, n + 1), w)),
                  key=lambda s: (len(s), sum(s), s))
    assert got == want


def _llr_from_sorted(mags, seed=0):
    """LLRs with the given sorted magnitudes, shuffled, random signs."""
    rng = np.random.default_rng(seed)
    m = np.asarray(mags, dtype=np.float32)
    perm = rng.permutation(m.shape[0])
    sign = rng.choice(np.array([-1.0, 1.0], dtype=np.float32), size=m.shape[0])
    return (m[perm] * sign).astype(np.float32)


@pytest.mark.parametrize("a,b,n,want", [
    (3.0, 0.5, 20, 6),       # L_i = 3 + 0.5 i: L_1 = 3.5, Q = 0.5, [7] - 1
    (0.0, 1.0, 30, 0),       # basic model through the origin: L_1 / Q = 1
    (0.0, 0.25, 64, 0),
    (10.0, 2.0, 127, 5),     # L_1 = 12, Q = 2, [6] - 1
    (-0.4, 1.0, 16, 0),      # L_1 = 0.6, Q = 1: [0.6] = 1
    (-0.8, 1.0, 16, -1),     # L_1 = 0.2, Q = 1: [0.2] = 0
    (1e4, 1e-3, 40, 1 << 20),  # L_1 / Q = 1e7: capped at 2^20, minus one
])
def test_fit_on_lines(a, b, n, want):
    mags = [a + b * i for i in range(1, n + 1)]
    if want == 1 << 20:
        want -= 1
    assert O.fit_j0(_llr_from_sorted(mags, seed=n)) == want


def test_fit_rounds_half_up_and_uses_floor_n_half():
    # n = 9: h = 4; L_1 = 2.5, L_4 = 5.5: Q = 1, L_1/Q = 2.5 -> [2.5] = 3, J0 = 2
    mags = [2.5, 3.5, 4.5, 5.5, 100.0, 100.0, 100.0, 100.0, 100.0]
    assert O.fit_j0(_llr_from_sorted(mags, seed=1)) == 2
    # the same with L_1 = 2.4: [2.4] = 2 -> J0 = 1 (Q = 3.1 / 3)
    mags2 = [2.4, 3.5, 4.5, 5.5, 100.0, 100.0, 100.0, 100.0, 100.0]
    q = np.float32(np.float32(5.5) - np.float32(2.4)) / np.float32(3)
    assert O.fit_j0(_llr_from_sorted(mags2, seed=2)) == int(np.floor(np.float32(2.4) / q + np.float32(0.5))) - 1


def test_fit_degenerate_cases_give_basic():
    assert O.fit_j0(np.full(40, 3.0, dtype=np.float32)) == 0          # Q = 0
    assert O.fit_j0(np.array([1.0, 2.0, 3.0], dtype=np.float32)) == 0  # h < 2
    x = np.linspace(1, 5, 40).astype(np.float32)
    x[7] = np.nan
    assert O.fit_j0(x) == O.fit_j0(x)                                   # deterministic
    y = np.linspace(1, 5, 40).astype(np.float32)
    y[:25] = np.inf
    assert O.fit_j0(y) == 0                                             # infinite magnitudes


def test_j0_forced_zero_equals_basic_decoder():
    H, G = codes.code("rlc32_26")
    llr, _ = channel.awgn_llr(G, 2000, 4.0, seed=5)
    c0, q0, a0 = O.decode(H, llr, 10 ** 4, THREADS)
    c1, q1, a1, j = O.decode_1line(H, llr, 10 ** 4, THREADS, j0_force=0)
    assert (c0 == c1).all() and (q0 == q1).all() and (a0 == a1).all() and (j == 0).all()


def _tiny_code(n, k, seed):
    rng = np.random.default_rng(seed)
    P = rng.integers(0, 2, size=(n - k, k), dtype=np.uint8)
    H = np.concatenate([P, np.eye(n - k, dtype=np.uint8)], axis=1)
    return H, codes.generator_matrix(H)


@pytest.mark.parametrize("n,k,seed", [(8, 4, 1), (10, 6, 2), (12, 7, 3)])
def test_decoder_equals_brute_force(n, k, seed):
    """Over all 2^k codewords c: the returned word minimises the key
    (J0 w_H(e) + w_L(e), w_H(e), ranks of e) of e = y xor c in rank space, and
    q = 1 + the number of patterns with a smaller key; J0 is the block's fit."""
    H, G = _tiny_code(n, k, seed)
    rng = np.random.default_rng(seed)
    msgs = np.array(list(itertools.product([0, 1], repeat=k)), dtype=np.uint8)
    cws = channel.encode(G, msgs)
    N = 60
    # offsets and slopes that spread J0 over -1 .. ~8
    llr = np.empty((N, n), dtype=np.float32)
    for b in range(N):
        off, slope = rng.uniform(0, 4), rng.uniform(0.2, 1.5)
        mags = off + slope * np.arange(1, n + 1) + rng.uniform(0, 0.1, n)
        llr[b] = _llr_from_sorted(mags.astype(np.float32), seed=seed * 100 + b)
    cw, q, ab, j0 = O.decode_1line(H, llr, 1 << n, THREADS)
    assert len(set(j0.tolist())) > 3
    for b in range(N):
        y = (llr[b] > 0).astype(np.uint8)
        pi = O.permutation(llr[b])
        rank = np.empty(n, dtype=np.int64)
        rank[pi] = np.arange(1, n + 1)
        J = int(j0[b])

        def key(c):
            e = np.nonzero(y ^ c)[0]
            r = tuple(sorted(int(rank[i]) for i in e))
            return (J * len(r) + sum(r), len(r), r)
        best = min(cws, key=key)
        assert (cw[b] == best).all() and ab[b] == 0
        kb = key(best)
        smaller = sum(1 for s in _brute_1line(n, J) if (J * len(s) + sum(s), len(s), s) < kb)
        assert int(q[b]) == smaller + 1


def test_members_and_budget_rules():
    H, G = codes.code("bch127_113")
    llr, _ = channel.awgn_llr(G, 300, 6.0, seed=9)
    cw, q, ab, j0 = O.decode_1line(H, llr, 3000, THREADS)
    assert ((q >= 1) & (q <= 3000)).all() and (q[ab == 1] == 3000).all()
    for b in np.nonzero(ab == 0)[0]:
        assert O.is_codeword(H, cw[b])
    assert (j0 >= -1).all() and len(set(j0.tolist())) > 3
    # a smaller budget truncates exactly, as for the basic order
    c2, q2, a2, _ = O.decode_1line(H, llr, 50, THREADS)
    kept = q <= 50
    assert (q2[kept] == q[kept]).all() and (c2[kept] == cw[kept]).all() and (a2[~kept] == 1).all()
