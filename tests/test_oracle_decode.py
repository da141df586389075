"""Pins of the oracle decoder (Algorithm 1 with the basic ORBGRAND order) against
brute force over all codewords of tiny codes, the soft-ML special case of
eq. (lw1), membership invariants and the budget / abandonment rules."""
import itertools
import struct

import numpy as np
import pytest

from oracle import oracle as O
from synth import channel, codes

THREADS = 4


def _abs_bits(x):
    return struct.unpack("<I", struct.pack("<f", abs(np.float32(x))))[0]


def _ranks_of(llr):
    """rank (1-based) of each received index; independent plain-Python sort on
    (bits of |LLR|, index)."""
    n = len(llr)
    order = sorted(range(n), key=lambda i: (_abs_bits(llr[i]), i))
    rank = [0] * n
    for j, i in enumerate(order):
        rank[i] = j + 1
    return rank


def _brute_order(n):
    subs = [c for w in range(n + 1) for c in itertools.combinations(range(1, n + 1), w)]
    subs.sort(key=lambda c: (sum(c), len(c), c))
    return subs


def _codebook(G):
    k, n = G.shape
    out = []
    for m in itertools.product([0, 1], repeat=k):
        out.append((np.array(m, dtype=np.int64) @ G.astype(np.int64)) % 2)
    return np.array(out, dtype=np.uint8)


def _brute_decode(book, index_of, llr, budget):
    """ORB-ML by exhaustion: the codeword whose noise pattern comes first in the
    (W, w, lex) order; q = its 1-based position."""
    y = (llr > 0).astype(np.uint8)
    rank = _ranks_of(llr)
    best = None
    for c in book:
        e = np.nonzero(y ^ c)[0]
        v = tuple(sorted(rank[i] for i in e))
        pos = index_of[v]
        if best is None or pos < best[0]:
            best = (pos, c)
    q = best[0] + 1
    if q > budget:
        return y, budget, 1
    return best[1], q, 0


def _tiny_code(n, k, seed):
    H = codes.rlc_H(n, k, seed)
    return H, codes.generator_matrix(H)


@pytest.mark.parametrize("n,k,seed", [(8, 3, 1), (10, 4, 2), (12, 5, 3), (14, 6, 4), (13, 9, 5)])
def test_matches_brute_force_ml_order(n, k, seed):
    H, G = _tiny_code(n, k, seed)
    book = _codebook(G)
    order = _brute_order(n)
    index_of = {v: i for i, v in enumerate(order)}
    rng = np.random.default_rng(seed)
    N = 60
    llr = (rng.standard_normal((N, n)) * 2.0 + (2 * book[rng.integers(0, len(book), N)] - 1)).astype(np.float32)
    for budget in (2 ** n, 7, 1):
        cw, q, ab = O.decode(H, llr, budget)
        for b in range(N):
            ec, eq, ea = _brute_decode(book, index_of, llr[b], budget)
            assert (cw[b] == ec).all() and int(q[b]) == eq and int(ab[b]) == ea, (b, budget)


def test_soft_ml_special_case_linear_reliabilities():
    """With |LLR| of the j-th least reliable bit equal to j (times a constant),
    Rel(z) = w_L(z) (eq. (lw1)), so the decoding attains min_c sum |LLR_i| (y+c)_i."""
    n, k = 12, 5
    H, G = _tiny_code(n, k, 11)
    book = _codebook(G)
    rng = np.random.default_rng(5)
    for _ in range(40):
        perm = rng.permutation(n)
        mag = np.empty(n)
        mag[perm] = 0.37 * np.arange(1, n + 1)
        sign = rng.choice([-1.0, 1.0], n)
        llr = (sign * mag).astype(np.float32)
        cw, q, ab = O.decode(H, llr[None], 2 ** n)
        y = (llr > 0).astype(np.uint8)
        cost = lambda c: float(np.sum(np.abs(llr) * (y ^ c)))
        best = min(cost(c) for c in book)
        assert ab[0] == 0
        assert abs(cost(cw[0]) - best) < 1e-4


def test_zero_syndrome_and_no_earlier_hit():
    H, G = codes.code("rlc32_26")
    from synth import channel
    llr, _ = channel.awgn_llr(G, 200, 3.0, seed=9)
    cw, q, ab = O.decode(H, llr, 10 ** 4)
    pats = O.order_prefix(32, 10 ** 4)
    for b in range(200):
        assert 1 <= q[b] <= 10 ** 4
        if ab[b]:
            assert q[b] == 10 ** 4
            continue
        assert O.is_codeword(H, cw[b])
        y = (llr[b] > 0).astype(np.uint8)
        pi = np.array(sorted(range(32), key=lambda i: (_abs_bits(llr[b][i]), i)))
        Hi = H.astype(np.int64)
        for g in range(int(q[b]) - 1):
            x = y.copy()
            for r in pats[g]:
                x[pi[r - 1]] ^= 1
            assert ((Hi @ x) % 2).any(), (b, g)
        x = y.copy()
        for r in pats[int(q[b]) - 1]:
            x[pi[r - 1]] ^= 1
        assert (x == cw[b]).all()


def test_budget_edges_and_abandon():
    H, G = _tiny_code(16, 6, 21)
    rng = np.random.default_rng(1)
    llr = rng.standard_normal((50, 16)).astype(np.float32)      # pure noise
    cw, q, ab = O.decode(H, llr, 2 ** 16)
    assert not ab.any()
    for b in range(50):
        qq = int(q[b])
        c1, q1, a1 = O.decode(H, llr[b:b + 1], qq)              # budget == q: found
        assert a1[0] == 0 and q1[0] == qq and (c1[0] == cw[b]).all()
        if qq > 1:
            c2, q2, a2 = O.decode(H, llr[b:b + 1], qq - 1)      # one short: abandon
            y = (llr[b] > 0).astype(np.uint8)
            assert a2[0] == 1 and q2[0] == qq - 1 and (c2[0] == y).all()
    # y already a codeword: q = 1 even with budget 1
    book = _codebook(G)
    llr = (2.0 * book[3].astype(np.float32) - 1.0) * 3.0
    c, q, a = O.decode(H, llr[None], 1)
    assert q[0] == 1 and a[0] == 0 and (c[0] == book[3]).all()


def test_hard_decision_and_tie_rules():
    """Reading R1 (only LLR > 0 decides 1; +-0 and NaN give 0) and reading R2
    (equal reliabilities ranked by received index)."""
    llr = np.array([0.0, -0.0, 1.0, -1.0, np.nan, 2.0, -2.0, 1.0], dtype=np.float32)
    pi = O.permutation(llr)
    assert list(pi) == [0, 1, 2, 3, 7, 5, 6, 4]                 # NaN bits sort last
    n = 8
    H, G = _tiny_code(n, 3, 2)
    cw, q, ab = O.decode(H, llr[None], 2 ** n)
    book = _codebook(G)
    order = _brute_order(n)
    index_of = {v: i for i, v in enumerate(order)}
    y = np.array([0, 0, 1, 0, 0, 1, 0, 1], dtype=np.uint8)
    rank = [0] * n
    for j, i in enumerate(pi):
        rank[i] = j + 1
    best = min(book, key=lambda c: index_of[tuple(sorted(rank[i] for i in np.nonzero(y ^ c)[0]))])
    assert (cw[0] == best).all()
    # all-equal reliabilities: rank follows the received index
    llr = np.full(10, -0.5, dtype=np.float32)
    assert list(O.permutation(llr)) == list(range(10))


def test_argument_validation():
    H, _ = _tiny_code(8, 3, 1)
    llr = np.zeros((1, 8), dtype=np.float32)
    with pytest.raises(ValueError):
        O.decode(H, llr, 0)
    Hb = H.copy()
    Hb[0, 0] = 2
    with pytest.raises(ValueError):
        O.decode(Hb, llr, 10)


def _brute_ordered(book, order_list, llr, budget, perm):
    y = (llr > 0).astype(np.uint8)
    rank = _ranks_of(llr)
    member = {tuple(c) for c in book}
    pi = sorted(range(len(llr)), key=lambda i: (_abs_bits(llr[i]), i))
    seq = [g for b in (int(x) for x in perm) for g in range(64 * b, 64 * b + 64) if g < len(order_list)]
    seq += list(range(4096, len(order_list)))
    for pos, g in enumerate(seq[:budget]):
        x = y.copy()
        for r in order_list[g]:
            x[pi[r - 1]] ^= 1
        if tuple(x) in member:
            return x, pos + 1, 0
    return y, budget, 1


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_ordered_decode_brute_force(seed):
    n, k = 13, 5
    H, G = _tiny_code(n, k, 40 + seed)
    book = _codebook(G)
    order_list = _brute_order(n)
    rng = np.random.default_rng(seed)
    N = 40
    llr = (rng.standard_normal((N, n)) * 1.5).astype(np.float32)
    perm = np.stack([rng.permutation(64) for _ in range(N)]).astype(np.uint8)
    for budget in (2 ** n, 100, 3):
        cw, q, ab = O.decode_ordered(H, llr, budget, perm)
        for b in range(N):
            ec, eq, ea = _brute_ordered(book, order_list, llr[b], budget, perm[b])
            assert (cw[b] == ec).all() and int(q[b]) == eq and int(ab[b]) == ea


def test_ordered_identity_equals_plain_and_far_hits_unchanged():
    H, G = codes.code("rlc32_26")
    from synth import channel
    llr, _ = channel.awgn_llr(G, 300, 2.0, seed=17)
    ident = np.tile(np.arange(64, dtype=np.uint8), (300, 1))
    c0, q0, a0 = O.decode(H, llr, 10 ** 4)
    c1, q1, a1 = O.decode_ordered(H, llr, 10 ** 4, ident)
    assert (c0 == c1).all() and (q0 == q1).all() and (a0 == a1).all()
    # 16 parity bits and pure-noise LLRs: many first hits lie beyond g = 4096,
    # where any permutation of the prefix leaves the result unchanged
    H = codes.rlc_H(24, 8, seed=77)
    rng = np.random.default_rng(3)
    llr = rng.standard_normal((120, 24)).astype(np.float32)
    c0, q0, a0 = O.decode(H, llr, 10 ** 5)
    perm = np.stack([rng.permutation(64) for _ in range(120)]).astype(np.uint8)
    c2, q2, a2 = O.decode_ordered(H, llr, 10 ** 5, perm)
    far = q0 > 4096
    assert far.sum() >= 20
    assert (c2[far] == c0[far]).all() and (q2[far] == q0[far]).all() and (a2[far] == a0[far]).all()
    near = ~far
    assert (q2[near] <= 4096).all()


def test_budget_truncation_is_exact():
    """A decode with a smaller budget b returns the full-budget result for blocks with
    q <= b and abandons the others with q = b and the hard decision (the order of
    patterns does not depend on the budget).  This is what makes the abandonment sweep
    of one decode exact."""
    H, G = codes.code("bch127_113")
    llr, _ = channel.awgn_llr(G, 300, 4.0, seed=77)
    cw, q, ab = O.decode(H, llr, 10 ** 4, THREADS)
    y = (llr > 0).astype(np.uint8)
    for b in (1, 7, 64, 500, 3000):
        cb, qb, abb = O.decode(H, llr, b, THREADS)
        kept = q <= b
        assert (qb[kept] == q[kept]).all() and (abb[kept] == ab[kept]).all() and (cb[kept] == cw[kept]).all()
        assert (qb[~kept] == b).all() and (abb[~kept] == 1).all() and (cb[~kept] == y[~kept]).all()
