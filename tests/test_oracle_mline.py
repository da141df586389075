"""Pins of the full (m-line) ORBGRAND oracle of Sec. III-D/III-E: the order against a
brute-force sort of all subsets by the key the section fixes (reliability
weight of eq. (W2IJ), then the split pattern in the nested-loop order of the
integer splitting algorithm, then the Cartesian product of eq. (cartP) with
each partial set by Hamming weight and Landslide order); invariants of the
model (a common scale of all J and beta, the basic and 1-line special cases);
the fit of eqs. (Q) and (quant) on piecewise-linear curves whose anchors and
quantized parameters are known by hand; and the decoder against brute force
over all codewords of tiny codes."""
import itertools
import os

import numpy as np
import pytest

from oracle import oracle as O
from synth import channel, codes

THREADS = min(8, os.cpu_count() or 1)


def _key(s, I, J, beta):
    """Sort key of the pattern s (ascending 1-based ranks) under the model."""
    m = len(J)
    parts, Ws = [], []
    for i in range(m):
        v = tuple(r - I[i] for r in s if I[i] < r <= I[i + 1])
        Ws.append(J[i] * len(v) + beta[i] * sum(v))
        parts.append((len(v), v))
    return (sum(Ws), tuple(Ws), tuple(parts))


def _brute(n, I, J, beta):
    subs = [c for w in range(n + 1) for c in itertools.combinations(range(1, n + 1), w)]
    return sorted(subs, key=lambda s: _key(s, I, J, beta))


MODELS = [
    (8, [0, 3, 8], [0, 2], [1, 2]),
    (8, [0, 2, 8], [-1, 3], [1, 1]),         # J0 = -beta1: rank 1 alone has weight 0
    (9, [0, 2, 5, 9], [-2, 3, 7], [2, 1, 3]),
    (10, [0, 4, 10], [5, 1], [3, 2]),
    (10, [0, 1, 2, 10], [0, 0, 0], [1, 1, 1]),
    (7, [0, 7], [2], [3]),
    (10, [0, 3, 6, 8, 10], [-3, 4, 9, 12], [3, 2, 2, 1]),
    (10, [0, 5, 10], [-2, 0], [2, 1]),
    (11, [0, 2, 4, 6, 11], [0, 3, 6, 10], [1, 1, 2, 2]),
]


@pytest.mark.parametrize("n,I,J,beta", MODELS)
def test_order_equals_brute_force(n, I, J, beta):
    got = O.order_mline_prefix(n, I, J, beta, 1 << n)
    assert got == _brute(n, I, J, beta)


def test_order_hand_example():
    """Ranks 1..3 weigh 1, 2, 3 and ranks 4..6 weigh 4, 6, 8: weight 5 holds
    {1,4} (split (1,4)) before {2,3} (split (5,0)); weight 7 holds {1,5}, then
    {3,4} and {1,2,4} (split (3,4), partial weight 3 by one flip, then two)."""
    got = O.order_mline_prefix(6, [0, 3, 6], [0, 2], [1, 2], 17)
    assert got == [(), (1,), (2,), (3,), (1, 2), (4,), (1, 3), (1, 4), (2, 3), (5,), (2, 4),
                   (1, 2, 3), (1, 5), (3, 4), (1, 2, 4), (6,), (2, 5)]


@pytest.mark.parametrize("j0", [-1, 0, 3, 17])
def test_one_segment_unit_slope_is_the_1line_order(j0):
    assert O.order_mline_prefix(127, [0, 127], [j0], [1], 5000) == O.order1_prefix(127, j0, 5000)


@pytest.mark.parametrize("beta", [1, 2, 7])
def test_one_segment_through_the_origin_is_the_basic_order(beta):
    """J0 = 0 scales every weight by beta: the basic order (eq. (llr2i))."""
    assert O.order_mline_prefix(63, [0, 63], [0], [beta], 4000) == O.order_prefix(63, 4000)


def test_common_scale_leaves_the_order():
    I, J, beta = [0, 5, 17, 40], [1, 9, 30], [1, 2, 4]
    base = O.order_mline_prefix(40, I, J, beta, 3000)
    for c in (2, 3):
        assert O.order_mline_prefix(40, I, [c * x for x in J], [c * x for x in beta], 3000) == base


def test_three_segments_n16_every_pattern():
    """All 2^16 patterns of a three-segment model, each once, in key order."""
    n, I, J, beta = 16, [0, 3, 9, 16], [0, 4, 15], [1, 2, 3]
    assert O.order_mline_prefix(n, I, J, beta, 1 << n) == _brute(n, I, J, beta)


def test_invalid_models_are_rejected():
    for args in [(8, [0, 3, 7], [0, 1], [1, 1]),     # I_m != n
                 (8, [0, 3, 3, 8], [0, 1, 1], [1, 1, 1]),
                 (8, [0, 8], [0], [0]),              # beta < 1
                 (8, [0, 8], [-2], [1])]:            # J < -beta
        with pytest.raises(ValueError):
            O.order_mline_prefix(*args, 10)


def _llr_from_sorted(mags, seed=0):
    rng = np.random.default_rng(seed)
    m = np.asarray(mags, dtype=np.float32)
    perm = rng.permutation(m.shape[0])
    sign = rng.choice(np.array([-1.0, 1.0], dtype=np.float32), size=m.shape[0])
    return (m[perm] * sign).astype(np.float32)


def test_fit_two_segment_curve():
    """L_j = j up to rank 4, then slope 3; n = 20 (h = 10).  The chord from
    rank 1 to 10 is farthest from the curve at the corner, rank 4; both
    segments are then exact lines, so no third anchor is added."""
    mags = [float(j) if j <= 4 else 4.0 + 3.0 * (j - 4) for j in range(1, 21)]
    llr = _llr_from_sorted(mags, seed=3)
    for mreq in (2, 3, 8):
        assert O.fit_mline(llr, mreq) == ([0, 4, 20], [0, 4], [1, 3])


def test_fit_three_segment_curve():
    """Slopes 0.5, 1, 2.5 between ranks 1-5, 5-12, 12-20 (n = 40, h = 20),
    offset so that the roundings fall on halves: Q = 0.5, beta = (1, 2, 5),
    J0 = [0.75/0.5] - 1 = 1, J1 = [2.75/0.5] = 6, J2 = [9.75/0.5] = 20."""
    def L(j):
        if j <= 5:
            return 0.25 + 0.5 * j
        if j <= 12:
            return 2.75 + 1.0 * (j - 5)
        if j <= 20:
            return 9.75 + 2.5 * (j - 12)
        return 29.75 + 5.0 * (j - 20)
    llr = _llr_from_sorted([L(j) for j in range(1, 41)], seed=4)
    assert O.fit_mline(llr, 3) == ([0, 5, 12, 40], [1, 6, 20], [1, 2, 5])
    # the J/beta variant: [1/1] 1, [6/2] 2, [20/5] 5
    assert O.fit_mline(llr, 3, jdiv=True) == ([0, 5, 12, 40], [1, 6, 20], [1, 2, 5])
    # the first anchor found is rank 12 (gap about 7.8 against 4.1 at rank 5);
    # with it alone: Q = 9/11 (chord 1-12), beta2 = [20 / (8 Q)] = [3.06] = 3,
    # J0 = [0.75 / Q] - 1 = [0.92] - 1 = 0, J1 = [9.75 / Q] = [11.92] = 12
    assert O.fit_mline(llr, 2) == ([0, 12, 40], [0, 12], [1, 3])


def test_fit_j_beta_rounding():
    """Slopes 1, 2, 5 from the origin-free curve L_j = j (j <= 5), 5 + 2(j-5)
    (j <= 12), 19 + 5(j-12): J = (0, 5, 19), beta = (1, 2, 5); the J/beta
    variant rounds 5/2 = 2.5 up to 3 (J1 = 6) and 19/5 = 3.8 to 4 (J2 = 20)."""
    def L(j):
        if j <= 5:
            return float(j)
        if j <= 12:
            return 5.0 + 2.0 * (j - 5)
        return 19.0 + 5.0 * (j - 12)
    llr = _llr_from_sorted([L(j) for j in range(1, 41)], seed=5)
    assert O.fit_mline(llr, 3) == ([0, 5, 12, 40], [0, 5, 19], [1, 2, 5])
    assert O.fit_mline(llr, 3, jdiv=True) == ([0, 5, 12, 40], [0, 6, 20], [1, 2, 5])


def test_fit_gap_ties_take_the_lower_rank():
    """L_j = j except L_4 = 3 and L_7 = 6: the chord 1-10 misses both by 1."""
    mags = [1, 2, 3, 3, 5, 6, 6, 8, 9, 10] + [11 + j for j in range(10)]
    I, _, _ = O.fit_mline(_llr_from_sorted(mags, seed=6), 2)
    assert I == [0, 4, 20]


def test_fit_one_segment_is_the_1line_fit():
    rng = np.random.default_rng(11)
    for b in range(300):
        n = int(rng.integers(4, 130))
        llr = (rng.normal(0, 1, n) * rng.uniform(0.2, 6) + rng.uniform(-3, 3)).astype(np.float32)
        I, J, beta = O.fit_mline(llr, 1)
        assert I == [0, n] and beta == [1] and J == [O.fit_j0(llr)]


def test_fit_degenerate_cases_give_basic():
    basic40 = ([0, 40], [0], [1])
    assert O.fit_mline(np.full(40, 3.0, dtype=np.float32), 3) == basic40           # Q = 0
    assert O.fit_mline(np.array([1, 2, 3], dtype=np.float32), 3) == ([0, 3], [0], [1])  # h < 2
    y = np.linspace(1, 5, 40).astype(np.float32)
    y[:25] = np.inf
    assert O.fit_mline(y, 3) == basic40
    # ranks 1-9 equal: the second anchor is rank 9 (gap 6.2) and the first
    # segment is flat, Q = 0: basic model; one line alone has Q = 7/9 and
    # J0 = [3 / Q] - 1 = [3.86] - 1 = 3
    mags = [3.0] * 9 + [10.0] + [11.0 + j for j in range(10)]
    llr = _llr_from_sorted(mags, seed=7)
    assert O.fit_mline(llr, 2) == ([0, 20], [0], [1])
    assert O.fit_mline(llr, 1) == ([0, 20], [3], [1])


def test_fit_anchor_count_and_bounds():
    """Any block: at most mreq segments, 0 = I_0 < ... < I_m = n with the inner
    anchors inside [2, h - 1], beta >= 1, J0 >= -beta1, J_i >= 0."""
    rng = np.random.default_rng(12)
    for b in range(400):
        n = int(rng.integers(4, 200))
        mreq = int(rng.integers(1, 9))
        llr = (rng.normal(0, 1, n) * rng.uniform(0.2, 6) + rng.uniform(-3, 3)).astype(np.float32)
        I, J, beta = O.fit_mline(llr, mreq)
        m = len(J)
        assert 1 <= m <= mreq and len(I) == m + 1 and I[0] == 0 and I[-1] == n
        assert all(a < b for a, b in zip(I, I[1:]))
        assert all(2 <= a <= n // 2 - 1 for a in I[1:-1])
        assert all(x >= 1 for x in beta) and J[0] >= -beta[0] and all(x >= 0 for x in J[1:])


def _tiny_code(n, k, seed):
    rng = np.random.default_rng(seed)
    P = rng.integers(0, 2, size=(n - k, k), dtype=np.uint8)
    H = np.concatenate([P, np.eye(n - k, dtype=np.uint8)], axis=1)
    return H, codes.generator_matrix(H)


@pytest.mark.parametrize("n,k,seed,mreq,jdiv", [(8, 4, 1, 2, False), (10, 6, 2, 3, False),
                                                (12, 7, 3, 3, False), (12, 7, 4, 4, True),
                                                (12, 8, 5, 2, True)])
def test_decoder_equals_brute_force(n, k, seed, mreq, jdiv):
    """Over all 2^k codewords c: the returned word minimises the order key of
    e = y xor c in rank space under the block's fitted model, and q = 1 + the
    number of the 2^n patterns with a smaller key."""
    H, G = _tiny_code(n, k, seed)
    rng = np.random.default_rng(seed)
    msgs = np.array(list(itertools.product([0, 1], repeat=k)), dtype=np.uint8)
    cws = channel.encode(G, msgs)
    N = 40
    llr = np.empty((N, n), dtype=np.float32)
    for b in range(N):
        j = np.arange(1, n + 1)
        mags = rng.uniform(0, 2) + rng.uniform(0.1, 1) * j + rng.uniform(0, 0.4) * j * j \
            + rng.uniform(0, 0.2, n)
        llr[b] = _llr_from_sorted(np.sort(mags).astype(np.float32), seed=seed * 100 + b)
    cw, q, ab, ms = O.decode_mline(H, llr, 1 << n, mreq, jdiv, THREADS)
    assert ms.max() > 1
    subs = [c for w in range(n + 1) for c in itertools.combinations(range(1, n + 1), w)]
    for b in range(N):
        I, J, beta = O.fit_mline(llr[b], mreq, jdiv)
        assert ms[b] == len(J)
        y = (llr[b] > 0).astype(np.uint8)
        pi = O.permutation(llr[b])
        rank = np.empty(n, dtype=np.int64)
        rank[pi] = np.arange(1, n + 1)

        def key(c):
            e = np.nonzero(y ^ c)[0]
            return _key(tuple(sorted(int(rank[i]) for i in e)), I, J, beta)
        best = min(cws, key=key)
        assert (cw[b] == best).all() and ab[b] == 0
        kb = key(best)
        assert int(q[b]) == 1 + sum(1 for s in subs if _key(s, I, J, beta) < kb)


def test_one_segment_decoder_is_the_1line_decoder():
    H, G = codes.code("bch127_113")
    llr, _ = channel.awgn_llr(G, 300, 5.0, seed=21)
    c1, q1, a1, _ = O.decode_1line(H, llr, 3000, THREADS)
    cm, qm, am, ms = O.decode_mline(H, llr, 3000, 1, False, THREADS)
    assert (c1 == cm).all() and (q1 == qm).all() and (a1 == am).all() and (ms == 1).all()


def test_members_and_budget_rules():
    H, G = codes.code("bch127_113")
    llr, _ = channel.awgn_llr(G, 200, 6.0, seed=22)
    cw, q, ab, ms = O.decode_mline(H, llr, 2000, 3, False, THREADS)
    assert ((q >= 1) & (q <= 2000)).all() and (q[ab == 1] == 2000).all()
    assert ms.max() == 3
    for b in np.nonzero(ab == 0)[0]:
        assert O.is_codeword(H, cw[b])
    c2, q2, a2, _ = O.decode_mline(H, llr, 40, 3, False, THREADS)
    kept = q <= 40
    assert (q2[kept] == q[kept]).all() and (c2[kept] == cw[kept]).all() and (a2[~kept] == 1).all()


def test_argument_errors():
    H, G = codes.code("rlc32_26")
    llr, _ = channel.awgn_llr(G, 4, 4.0, seed=1)
    for mreq in (0, 9):
        with pytest.raises(ValueError):
            O.decode_mline(H, llr, 100, mreq)
        with pytest.raises(ValueError):
            O.fit_mline(llr[0], mreq)
