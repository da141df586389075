"""Pins of the oracle's query order (Sec. III-B/C) against things other than itself:
the paper's worked partition example, its first queries, brute-force enumeration
of distinct-part sets, and closed-form counts."""
import itertools
import os

import numpy as np
import pytest

from oracle import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_fixture(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line)
    return rows


def test_landslide_worked_example():
    rows = _read_fixture("landslide_worked_example.txt")
    kv = {r.split()[0]: r.split()[1:] for r in rows}
    Wp, w, np_ = (int(x.split("=")[1]) for x in kv["setting"])
    parts = O.landslide(Wp, w, np_)
    assert len(parts) == int(kv["count"][0])
    assert parts[0] == tuple(int(x) for x in kv["a"])
    assert parts[4] == tuple(int(x) for x in kv["e"])        # (e) is the fifth diagram
    assert parts[7] == tuple(int(x) for x in kv["h"])
    assert parts[3][0] == 0 and parts[4][0] == 1              # (d) u_1 = 0, (e) u_1 = 1
    # (h): accumulated drop D(1) = u_w - u_1 <= 1; every earlier one has D(1) >= 2
    assert parts[7][-1] - parts[7][0] <= 1
    assert all(p[-1] - p[0] >= 2 for p in parts[:7])
    # Landslide figure: W = 18, w = 4, n = 8 -> v = u + (1, 2, 3, 4)
    off = [int(x) for x in kv["distinct"][4:]]
    vs = [tuple(u + o for u, o in zip(p, off)) for p in parts]
    brute = [c for c in itertools.combinations(range(1, 9), 4) if sum(c) == 18]
    assert sorted(vs) == brute


def test_first_queries_golden():
    rows = _read_fixture("first_queries.txt")
    pats = O.order_prefix(10, 5)
    assert pats[0] == ()
    assert pats[1] == tuple(int(x) for x in rows[1].split()[1:])
    assert pats[2] == tuple(int(x) for x in rows[2].split()[1:])
    left, right = rows[3].split(None, 1)[1].split("|")
    tie = {tuple(int(x) for x in left.split()), tuple(int(x) for x in right.split())}
    assert set(pats[3:5]) == tie
    # reading R3 (Hamming weight ascending inside a logistic weight) picks {3} first
    assert pats[3] == (3,) and pats[4] == (1, 2)


@pytest.mark.parametrize("np_", range(0, 7))
@pytest.mark.parametrize("w", range(1, 6))
def test_landslide_is_lex_order_of_bounded_partitions(w, np_):
    """Every (W', w, n') with small sizes: Landslide emits each non-decreasing
    partition exactly once, in lexicographically ascending order."""
    for Wp in range(0, w * np_ + 1):
        brute = sorted(p for p in itertools.combinations_with_replacement(range(np_ + 1), w)
                       if sum(p) == Wp)
        assert O.landslide(Wp, w, np_) == brute, (Wp, w, np_)
    assert O.landslide(w * np_ + 1, w, np_) == []


def _brute_order(n):
    subs = [c for w in range(n + 1) for c in itertools.combinations(range(1, n + 1), w)]
    subs.sort(key=lambda c: (sum(c), len(c), c))
    return subs


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 11, 13, 16])
def test_whole_order_exhaustive(n):
    """The order visits all 2^n subsets once, by (logistic weight, Hamming weight,
    lexicographic ranks) -- the reading of eq. (fractionation) and Algorithm 2."""
    got = O.order_prefix(n, 2 ** n + 3)
    assert len(got) == 2 ** n
    assert got == _brute_order(n)


def _distinct_part_counts(n, Wmax):
    # coefficients of prod_{i=1}^{n} (1 + x^i), truncated at Wmax
    c = np.zeros(Wmax + 1, dtype=object)
    c[0] = 1
    for i in range(1, n + 1):
        c[i:] = c[i:] + c[:-i].copy() if i <= Wmax else c[i:]
    return c


@pytest.mark.parametrize("n", [20, 32, 64])
def test_weight_class_sizes_match_generating_function(n):
    count = 20000
    pats = O.order_prefix(n, count)
    W = [sum(p) for p in pats]
    assert all(a <= b for a, b in zip(W, W[1:]))                 # non-decreasing w_L
    full = max(W) - 1                                            # last complete class
    gf = _distinct_part_counts(n, full)
    hist = np.bincount(np.array(W), minlength=full + 2)
    assert [int(x) for x in hist[:full + 1]] == [int(x) for x in gf]
    for p in pats:                                               # eq. (fractionation) bound
        Wl = sum(p)
        assert len(p) <= int((np.sqrt(1 + 8 * Wl) - 1) // 2) if Wl else len(p) == 0
        assert all(1 <= r <= n for r in p)


def test_known_partition_counts():
    # distinct-part partition numbers q(W) for W = 0..20 (no cap: n >= W)
    known = [1, 1, 1, 2, 2, 3, 4, 5, 6, 8, 10, 12, 15, 18, 22, 27, 32, 38, 46, 54, 64]
    pats = O.order_prefix(40, 2000)
    hist = np.bincount([sum(p) for p in pats])
    assert list(hist[:21]) == known


def test_max_logistic_weight():
    n = 7
    pats = O.order_prefix(n, 2 ** n)
    assert sum(pats[-1]) == n * (n + 1) // 2 and pats[-1] == tuple(range(1, n + 1))


def test_golden_prefix_twenty():
    want = [(), (1,), (2,), (3,), (1, 2), (4,), (1, 3), (5,), (1, 4), (2, 3), (6,), (1, 5),
            (2, 4), (1, 2, 3), (7,), (1, 6), (2, 5), (3, 4), (1, 2, 4), (8,)]
    assert O.order_prefix(64, 20) == want
