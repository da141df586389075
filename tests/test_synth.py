"""Checks of the seeded input generators (codes and channel)."""
import itertools
import math

import numpy as np

from synth import channel, codes


def _Q(x):
    return 0.5 * math.erfc(x / math.sqrt(2.0))


def test_bch127_113_structure():
    H = codes.bch_H(127, 113)
    assert H.shape == (14, 127)
    assert codes.gf2_rank(H) == 14
    cols = [int("".join(map(str, H[:, i][::-1])), 2) for i in range(127)]
    assert len(set(cols)) == 127 and 0 not in cols
    # t = 2 => minimum distance >= 5: no 1..4 columns XOR to zero.  Pairs are
    # covered by distinctness; triples and quadruples by a set lookup.
    s = set(cols)
    for a, b in itertools.combinations(cols, 2):
        assert (a ^ b) not in s or (a ^ b) in (a, b)
    pair = {}
    for i, j in itertools.combinations(range(127), 2):
        x = cols[i] ^ cols[j]
        if x in pair:
            i2, j2 = pair[x]
            assert len({i, j, i2, j2}) < 4, "four columns sum to zero"
        pair[x] = (i, j)
    # alpha^7 = alpha^3 + 1 on x^7 + x^3 + 1
    pw = codes.gf2m_powers(7, 0b10001001)
    assert pw[7] == 0b0001001 and len(set(pw.tolist())) == 127


def test_generator_bases_span_kernel():
    for name in ["rlc32_26", "bch127_113", "rlc64_52", "rlc128_116", "rlc256_240", "rlc256_234", "rlc128_105"]:
        H, G = codes.code(name)
        n = H.shape[1]
        assert G.shape == (n - H.shape[0], n)
        assert not ((H.astype(np.int64) @ G.T.astype(np.int64)) % 2).any()
        assert codes.gf2_rank(G) == G.shape[0]


def test_channel_hard_decision_ber_matches_q_function():
    H, G = codes.code("rlc64_52")
    for ebn0 in (3.0, 5.0):
        llr, c = channel.awgn_llr(G, 20000, ebn0, seed=5)
        ber = float(((llr > 0).astype(np.uint8) != c).mean())
        R = 52 / 64
        want = _Q(math.sqrt(2 * R * 10 ** (ebn0 / 10)))
        sd = math.sqrt(want * (1 - want) / llr.size)
        assert abs(ber - want) < 6 * sd, (ebn0, ber, want)
        # LLR = 2Y / sigma^2: the mean LLR of a sent 1 is 2 / sigma^2
        s2 = channel.sigma2(ebn0, R)
        assert abs(llr[c == 1].mean() - 2 / s2) < 0.02 * (2 / s2)


def test_paper_snr_calibration():
    """The paper quotes 9.8 dB (SNR = 1/sigma^2) for an uncoded flip probability
    of 1e-3 (Sec. IV-A): Q(sqrt(10^0.98)) is 1e-3 to two digits."""
    p = _Q(math.sqrt(10 ** 0.98))
    assert abs(p - 1e-3) < 0.05e-3


def test_poisson_arrivals_rate_and_gaps():
    """Exponential gaps: mean 1/rate, coefficient of variation 1, P(gap > 1/rate) = 1/e."""
    from synth import stream
    t = stream.poisson_arrivals(200000, 1e5, seed=3)
    assert t[0] == 0.0 and (np.diff(t) >= 0).all()
    g = np.diff(t)
    assert abs(g.mean() * 1e5 - 1) < 0.01
    assert abs(g.std() / g.mean() - 1) < 0.01
    assert abs((g > 1e-5).mean() - np.exp(-1)) < 0.005
    assert (stream.poisson_arrivals(1000, 1e6, seed=3) == stream.poisson_arrivals(1000, 1e6, seed=3)).all()


def test_mixed_snr_range_layout():
    """Per-block Eb/N0 in range, rows at their offsets are codewords' noisy images of the right length."""
    import torch
    from synth import codes, mixed
    gens = [codes.code(nm)[1] for nm in ("rlc64_52", "bch127_113")]
    llr, sent, bc, ro, snr = mixed.mixed_llr_torch_snr_range(gens, [1, 1], 400, 3.0, 6.0, seed=9, device="cpu")
    assert llr.shape == sent.shape and bc.shape == (400,) and snr.shape == (400,)
    assert float(snr.min()) >= 3.0 and float(snr.max()) <= 6.0
    ns = np.array([64, 127])[bc.numpy()]
    assert (np.diff(ro.numpy()) == ns[:-1]).all() and int(ro[-1]) + ns[-1] == llr.numel()
    for i in range(0, 400, 37):
        H, _ = codes.code(("rlc64_52", "bch127_113")[int(bc[i])])
        c = sent[int(ro[i]):int(ro[i]) + ns[i]].numpy().astype(np.int64)
        assert not ((H.astype(np.int64) @ c) % 2).any()
