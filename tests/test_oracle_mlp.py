"""Pins of the learned-proposal reference (oracle/mlp_ref.py): BF16 rounding by
hand-checked bit patterns, closed forms of the network at special weights,
finite differences of the loss, the first Adam step, the order rule."""
import numpy as np
import pytest

from oracle import mlp_ref as M


def test_parameter_count():
    assert M.NPARAM == 256 * 128 + 256 + 256 * 256 + 256 + 64 * 256 + 64 == 115264


@pytest.mark.parametrize("value,bits", [
    (1.0, 0x3F80), (-2.0, 0xC000), (0.0, 0x0000), (-0.0, 0x8000),
    (1.0 + 2.0 ** -8, 0x3F80),                 # exactly half way, even neighbour is 1.0
    (1.0 + 3 * 2.0 ** -8, 0x3F82),             # half way above 1.0078125 -> even 1.015625
    (1.0 + 2.0 ** -8 + 2.0 ** -20, 0x3F81),    # just above half way rounds up
    (3.0e38, 0x7F62), (np.inf, 0x7F80), (-np.inf, 0xFF80), (0.1, 0x3DCD)])
def test_bf16_round_known_patterns(value, bits):
    assert int(M.bf16_bits(np.float32(value))) == bits


def test_bf16_nan_stays_nan():
    assert np.isnan(M.bf16_round(np.float32(np.nan)))


def test_features_sorted_scaled():
    llr = np.array([[-3.0, 0.5, -0.25, 8.0] + [1.0] * 124], dtype=np.float32)
    f = M.features(llr)
    assert f[0, 0] == np.float32(0.25 / 8) and f[0, -1] == np.float32(1.0)
    assert (np.diff(f[0]) >= 0).all()


def test_zero_network_closed_forms():
    """All weights zero: logits = b3; with b3 = 0 the loss is log 64 and the bias
    gradient is softmax - onehot averaged: 1/64 - [label]/N."""
    p = np.zeros(M.NPARAM)
    x = np.random.default_rng(0).standard_normal((5, 128))
    labels = np.array([0, 3, 3, 63, 10])
    loss, g = M.backward(p, x, labels)
    assert abs(loss - np.log(64)) < 1e-12
    gb3 = M.unflatten(g)["b3"]
    want = np.full(64, 1 / 64)
    for lab in labels:
        want[lab] -= 1 / len(labels)
    assert np.allclose(gb3, want, atol=1e-15)
    d = M.unflatten(p.copy())
    d["b3"][:] = np.arange(64)
    logits, _ = M.forward(M.flatten(d), x)
    assert np.allclose(logits, np.arange(64)[None, :])


def test_single_path_by_hand():
    """One active path: h1_0 = relu(2 x_0 + 1), h2_0 = relu(-3 h1_0 + 0.5), logit_5 = 4 h2_0 - 1."""
    d = M.unflatten(np.zeros(M.NPARAM))
    d["W1"][0, 0], d["b1"][0] = 2.0, 1.0
    d["W2"][0, 0], d["b2"][0] = -3.0, 0.5
    d["W3"][5, 0], d["b3"][5] = 4.0, -1.0
    x = np.zeros((2, 128))
    x[0, 0], x[1, 0] = -0.25, -1.0
    logits, c = M.forward(M.flatten(d), x)
    assert logits[0, 5] == 4 * max(-3 * max(2 * -0.25 + 1, 0) + 0.5, 0) - 1     # h1 = 0.5 -> h2 = 0 -> -1
    assert logits[1, 5] == 4 * max(-3 * max(2 * -1.0 + 1, 0) + 0.5, 0) - 1      # h1 = 0 -> h2 = 0.5 -> 1
    assert logits[1, 5] == 1.0 and logits[0, 5] == -1.0


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(3)
    p = M.init(7).astype(np.float64) * 0.5
    d = M.unflatten(p)
    d["b1"][:] = rng.standard_normal(256) * 0.1
    d["b2"][:] = rng.standard_normal(256) * 0.1
    d["b3"][:] = rng.standard_normal(64) * 0.1
    p = M.flatten(d)
    # exact-arithmetic network (no BF16 rounding), so finite differences apply
    pw = p.copy()
    for name in ("W1", "W2", "W3"):
        M.unflatten(pw)[name][...] = M.bf16_round(M.unflatten(pw)[name])
    x = M.bf16_round(rng.standard_normal((6, 128))).astype(np.float64)
    labels = rng.integers(0, 64, 6)
    _, g = M.backward(pw, x, labels, round_activations=False)
    # perturb only biases (weights are rounded to BF16 inside the forward)
    offs = {}
    o = 0
    for name, shape in M.SHAPES:
        offs[name] = o
        o += int(np.prod(shape))
    idx = [offs["b3"] + i for i in (0, 7, 63)] + [offs["b2"] + i for i in (1, 100)] + \
          [offs["b1"] + i for i in (2, 200)]
    eps = 1e-6
    for i in idx:
        pp, pm = pw.copy(), pw.copy()
        pp[i] += eps
        pm[i] -= eps
        lp, _ = M.loss_and_dlogits(M.forward(pp, x, False)[0], labels)
        lm, _ = M.loss_and_dlogits(M.forward(pm, x, False)[0], labels)
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - g[i]) < 1e-7 + 1e-5 * abs(fd), (i, fd, g[i])


def test_weight_gradient_matches_finite_differences():
    """Weight gradients through a network whose weights are already BF16 values
    and perturbations that keep them BF16 values (steps of one BF16 ulp are too
    coarse for differences, so check linearity in the last layer instead)."""
    rng = np.random.default_rng(4)
    p = M.init(9).astype(np.float64)
    x = M.bf16_round(rng.standard_normal((4, 128))).astype(np.float64)
    labels = rng.integers(0, 64, 4)
    loss, g = M.backward(p, x, labels, round_activations=False)
    logits, c = M.forward(p, x, False)
    _, dl = M.loss_and_dlogits(logits, labels)
    gW3 = M.unflatten(g)["W3"]
    assert np.allclose(gW3, dl.T @ c["h2"])
    # the first-layer gradient equals the chain rule written with explicit loops on one entry
    W = c["W"]
    j, i = 17, 33
    dz2 = (dl @ W["W3"]) * (c["z2"] > 0)
    dz1 = (dz2 @ W["W2"]) * (c["z1"] > 0)
    assert abs(M.unflatten(g)["W1"][j, i] - sum(dz1[b, j] * x[b, i] for b in range(4))) < 1e-12


def test_adam_first_step_is_lr_times_sign():
    g = np.array([0.5, -2.0, 1e-3, -7.0])
    w, m, v = M.adam(np.zeros(4), np.zeros(4), np.zeros(4), g, lr=0.01, step=1)
    assert np.allclose(w, -0.01 * np.sign(g) * np.abs(g) / (np.abs(g) + 1e-8))
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_order_descending_ties_low_index():
    logits = np.array([[0.0] * 64])
    logits[0, 5] = 2.0
    logits[0, 9] = 2.0
    logits[0, 1] = -1.0
    o = M.order(logits)[0]
    assert list(o[:2]) == [5, 9] and o[-1] == 1 and sorted(o) == list(range(64))
    assert list(o[2:8]) == [0, 2, 3, 4, 6, 7]


def _offsets():
    offs, o = {}, 0
    for name, shape in M.SHAPES:
        offs[name] = o
        o += int(np.prod(shape))
    return offs


def test_weight_gradients_match_central_differences():
    """Every weight matrix's gradient against fp64 central differences of the
    loss, in the exact-arithmetic form of the network (weights and activations
    not rounded), at entries of W1, W2 (an off-diagonal pair (i, j) / (j, i)
    whose two gradients differ, so a transposed gradient fails) and W3."""
    rng = np.random.default_rng(11)
    d = M.unflatten(M.init(13).astype(np.float64) * 0.5)
    for name in ("b1", "b2", "b3"):
        d[name][:] = rng.standard_normal(d[name].shape) * 0.1
    p = M.flatten(d)
    x = M.bf16_round(rng.standard_normal((8, 128))).astype(np.float64)
    labels = rng.integers(0, 64, 8)
    _, g = M.backward(p, x, labels, round_activations=False, round_weights=False)
    offs = _offsets()
    entries = [("W1", (5, 17)), ("W1", (200, 127)), ("W1", (17, 5)),
               ("W2", (3, 40)), ("W2", (40, 3)), ("W2", (255, 0)), ("W2", (128, 128)),
               ("W3", (0, 255)), ("W3", (63, 7)), ("W3", (7, 63))]
    eps = 1e-6
    fd = {}
    for name, (r, c) in entries:
        cols = dict(M.SHAPES)[name][1]
        i = offs[name] + r * cols + c
        pp, pm = p.copy(), p.copy()
        pp[i] += eps
        pm[i] -= eps
        lp, _ = M.loss_and_dlogits(M.forward(pp, x, False, False)[0], labels)
        lm, _ = M.loss_and_dlogits(M.forward(pm, x, False, False)[0], labels)
        fd[(name, r, c)] = (lp - lm) / (2 * eps)
        assert abs(fd[(name, r, c)] - g[i]) < 1e-8 + 1e-5 * abs(fd[(name, r, c)]), (name, r, c, fd[(name, r, c)], g[i])
    # the pair (3, 40) / (40, 3) of W2 tells a transposed gradient apart
    a, b = fd[("W2", 3, 40)], fd[("W2", 40, 3)]
    assert abs(a - b) > 1e-3 * max(abs(a), abs(b)) and max(abs(a), abs(b)) > 1e-6
    gw = M.unflatten(g)
    assert abs(gw["W2"].T[3, 40] - a) > 1e-7 + 1e-5 * abs(a)


def test_planted_gradient_mistakes_fail_the_difference_check():
    """The central-difference check above rejects a transposed W2 gradient and a
    W1 gradient formed with the hidden activations in place of the inputs: both
    mistakes planted in a copy of the reference's backward."""
    rng = np.random.default_rng(12)
    d = M.unflatten(M.init(14).astype(np.float64) * 0.5)
    p = M.flatten(d)
    x = M.bf16_round(rng.standard_normal((6, 128))).astype(np.float64)
    labels = rng.integers(0, 64, 6)
    logits, c = M.forward(p, x, False, False)
    _, dl = M.loss_and_dlogits(logits, labels)
    W = c["W"]
    dz2 = (dl @ W["W3"]) * (c["z2"] > 0)
    dz1 = (dz2 @ W["W2"]) * (c["z1"] > 0)
    wrong_W2 = (dz2.T @ c["h1"]).T
    wrong_W1 = dz1.T @ c["h1"][:, :128]
    offs = _offsets()
    eps = 1e-6

    def fd(name, r, cc):
        i = offs[name] + r * dict(M.SHAPES)[name][1] + cc
        pp, pm = p.copy(), p.copy()
        pp[i] += eps
        pm[i] -= eps
        lp, _ = M.loss_and_dlogits(M.forward(pp, x, False, False)[0], labels)
        lm, _ = M.loss_and_dlogits(M.forward(pm, x, False, False)[0], labels)
        return (lp - lm) / (2 * eps)

    bad_w2 = [abs(fd("W2", r, cc) - wrong_W2[r, cc]) > 1e-8 + 1e-5 * abs(wrong_W2[r, cc])
              for r, cc in ((3, 40), (40, 3), (100, 9))]
    bad_w1 = [abs(fd("W1", r, cc) - wrong_W1[r, cc]) > 1e-8 + 1e-5 * abs(wrong_W1[r, cc])
              for r, cc in ((5, 17), (17, 5), (200, 127))]
    assert any(bad_w2) and any(bad_w1)
