"""GPU: the learned-proposal kernels against the fp64 reference, and what the
trained network gains over plain ORBGRAND.

Tolerances: features and the batch order are compared bit for bit (same
rounding, same comparison rule).  Logits: BF16 activations are rounded at the
same points on both sides, but FP32 accumulation in a different order can move
an activation across a BF16 rounding boundary, so |gpu - ref| <= 2e-2 (1 + |ref|).
Gradients: the GPU also rounds the backward's GEMM inputs to BF16 (relative
error 2^-9 per value), so each parameter tensor must reach cosine >= 0.999 and
a relative norm error <= 3e-2; the loss matches to 1e-3 relative.
"""
import os

import numpy as np
import pytest
import torch

from oracle import mlp_ref as M
from oracle import oracle as O
from paper_2202_13951_amd import binding, learned
from synth import channel, codes

pytestmark = pytest.mark.gpu
THREADS = min(16, os.cpu_count() or 1)


def _bits_to_f32(t):
    return M.from_bf16_bits(t.cpu().numpy().view(np.uint16))


def _setup(w, dev):
    p = learned.Proposal(dev, w=torch.from_numpy(np.asarray(w, dtype=np.float32)))
    return p


def test_features_bit_exact(gpu_device):
    rng = np.random.default_rng(0)
    llr = (rng.standard_normal((300, 128)) * 5).astype(np.float32)
    llr[0] = np.round(llr[0])                  # ties
    llr[1, :10] = -0.0
    llr[2] = 1e-40                             # subnormal
    x = learned.features(torch.from_numpy(llr).to(gpu_device))
    torch.cuda.synchronize()
    want = M.bf16_bits(np.sort(np.abs(llr), axis=1) * np.float32(0.125))
    assert (x.cpu().numpy().view(np.uint16) == want).all()


@pytest.mark.parametrize("N", [1, 100, 2500])
def test_forward_matches_reference(gpu_device, N):
    w = M.init(3)
    d = M.unflatten(w.astype(np.float64))
    rng = np.random.default_rng(N)
    d["b1"][:] = rng.standard_normal(256) * 0.1
    d["b3"][:] = rng.standard_normal(64) * 0.1
    w = M.flatten(d).astype(np.float32)
    llr = (rng.standard_normal((N, 128)) * 6).astype(np.float32)
    p = _setup(w, gpu_device)
    x = learned.features(torch.from_numpy(llr).to(gpu_device))
    lg = p.logits(x).cpu().numpy()
    ref, _ = M.forward(w, _bits_to_f32(x))
    assert (np.abs(lg - ref) <= 2e-2 * (1 + np.abs(ref))).all()
    # the BF16 copies are the reference rounding of the masters
    assert (p.wb.cpu().numpy().view(np.uint16) == M.bf16_bits(w)).all()
    wt = p.wt.cpu().numpy().view(np.uint16)
    u = M.unflatten(M.bf16_bits(w).astype(np.float64))
    want_t = np.concatenate([u["W1"].T.reshape(-1), u["W2"].T.reshape(-1), u["W3"].T.reshape(-1)]).astype(np.uint16)
    assert (wt == want_t).all()


@pytest.mark.parametrize("N", [7, 1000, 2500])
def test_backward_matches_reference(gpu_device, N):
    w = M.init(5)
    rng = np.random.default_rng(N + 1)
    llr = (rng.standard_normal((N, 128)) * 6).astype(np.float32)
    labels = rng.integers(0, 64, N).astype(np.int32)
    p = _setup(w, gpu_device)
    x = learned.features(torch.from_numpy(llr).to(gpu_device))
    y = torch.from_numpy(labels).to(gpu_device)
    binding.orbg_mlp_backward(p.w, p.wb, p.wt, x, y, p.grads, p.loss, p.workspace(N))
    torch.cuda.synchronize()
    g = p.grads.cpu().numpy().astype(np.float64)
    loss = float(p.loss.item())
    rloss, rg = M.backward(w, _bits_to_f32(x), labels)
    assert abs(loss - rloss) <= 1e-3 * abs(rloss)
    G, R = M.unflatten(g), M.unflatten(rg)
    for name, _ in M.SHAPES:
        a, b = G[name].reshape(-1), R[name].reshape(-1)
        cos = float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-300))
        rel = float(np.linalg.norm(a - b) / (np.linalg.norm(b) + 1e-300))
        assert cos >= 0.999 and rel <= 3e-2, (name, cos, rel)


def test_adam_matches_reference(gpu_device):
    rng = np.random.default_rng(9)
    w = rng.standard_normal(M.NPARAM).astype(np.float32)
    m = (rng.standard_normal(M.NPARAM) * 1e-2).astype(np.float32)
    v = (rng.random(M.NPARAM) * 1e-3).astype(np.float32)
    g = (rng.standard_normal(M.NPARAM) * 1e-2).astype(np.float32)
    p = _setup(w, gpu_device)
    p.m.copy_(torch.from_numpy(m))
    p.v.copy_(torch.from_numpy(v))
    p.grads.copy_(torch.from_numpy(g))
    binding.orbg_mlp_adam(p.w, p.m, p.v, p.grads, 3e-3, 4, p.wb, p.wt)
    torch.cuda.synchronize()
    rw, rm, rv = M.adam(w, m, v, g, 3e-3, 4)
    assert np.allclose(p.m.cpu().numpy(), rm, rtol=1e-5, atol=1e-9)
    assert np.allclose(p.v.cpu().numpy(), rv, rtol=1e-5, atol=1e-12)
    assert np.allclose(p.w.cpu().numpy(), rw, rtol=1e-5, atol=1e-6)
    assert (p.wb.cpu().numpy().view(np.uint16) == M.bf16_bits(p.w.cpu().numpy())).all()


def test_order_bit_exact(gpu_device):
    rng = np.random.default_rng(2)
    lg = rng.standard_normal((500, 64)).astype(np.float32)
    lg[0] = 0.0
    lg[1, ::2] = -0.0
    lg[2, 5] = np.nan
    lg[3] = np.round(lg[3])
    lg[4, :32] = np.inf
    t = torch.from_numpy(lg).to(gpu_device)
    order = torch.empty((500, 64), dtype=torch.uint8, device=gpu_device)
    binding.orbg_mlp_order(t, order)
    torch.cuda.synchronize()
    assert (order.cpu().numpy() == M.order(lg)).all()


def test_trained_proposal_gains_over_plain(gpu_device):
    """Train on pairs the decoder generates (RLC(128,105), Eb/N0 ~ U[3,5] dB), then
    on held-out blocks at 4 dB: mean queries drop (paired 95% interval below 0),
    block errors stay within their 95% interval, and the ordered decode with the
    learned order equals the oracle's ordered decode bit for bit on a sample."""
    print("train proposal", flush=True)
    H, G = codes.code("rlc128_105")
    x, y = learned.generate_pairs(H, G, 600000, 3.0, 5.0, seed=1, device=gpu_device)
    assert x.shape[0] > 300000
    prop = learned.Proposal(gpu_device, seed=0)
    losses = learned.train(prop, x, y, epochs=3, batch=8192, lr=2e-3)
    assert losses[-1] < 0.8 * np.log(64), losses
    print(f"losses {losses}", flush=True)
    llr, sent = channel.awgn_llr_torch(G, 40000, 4.0, seed=777, device=gpu_device)
    budget = 10 ** 5
    pc, pq, pab = binding.orbg_decode(H, llr, budget)
    lc, lq, lab = learned.decode_learned(prop, H, llr, budget)
    torch.cuda.synchronize()
    pq, lq = pq.cpu().numpy().astype(np.float64), lq.cpu().numpy().astype(np.float64)
    mu, (lo, hi) = learned.paired_ci(lq - pq)
    print(f"mean queries plain {pq.mean():.2f} learned {lq.mean():.2f} diff {mu:.2f} [{lo:.2f}, {hi:.2f}]",
          flush=True)
    assert hi < 0
    pe = int((pc != sent).any(dim=1).sum())
    le = int((lc != sent).any(dim=1).sum())
    assert abs(le - pe) <= 1.96 * np.sqrt(pe + le) + 2, (pe, le)
    # bit-exact against the oracle's ordered decode on a sample, with the GPU's order
    order = prop.order(learned.features(llr))
    idx = np.arange(0, 40000, 100)
    oc, oq, oab = O.decode_ordered(H, llr.cpu().numpy()[idx], budget, order.cpu().numpy()[idx], THREADS)
    assert (lc.cpu().numpy()[idx] == oc).all() and (lq[idx].astype(np.uint64) == oq).all()
