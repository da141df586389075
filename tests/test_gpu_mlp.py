"""GPU: the learned-proposal kernels against the fp64 reference, and what the
trained network gains over plain ORBGRAND.

Tolerances: features and the batch order are compared bit for bit (same
rounding, same comparison rule).  Logits: BF16 activations are rounded at the
same points on both sides, but FP32 accumulation in a different order can move
an activation across a BF16 rounding boundary (one BF16 step, 2^-8 relative),
so each row's logits must agree in the max norm to 1e-2 of the row's largest
|logit| (measured: below 1e-6 for 100 rows, 8e-4 for 2500, 2.6e-3 for 20000).
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
    rowmax = np.abs(ref).max(axis=1, keepdims=True)
    assert (np.abs(lg - ref) <= 1e-2 * rowmax).all(), float((np.abs(lg - ref) / rowmax).max())
    # the BF16 copies are the reference rounding of the masters
    assert (p.wb.cpu().numpy().view(np.uint16) == M.bf16_bits(w)).all()
    wt = p.wt.cpu().numpy().view(np.uint16)
    u = M.unflatten(M.bf16_bits(w).astype(np.float64))
    want_t = np.concatenate([u["W1"].T.reshape(-1), u["W2"].T.reshape(-1), u["W3"].T.reshape(-1)]).astype(np.uint16)
    assert (wt == want_t).all()


@pytest.mark.parametrize("N", [1, 31, 1000])
def test_fused_inference_equals_unfused(gpu_device, N):
    """orbg_mlp_infer (features, three layers with on-chip activations, order in
    one launch) against the unfused kernels, bit for bit: logits from given
    features, from llr rows, and from an id list with ids outside the llr rows
    (zero features); orders against orbg_mlp_order, with batch 0 pinned first."""
    print(f"fused inference N={N}", flush=True)
    w = M.init(7)
    d = M.unflatten(w.astype(np.float64))
    rng = np.random.default_rng(100 + N)
    for b in ("b1", "b2", "b3"):
        d[b][:] = rng.standard_normal(d[b].shape) * 0.1
    w = M.flatten(d).astype(np.float32)
    p = _setup(w, gpu_device)
    llr = torch.from_numpy((rng.standard_normal((N, 128)) * 6).astype(np.float32)).to(gpu_device)
    x = learned.features(llr)
    ref = p.logits(x)
    lg = torch.empty((N, 64), dtype=torch.float32, device=gpu_device)
    binding.orbg_mlp_infer(p.w, p.wb, x=x, logits=lg)
    torch.cuda.synchronize()
    assert torch.equal(lg, ref)
    lg2 = torch.empty_like(lg)
    od2 = torch.empty((N, 64), dtype=torch.uint8, device=gpu_device)
    binding.orbg_mlp_infer(p.w, p.wb, llr=llr, logits=lg2, order=od2)
    want_od = torch.empty_like(od2)
    binding.orbg_mlp_order(ref, want_od)
    torch.cuda.synchronize()
    assert torch.equal(lg2, ref) and torch.equal(od2, want_od)
    # an id list: a permutation of the rows with two ids past the array
    ids_np = rng.permutation(N).astype(np.int64)
    ids_np = np.concatenate([ids_np, [-1, N + 5]])
    ids = torch.from_numpy(ids_np).to(gpu_device)
    lg3 = torch.empty((ids.numel(), 64), dtype=torch.float32, device=gpu_device)
    od3 = torch.empty((ids.numel(), 64), dtype=torch.uint8, device=gpu_device)
    binding.orbg_mlp_infer(p.w, p.wb, llr=llr, ids=ids, logits=lg3, order=od3, pin0=True)
    zero = p.logits(torch.zeros((1, 128), dtype=torch.int16, device=gpu_device))
    want3 = torch.cat([ref[ids[:N]], zero, zero])
    pinned = want3.clone()
    pinned[:, 0] = float("inf")
    want_od3 = torch.empty_like(od3)
    binding.orbg_mlp_order(pinned, want_od3)
    torch.cuda.synchronize()
    assert torch.equal(lg3, want3) and torch.equal(od3, want_od3)
    assert (od3[:, 0] == 0).all()


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


def test_trained_proposal_gains_over_plain_and_prior(gpu_device):
    """Train on the pairs the gated decode asks about (RLC(128,105), Eb/N0 ~
    U[3,5] dB, blocks whose first hit lies in batches 1..63); the final training
    loss ends below the entropy of the labels (what predicting the label
    frequencies alone gives).  On held-out blocks at 4 dB the gated decode needs
    fewer queries than plain ORBGRAND and than the fixed prior order (batch 0,
    then batches by training-label frequency), both paired 95% intervals below
    0, and its block errors stay within their 95% interval of plain's."""
    print("train proposal", flush=True)
    H, G = codes.code("rlc128_105")
    x, y = learned.generate_pairs(H, G, 3000000, 3.0, 5.0, seed=1, device=gpu_device, gated=True)
    assert x.shape[0] > 600000 and int(y.min()) >= 1
    hist = torch.bincount(y.long(), minlength=64).cpu().numpy().astype(np.float64)
    p = hist[hist > 0] / hist.sum()
    entropy = float(-(p * np.log(p)).sum())
    prop = learned.Proposal(gpu_device, seed=0)
    losses = learned.train(prop, x, y, epochs=4, batch=8192, lr=2e-3)
    print(f"losses {losses}, label entropy {entropy:.4f}", flush=True)
    assert losses[-1] < entropy, (losses, entropy)
    prior = learned.prior_order(y, gpu_device)
    llr, sent = channel.awgn_llr_torch(G, 200000, 4.0, seed=777, device=gpu_device)
    budget = 10 ** 5
    pc, pq, pab = binding.orbg_decode(H, llr, budget)
    lc, lq, lab, rest = learned.decode_learned_gated(prop, H, llr, budget)
    rc, rq, rab = binding.orbg_decode_ordered(H, llr, budget, prior.unsqueeze(0).expand(llr.shape[0], 64).contiguous())
    torch.cuda.synchronize()
    pqn, lqn, rqn = (t.cpu().numpy().astype(np.float64) for t in (pq, lq, rq))
    mu, (lo, hi) = learned.paired_ci(lqn - pqn)
    mur, (lor, hir) = learned.paired_ci(lqn - rqn)
    print(f"network ran on {rest} blocks; mean queries plain {pqn.mean():.2f} learned {lqn.mean():.2f} "
          f"prior {rqn.mean():.2f}; learned - plain {mu:.2f} [{lo:.2f}, {hi:.2f}], "
          f"learned - prior {mur:.2f} [{lor:.2f}, {hir:.2f}]", flush=True)
    assert hi < 0 and hir < 0
    pe = int((pc != sent).any(dim=1).sum())
    le = int((lc != sent).any(dim=1).sum())
    assert abs(le - pe) <= 1.96 * np.sqrt(pe + le) + 2, (pe, le)


def _listed_case(dev, N=6000, ebn0=3.5, seed=4242):
    H, G = codes.code("rlc128_105")
    llr, sent = channel.awgn_llr_torch(G, N, ebn0, seed=seed, device=dev)
    return H, G, llr, sent


@pytest.mark.parametrize("budget", [64, 3000, 10 ** 5])
def test_gated_decode_matches_oracle(gpu_device, budget):
    """The gated decode (batch 0 for every block, the network and the ordered
    search for the rest) against the oracle's ordered decode with the order each
    block was given: every block's codeword, queries and flag, bit for bit; the
    blocks the network ran on are exactly those plain ORBGRAND does not decide in
    its first 64 queries, their orders start with batch 0 and rank the others by
    the network's logits; every other block keeps the identity order."""
    print(f"gated decode, budget {budget}", flush=True)
    H, G, llr, sent = _listed_case(gpu_device)
    N = llr.shape[0]
    prop = learned.Proposal(gpu_device, seed=3)          # an untrained network gives some order
    order = torch.empty((N, 64), dtype=torch.uint8, device=gpu_device)
    cw, q, ab, rest = learned.decode_learned_gated(prop, H, llr, budget, order_out=order)
    pc, pq, pab = binding.orbg_decode(H, llr, budget)
    torch.cuda.synchronize()
    llr_np, order_np = llr.cpu().numpy(), order.cpu().numpy()
    pqn = pq.cpu().numpy()
    listed = pqn > 64
    assert rest == int(listed.sum())
    assert rest > (0 if budget > 64 else -1)
    ident = np.arange(64, dtype=np.uint8)
    assert (order_np[~listed] == ident).all()
    oc, oq, oab = O.decode_ordered(H, llr_np, budget, order_np, THREADS)
    assert (cw.cpu().numpy() == oc).all()
    assert (q.cpu().numpy().astype(np.uint64) == oq).all()
    assert (ab.cpu().numpy() == oab).all()
    if rest:
        idx = np.nonzero(listed)[0]
        rows = torch.from_numpy(idx).to(gpu_device)
        x = learned.features(llr[rows].contiguous())
        lg = prop.logits(x).cpu().numpy()
        want = M.order(np.concatenate([np.full((len(idx), 1), np.inf), lg[:, 1:]], axis=1))
        assert (order_np[idx] == want).all()
