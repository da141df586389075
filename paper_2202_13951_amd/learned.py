"""Learned batch-order proposal: training pairs from the decoder itself,
training and inference through the library's kernels, ordered decoding.

Pairs: blocks are decoded by plain ORBGRAND with a budget of 4096 queries; a
block whose first hit lies in the first 4096 patterns gives the pair (sorted
|LLR| features, label = index of the 64-pattern batch holding the hit).
Blocks without a hit there are left out: every order of the first 64 batches
treats them alike.  Training minimises softmax cross-entropy with Adam.  At
decode time the batches are tested by decreasing logit, then the plain order
continues (orbg_decode_ordered); each decision is a parity-checked codeword.

Everything numeric runs in liborbgrand; this module sequences calls and holds
the device tensors.
"""
from __future__ import annotations

import math

import numpy as np

from . import binding as B

PREFIX = 4096


class Proposal:
    """Parameters, optimizer state and work spaces of one network on one device."""

    def __init__(self, device, seed: int = 0, w=None):
        import torch
        self.device = device
        if w is None:
            gen = torch.Generator(device="cpu")
            gen.manual_seed(seed)
            parts = []
            for rows, cols in ((256, 128), (256, 0), (256, 256), (256, 0), (64, 256), (64, 0)):
                if cols:        # He-uniform weights
                    lim = math.sqrt(6.0 / cols)
                    parts.append((torch.rand(rows * cols, generator=gen, dtype=torch.float64) * 2 - 1) * lim)
                else:           # zero biases
                    parts.append(torch.zeros(rows, dtype=torch.float64))
            w = torch.cat(parts).to(torch.float32)
        self.w = torch.as_tensor(w, dtype=torch.float32).to(device).contiguous()
        assert self.w.numel() == B.MLP_PARAMS
        self.m = torch.zeros_like(self.w)
        self.v = torch.zeros_like(self.w)
        self.wb = torch.empty(B.MLP_PARAMS, dtype=torch.int16, device=device)
        self.wt = torch.empty(B.MLP_TPARAMS, dtype=torch.int16, device=device)
        self.grads = torch.zeros_like(self.w)
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)
        self.step = 0
        self._ws = {}
        B.orbg_mlp_prepare(self.w, self.wb, self.wt)

    def workspace(self, batch: int):
        import torch
        need = B.orbg_mlp_workspace_bytes(batch)
        ws = self._ws.get("buf")
        if ws is None or ws.numel() < need:
            ws = torch.empty(need, dtype=torch.uint8, device=self.device)
            self._ws["buf"] = ws
        return ws

    def logits(self, x):
        import torch
        out = torch.empty((x.shape[0], 64), dtype=torch.float32, device=self.device)
        step = 1 << 18
        for s in range(0, x.shape[0], step):
            e = min(x.shape[0], s + step)
            B.orbg_mlp_forward(self.w, self.wb, x[s:e], out[s:e], self.workspace(e - s))
        return out

    def order(self, x):
        import torch
        lg = self.logits(x)
        order = torch.empty((x.shape[0], 64), dtype=torch.uint8, device=self.device)
        B.orbg_mlp_order(lg, order)
        return order

    def train_step(self, x, labels, lr: float):
        B.orbg_mlp_backward(self.w, self.wb, self.wt, x, labels, self.grads, self.loss, self.workspace(x.shape[0]))
        self.step += 1
        B.orbg_mlp_adam(self.w, self.m, self.v, self.grads, lr, self.step, self.wb, self.wt)
        return self.loss


def features(llr):
    import torch
    x = torch.empty(llr.shape, dtype=torch.int16, device=llr.device)
    B.orbg_mlp_features(llr, x)
    return x


def generate_pairs(H, G, n_blocks: int, ebn0_lo: float, ebn0_hi: float, seed: int, device, gated: bool = False):
    """Decodes n_blocks fresh blocks (Eb/N0 uniform per block) with a 4096-query
    budget; returns (features int16 [M,128], labels int32 [M]) of the M blocks
    whose first hit falls in the first 4096 patterns (gated: only those whose
    first hit lies past batch 0, the blocks the gated decode asks the network
    about)."""
    import torch
    from synth import channel
    xs, ys = [], []
    chunk = 1 << 20
    for i, s in enumerate(range(0, n_blocks, chunk)):
        e = min(n_blocks, s + chunk)
        llr, _, _ = channel.awgn_llr_torch_snr_range(G, e - s, ebn0_lo, ebn0_hi, seed * 1000 + i, device)
        _, q, ab = B.orbg_decode(H, llr, PREFIX)
        keep = (ab == 0) & (q > 64) if gated else ab == 0
        x = features(llr)
        xs.append(x[keep])
        ys.append(((q[keep] - 1) // 64).to(torch.int32))
        del llr
    return torch.cat(xs), torch.cat(ys)


def train(prop: Proposal, x, y, epochs: int = 1, batch: int = 8192, lr: float = 1e-3, seed: int = 0, log=None):
    """Minibatch Adam over shuffled pairs; returns the mean loss of each epoch."""
    import torch
    gen = torch.Generator(device=prop.device)
    gen.manual_seed(seed)
    N = x.shape[0]
    losses = []
    for ep in range(epochs):
        perm = torch.randperm(N, generator=gen, device=prop.device)
        tot = torch.zeros(1, dtype=torch.float32, device=prop.device)
        nb = 0
        for s in range(0, N - batch + 1, batch):
            idx = perm[s:s + batch]
            tot += prop.train_step(x[idx].contiguous(), y[idx].contiguous(), lr)
            nb += 1
        losses.append(float(tot.item()) / max(nb, 1))
        if log:
            log(f"epoch {ep}: loss {losses[-1]:.4f}")
    return losses


def decode_learned(prop: Proposal, H, llr, budget: int, out=None, params=None):
    """Ordered decode of llr with the network's batch order (features, forward,
    order, decode: four launches on the current stream)."""
    order = prop.order(features(llr))
    return B.orbg_decode_ex(H, llr, budget, order=order, params=params, out=out)


def decode_learned_gated(prop: Proposal, H, llr, budget: int, out=None, order_out=None, params=None):
    """Gated decode (one library call): the first batch of the plain order for
    every block; the network and the ordered search (batch 0 first, batches 1..63
    by the network) only for the blocks it does not decide.  Returns (codeword,
    queries, abandoned, number of blocks the network ran on)."""
    import torch
    need = B.orbg_learned_workspace_bytes(llr.shape[0])
    ws = prop._ws.get("learned")
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=prop.device)
        prop._ws["learned"] = ws
    return B.orbg_decode_learned(H, llr, budget, prop.w, prop.wb, ws, out=out, order_out=order_out, params=params)


def prior_order(labels, device):
    """The fixed order a network without inputs would give: batch 0 first, then
    batches 1..63 by decreasing frequency among the training labels (ties to the
    lower index).  [64] uint8."""
    import torch
    counts = torch.bincount(labels.long(), minlength=64)[:64].cpu().numpy().astype(np.int64)
    rest = sorted(range(1, 64), key=lambda b: (-counts[b], b))
    return torch.tensor([0] + rest, dtype=torch.uint8, device=device)


def paired_ci(diff: np.ndarray, z: float = 1.96):
    """Mean and 95% normal interval of paired differences."""
    d = np.asarray(diff, dtype=np.float64)
    mu = d.mean()
    se = d.std(ddof=1) / math.sqrt(len(d)) if len(d) > 1 else float("inf")
    return mu, (mu - z * se, mu + z * se)
