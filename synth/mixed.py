"""Seeded mixed-code workloads: blocks of several codes interleaved in one flat
buffer (input generation only).

Block i belongs to code block_code[i]; its n LLRs start at element
row_offset[i] of the flat FP32 buffer (and its codeword at the same offset of
the flat byte buffer).  Codes are mixed in the given ratio and interleaved by
a seeded shuffle.
"""
from __future__ import annotations

import numpy as np

from synth import channel


def plan(ns, ratio, n_blocks: int, seed: int):
    """Block -> code assignment (seeded shuffle of counts in `ratio`) and row offsets."""
    ratio = np.asarray(ratio, dtype=np.float64)
    counts = np.floor(n_blocks * ratio / ratio.sum()).astype(np.int64)
    counts[0] += n_blocks - counts.sum()
    block_code = np.concatenate([np.full(c, i, dtype=np.uint8) for i, c in enumerate(counts)])
    rng = np.random.Generator(np.random.PCG64(seed))
    rng.shuffle(block_code)
    lens = np.asarray(ns, dtype=np.int64)[block_code]
    row_offset = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.int64)
    return block_code, row_offset, int(lens.sum())


def mixed_llr(gens, ratio, n_blocks: int, ebn0_db, seed: int):
    """numpy: gens = generator matrices; ebn0_db: one value or one per block.
    Returns (llr flat f32, sent flat u8, block_code u8, row_offset i64)."""
    ns = [G.shape[1] for G in gens]
    block_code, row_offset, total = plan(ns, ratio, n_blocks, seed)
    llr = np.empty(total, dtype=np.float32)
    sent = np.empty(total, dtype=np.uint8)
    for ci, G in enumerate(gens):
        idx = np.nonzero(block_code == ci)[0]
        if idx.size == 0:
            continue
        x, c = channel.awgn_llr(G, idx.size, float(ebn0_db), seed=seed * 31 + ci)
        n = G.shape[1]
        pos = row_offset[idx][:, None] + np.arange(n)[None, :]
        llr[pos] = x
        sent[pos] = c
    return llr, sent, block_code, row_offset


def mixed_llr_torch(gens, ratio, n_blocks: int, ebn0_db: float, seed: int, device):
    """torch on `device` (same layout as mixed_llr, not the same draws)."""
    import torch
    ns = [G.shape[1] for G in gens]
    block_code, row_offset, total = plan(ns, ratio, n_blocks, seed)
    bc = torch.from_numpy(block_code).to(device)
    ro = torch.from_numpy(row_offset).to(device)
    llr = torch.empty(total, dtype=torch.float32, device=device)
    sent = torch.empty(total, dtype=torch.uint8, device=device)
    for ci, G in enumerate(gens):
        idx = torch.nonzero(bc == ci).flatten()
        if idx.numel() == 0:
            continue
        x, c = channel.awgn_llr_torch(G, idx.numel(), ebn0_db, seed=seed * 31 + ci, device=device)
        n = G.shape[1]
        pos = (ro[idx][:, None] + torch.arange(n, device=device)[None, :]).reshape(-1)
        llr[pos] = x.reshape(-1)
        sent[pos] = c.reshape(-1)
    return llr, sent, bc, ro


def mixed_llr_torch_snr_range(gens, ratio, n_blocks: int, ebn0_lo: float, ebn0_hi: float, seed: int, device):
    """torch on `device`: like mixed_llr_torch, but every block draws its own
    Eb/N0 uniformly in [lo, hi] dB.  Returns (llr, sent, block_code, row_offset, ebn0)."""
    import torch
    ns = [G.shape[1] for G in gens]
    block_code, row_offset, total = plan(ns, ratio, n_blocks, seed)
    bc = torch.from_numpy(block_code).to(device)
    ro = torch.from_numpy(row_offset).to(device)
    llr = torch.empty(total, dtype=torch.float32, device=device)
    sent = torch.empty(total, dtype=torch.uint8, device=device)
    snr = torch.empty(n_blocks, dtype=torch.float32, device=device)
    for ci, G in enumerate(gens):
        idx = torch.nonzero(bc == ci).flatten()
        if idx.numel() == 0:
            continue
        x, c, e = channel.awgn_llr_torch_snr_range(G, idx.numel(), ebn0_lo, ebn0_hi, seed=seed * 31 + ci,
                                                   device=device)
        n = G.shape[1]
        pos = (ro[idx][:, None] + torch.arange(n, device=device)[None, :]).reshape(-1)
        llr[pos] = x.reshape(-1)
        sent[pos] = c.reshape(-1)
        snr[idx] = e
    return llr, sent, bc, ro, snr
