"""Seeded BPSK / AWGN channel: random codewords in, FP32 LLRs out.

Input generation only (no decoder arithmetic).  Follows the channel of the
paper's Sec. III-A: a codeword bit c is sent as 2c - 1, received as
Y = 2c - 1 + N with N ~ N(0, sigma^2), and the log-likelihood ratio
log f(Y|1)/f(Y|0) equals 2Y/sigma^2, so a positive LLR means bit 1.  Noise is
set from Eb/N0 in dB for a rate R = k/n code: sigma^2 = 1 / (2 R 10^(EbN0/10)).
"""
from __future__ import annotations

import numpy as np


def sigma2(ebn0_db: float, rate: float) -> float:
    return 1.0 / (2.0 * rate * 10.0 ** (ebn0_db / 10.0))


def encode(G: np.ndarray, msgs: np.ndarray) -> np.ndarray:
    """c = m G over GF(2); msgs is N x k of 0/1."""
    acc = msgs.astype(np.float32) @ G.astype(np.float32)
    return (acc.astype(np.int64) & 1).astype(np.uint8)


def awgn_llr(G: np.ndarray, n_blocks: int, ebn0_db: float, seed: int,
             chunk: int = 1 << 16):
    """Returns (llr float32 [N, n], codewords uint8 [N, n]) from a seeded PCG64."""
    k, n = G.shape
    s2 = sigma2(ebn0_db, k / n)
    sd = np.sqrt(s2)
    rng = np.random.Generator(np.random.PCG64(seed))
    llr = np.empty((n_blocks, n), dtype=np.float32)
    cws = np.empty((n_blocks, n), dtype=np.uint8)
    for s in range(0, n_blocks, chunk):
        e = min(n_blocks, s + chunk)
        m = rng.integers(0, 2, size=(e - s, k), dtype=np.uint8)
        c = encode(G, m)
        y = (2.0 * c.astype(np.float64) - 1.0) + sd * rng.standard_normal((e - s, n))
        llr[s:e] = (2.0 * y / s2).astype(np.float32)
        cws[s:e] = c
    return llr, cws


def awgn_llr_torch(G: np.ndarray, n_blocks: int, ebn0_db: float, seed: int, device):
    """Same channel drawn with torch on `device` (used where the batch is large);
    not bit-identical to awgn_llr, same distribution."""
    import torch
    k, n = G.shape
    s2 = sigma2(ebn0_db, k / n)
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    Gt = torch.as_tensor(G, dtype=torch.float32, device=device)
    llr = torch.empty((n_blocks, n), dtype=torch.float32, device=device)
    cws = torch.empty((n_blocks, n), dtype=torch.uint8, device=device)
    chunk = 1 << 18
    for s in range(0, n_blocks, chunk):
        e = min(n_blocks, s + chunk)
        m = torch.randint(0, 2, (e - s, k), generator=gen, device=device, dtype=torch.float32)
        c = (m @ Gt).to(torch.int64) & 1
        noise = torch.randn((e - s, n), generator=gen, device=device, dtype=torch.float32)
        y = (2.0 * c.to(torch.float32) - 1.0) + float(np.sqrt(s2)) * noise
        llr[s:e] = 2.0 * y / float(s2)
        cws[s:e] = c.to(torch.uint8)
    return llr, cws


def awgn_llr_torch_snr_range(G: np.ndarray, n_blocks: int, ebn0_lo: float, ebn0_hi: float, seed: int, device):
    """torch on `device`: each block draws its own Eb/N0 uniformly in [lo, hi] dB.
    Returns (llr float32 [N, n], codewords uint8 [N, n], ebn0 float32 [N])."""
    import torch
    k, n = G.shape
    R = k / n
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    Gt = torch.as_tensor(G, dtype=torch.float32, device=device)
    llr = torch.empty((n_blocks, n), dtype=torch.float32, device=device)
    cws = torch.empty((n_blocks, n), dtype=torch.uint8, device=device)
    snr = torch.empty(n_blocks, dtype=torch.float32, device=device)
    chunk = 1 << 18
    for s in range(0, n_blocks, chunk):
        e = min(n_blocks, s + chunk)
        eb = ebn0_lo + (ebn0_hi - ebn0_lo) * torch.rand(e - s, generator=gen, device=device)
        s2 = 1.0 / (2.0 * R * torch.pow(10.0, eb / 10.0))
        m = torch.randint(0, 2, (e - s, k), generator=gen, device=device, dtype=torch.float32)
        c = (m @ Gt).to(torch.int64) & 1
        noise = torch.randn((e - s, n), generator=gen, device=device, dtype=torch.float32)
        y = (2.0 * c.to(torch.float32) - 1.0) + torch.sqrt(s2)[:, None] * noise
        llr[s:e] = 2.0 * y / s2[:, None]
        cws[s:e] = c.to(torch.uint8)
        snr[s:e] = eb
    return llr, cws, snr
