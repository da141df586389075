"""GPU parity: the HIP decoder (through the C-ABI) against the CPU oracle, bit for
bit -- codeword, query count and abandon flag -- on the same seeded inputs."""
import os

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2202_13951_amd import binding
from synth import channel, codes

pytestmark = pytest.mark.gpu
THREADS = min(16, os.cpu_count() or 1)


def _gpu_decode(H, llr, budget, dev):
    cw, q, ab = binding.orbg_decode(H, torch.from_numpy(np.ascontiguousarray(llr)).to(dev), budget)
    torch.cuda.synchronize()
    return cw.cpu().numpy(), q.cpu().numpy().astype(np.uint64), ab.cpu().numpy()


def _assert_same(got, want, tag=""):
    gcw, gq, gab = got
    ocw, oq, oab = want
    bad = np.nonzero((gcw != ocw).any(axis=1) | (gq != oq) | (gab != oab))[0]
    assert bad.size == 0, (f"{tag}: {bad.size} blocks differ, first {bad[:8].tolist()}: "
                           f"gpu q={gq[bad[:4]].tolist()} oracle q={oq[bad[:4]].tolist()}")


@pytest.mark.parametrize("n,count", [(13, 2 ** 13), (32, 10 ** 4), (64, 70000), (127, 10 ** 5),
                                     (256, 2 ** 17)])
def test_schedule_equals_oracle_order(gpu_device, n, count):
    print(f"schedule n={n} count={count}", flush=True)
    got = binding.orbg_schedule_export(n, count).astype(np.int32)
    want = O.order_prefix_array(n, count)
    assert got.shape == want.shape
    bad = np.nonzero((got != want).any(axis=1))[0]
    assert bad.size == 0, f"first differing entry {bad[0]}: gpu {got[bad[0]]} oracle {want[bad[0]]}"


def test_rlc32_26_full_workload(gpu_device):
    """RLC(32,26), 4 dB, 10^4 blocks, budget 10^4: every block."""
    print("rlc32_26 4dB 1e4 blocks", flush=True)
    H, G = codes.code("rlc32_26")
    llr, _ = channel.awgn_llr(G, 10 ** 4, 4.0, seed=101)
    _assert_same(_gpu_decode(H, llr, 10 ** 4, gpu_device), O.decode(H, llr, 10 ** 4, THREADS), "rlc32")


@pytest.mark.parametrize("ebn0", [4.0, 5.5, 7.0])
def test_bch127_113_parity(gpu_device, ebn0):
    print(f"bch127 {ebn0} dB", flush=True)
    H, G = codes.code("bch127_113")
    llr, _ = channel.awgn_llr(G, 3000, ebn0, seed=int(ebn0 * 10))
    _assert_same(_gpu_decode(H, llr, 10 ** 5, gpu_device), O.decode(H, llr, 10 ** 5, THREADS), "bch")


@pytest.mark.parametrize("name,ebn0,N,budget", [
    ("rlc64_52", 3.0, 3000, 10 ** 6), ("rlc128_116", 3.0, 2000, 10 ** 6),
    ("rlc256_240", 4.0, 400, 10 ** 6), ("rlc128_105", 3.0, 400, 10 ** 6)])
def test_batched_codes_parity(gpu_device, name, ebn0, N, budget):
    print(f"{name} {ebn0} dB N={N}", flush=True)
    H, G = codes.code(name)
    llr, _ = channel.awgn_llr(G, N, ebn0, seed=N + 7)
    _assert_same(_gpu_decode(H, llr, budget, gpu_device), O.decode(H, llr, budget, THREADS), name)


@pytest.mark.parametrize("n,k", [(8, 3), (12, 2), (63, 50), (65, 52), (100, 36), (200, 180), (300, 280),
                                 (513, 500), (1024, 1000)])
def test_shapes_and_ragged_lengths(gpu_device, n, k):
    """Lengths that do not fill the 64-lane tiles, up to the 1024 maximum, and
    n - k = 64 (one full syndrome word)."""
    print(f"shape n={n} k={k}", flush=True)
    H = codes.rlc_H(n, k, seed=n * 7 + k)
    G = codes.generator_matrix(H)
    llr, _ = channel.awgn_llr(G, 300, 2.5, seed=n + k)
    budget = min(2 ** n, 3000)
    _assert_same(_gpu_decode(H, llr, budget, gpu_device), O.decode(H, llr, budget, THREADS), f"n={n}")


@pytest.mark.parametrize("n,k,N", [(127, 113, 1001), (100, 88, 777), (65, 52, 515)])
def test_rows_stay_inside_their_views(gpu_device, n, k, N):
    """Each block's outputs are written inside their own bytes only, and each
    block is decoded from its own row: the LLRs and the outputs are views one
    row into larger buffers whose first and last rows hold other data (LLRs of
    a large magnitude, so a row read from the wrong offset changes the
    results; sentinel bytes, which a stray store would change).  Several
    launch shapes, partial screening groups among them."""
    print(f"row views n={n} k={k} N={N}", flush=True)
    H = codes.bch_H(127, 113) if n == 127 else codes.rlc_H(n, k, seed=n * 11 + k)
    G = codes.generator_matrix(H)
    llr, _ = channel.awgn_llr(G, N, 4.0, seed=n + N)
    budget = 10 ** 4
    want = O.decode(H, llr, budget, THREADS)
    big = np.full((N + 2, n), -40.0, dtype=np.float32)
    big[1:N + 1] = llr
    xb = torch.from_numpy(big).to(gpu_device)
    for wgs, chunk in [(0, 0), (1, 5), (32, 32), (48, 3)]:
        cwb = torch.full((N + 2, n), 7, dtype=torch.uint8, device=gpu_device)
        qb = torch.full((N + 2,), -1, dtype=torch.int64, device=gpu_device)
        abb = torch.full((N + 2,), 9, dtype=torch.uint8, device=gpu_device)
        params = binding.LaunchParams(workgroups_per_cu=wgs, chunk=chunk, split_steps=0) if wgs else None
        binding.orbg_decode_ex(H, xb[1:N + 1], budget, params=params, out=(cwb[1:N + 1], qb[1:N + 1], abb[1:N + 1]))
        torch.cuda.synchronize()
        cw, q, ab = cwb.cpu().numpy(), qb.cpu().numpy(), abb.cpu().numpy()
        for r in (0, N + 1):
            assert (cw[r] == 7).all() and q[r] == -1 and ab[r] == 9, (wgs, chunk, r)
        _assert_same((cw[1:N + 1], q[1:N + 1].astype(np.uint64), ab[1:N + 1]), want, f"n={n} shape {wgs}/{chunk}")


def test_budget_edges_and_abandon(gpu_device):
    print("budget edges", flush=True)
    H = codes.rlc_H(40, 20, seed=5)                      # 20 parity bits: pure noise abandons
    rng = np.random.default_rng(8)
    llr = rng.standard_normal((200, 40)).astype(np.float32)
    for budget in (1, 2, 63, 64, 65, 127, 4097, 30000):
        got = _gpu_decode(H, llr, budget, gpu_device)
        _assert_same(got, O.decode(H, llr, budget, THREADS), f"budget={budget}")
    assert got[2].sum() > 0                              # some abandoned at 30000


def test_special_values_and_ties(gpu_device):
    print("special values", flush=True)
    H, G = codes.code("rlc64_52")
    rng = np.random.default_rng(4)
    llr = rng.standard_normal((64, 64)).astype(np.float32)
    llr[0] = 0.0
    llr[1] = -0.0
    llr[2] = 0.75                                        # all equal, all ones
    llr[3] = -0.75
    llr[4, ::3] = np.nan
    llr[5, :10] = np.inf
    llr[6, :10] = -np.inf
    llr[7] = np.round(llr[7])                            # many exact ties
    llr[8:16] = np.round(llr[8:16] * 4) / 4
    book = channel.encode(G, rng.integers(0, 2, (8, 52), dtype=np.uint8))
    llr[16:24] = (2.0 * book - 1.0) * 5.0                # already codewords: q = 1
    _assert_same(_gpu_decode(H, llr, 5000, gpu_device), O.decode(H, llr, 5000, THREADS), "special")


def test_empty_batch(gpu_device):
    H, _ = codes.code("rlc32_26")
    llr = torch.empty((0, 32), dtype=torch.float32, device=gpu_device)
    cw, q, ab = binding.orbg_decode(H, llr, 100)
    torch.cuda.synchronize()
    assert cw.shape == (0, 32) and q.shape == (0,)


def test_repeat_runs_identical(gpu_device):
    H, G = codes.code("bch127_113")
    llr, _ = channel.awgn_llr(G, 20000, 4.0, seed=3)
    a = _gpu_decode(H, llr, 10 ** 5, gpu_device)
    b = _gpu_decode(H, llr, 10 ** 5, gpu_device)
    for x, y in zip(a, b):
        assert (x == y).all()


@pytest.mark.parametrize("name,ebn0,N", [("rlc32_26", 3.0, 2000), ("rlc128_105", 3.5, 300)])
def test_ordered_decode_parity(gpu_device, name, ebn0, N):
    print(f"ordered {name}", flush=True)
    H, G = codes.code(name)
    llr, _ = channel.awgn_llr(G, N, ebn0, seed=99)
    rng = np.random.default_rng(1)
    order = np.stack([rng.permutation(64) for _ in range(N)]).astype(np.uint8)
    order[: N // 4] = np.arange(64, dtype=np.uint8)      # identity rows
    budget = 10 ** 4 if name == "rlc32_26" else 10 ** 6
    d = gpu_device
    cw, q, ab = binding.orbg_decode_ordered(H, torch.from_numpy(llr).to(d), budget,
                                            torch.from_numpy(order).to(d))
    torch.cuda.synchronize()
    got = (cw.cpu().numpy(), q.cpu().numpy().astype(np.uint64), ab.cpu().numpy())
    _assert_same(got, O.decode_ordered(H, llr, budget, order, THREADS), f"ordered {name}")
    plain = _gpu_decode(H, llr[: N // 4], budget, d)
    for x, y in zip(plain, (g[: N // 4] for g in got)):
        assert (x == y).all()


def test_bch_full_size_sampled(gpu_device):
    """The benchmark's shape (BCH(127,113), 10^6 blocks, budget 10^5, one launch
    in the tuned launch shape the benchmark times): sampled blocks against the
    oracle, invariants on every block, and the same results in the library's
    default launch shape."""
    print("bch full size", flush=True)
    from paper_2202_13951_amd import autotune
    H, G = codes.code("bch127_113")
    N, budget = 10 ** 6, 10 ** 5
    llr, _ = channel.awgn_llr(G, N, 4.0, seed=4242)
    knobs = autotune.load_tuned("bch127")
    assert knobs is not None
    x = torch.from_numpy(llr).to(gpu_device)
    cw_t, q_t, ab_t = binding.orbg_decode_ex(H, x, budget, params=binding.LaunchParams(**knobs))
    torch.cuda.synchronize()
    gcw, gq, gab = cw_t.cpu().numpy(), q_t.cpu().numpy().astype(np.uint64), ab_t.cpu().numpy()
    dcw, dq, dab = _gpu_decode(H, llr, budget, gpu_device)
    assert (dcw == gcw).all() and (dq == gq).all() and (dab == gab).all()
    rng = np.random.default_rng(0)
    idx = np.sort(np.concatenate([rng.choice(N, 400, replace=False), np.argsort(gq)[-50:]]))
    _assert_same((gcw[idx], gq[idx], gab[idx]), O.decode(H, llr[idx], budget, THREADS), "bch sampled")
    assert ((gq >= 1) & (gq <= budget)).all()
    assert (gq[gab == 1] == budget).all()
    Hf = torch.from_numpy(H.astype(np.float32)).to(gpu_device)
    ok = torch.from_numpy(gab == 0).to(gpu_device)
    syn = (torch.from_numpy(gcw).to(gpu_device).float() @ Hf.T).remainder(2)
    assert not syn[ok].any()


W99_PATTERNS = 4827382          # patterns of logistic weight <= 99 for n >= 99 (the coefficients of eq. (intpart))


@pytest.mark.parametrize("n", [64, 100, 256])
def test_schedule_to_the_papers_threshold(gpu_device, n):
    """The schedule for the paper's abandonment threshold of 5 x 10^6 queries
    (Sec. IV-A) equals the oracle's order entry for entry: all patterns of
    logistic weight <= 99, then those of weight 100 (which the schedule holds up
    to the one pattern with eight ranks above 8)."""
    count = 5 * 10 ** 6
    print(f"schedule n={n} count={count}", flush=True)
    got = binding.orbg_schedule_export(n, count).astype(np.int32)
    want = O.order_prefix_array(n, count)
    assert got.shape == want.shape == (count, 16)
    bad = np.nonzero((got != want).any(axis=1))[0]
    assert bad.size == 0, f"first differing entry {bad[0]}: gpu {got[bad[0]]} oracle {want[bad[0]]}"
    assert int(got[-1].sum()) == 100
    if n >= 99:
        assert int(got[W99_PATTERNS - 1].sum()) == 99 and int(got[W99_PATTERNS].sum()) == 100


def test_rlc256_234_at_the_papers_threshold(gpu_device):
    """RLC(256,234) (22 parity bits: the length and redundancy of the paper's
    CA-Polar[256,234]) at 4 dB with the paper's budget of 5 x 10^6 queries:
    every search that ends among the weight-100 patterns, some abandoned ones
    and a random sample, against the oracle element by element."""
    print("rlc256_234 budget 5e6", flush=True)
    H, G = codes.code("rlc256_234")
    N, budget = 3000, 5 * 10 ** 6
    llr, _ = channel.awgn_llr(G, N, 4.0, seed=606)
    gcw, gq, gab = _gpu_decode(H, llr, budget, gpu_device)
    assert ((gq >= 1) & (gq <= budget)).all() and (gq[gab == 1] == budget).all()
    w100 = np.nonzero((gq > W99_PATTERNS) & (gab == 0))[0]
    print(f"{w100.size} searches end among the weight-100 patterns, {int(gab.sum())} abandoned", flush=True)
    assert w100.size >= 1
    rng = np.random.default_rng(1)
    idx = np.unique(np.concatenate([w100[:8], np.nonzero(gab == 1)[0][:4], rng.choice(N, 32, replace=False)]))
    _assert_same((gcw[idx], gq[idx], gab[idx]), O.decode(H, llr[idx], budget, THREADS), "rlc256 5e6")
