"""GPU parity of 1-line ORBGRAND (Sec. III-D/III-E with one segment): the device schedules
against the oracle's order for every offset class, and the HIP decoder against the
oracle decoder bit for bit -- codeword, query count, abandon flag and the fitted
offset J0 -- on the same seeded inputs."""
import os

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2202_13951_amd import binding
from synth import channel, codes

pytestmark = pytest.mark.gpu
THREADS = min(16, os.cpu_count() or 1)


def _gpu(H, llr, budget, dev, j0=True, params=None):
    cw, q, ab, jj = binding.orbg_decode_1line(H, torch.from_numpy(np.ascontiguousarray(llr)).to(dev), budget,
                                              j0=j0, params=params)
    torch.cuda.synchronize()
    return (cw.cpu().numpy(), q.cpu().numpy().astype(np.uint64), ab.cpu().numpy(),
            None if jj is None else jj.cpu().numpy())


def _assert_same(got, want, tag="", check_j0=True):
    gcw, gq, gab, gj = got
    ocw, oq, oab, oj = want
    diff = (gcw != ocw).any(axis=1) | (gq != oq) | (gab != oab)
    if check_j0:
        diff |= gj != oj
    bad = np.nonzero(diff)[0]
    assert bad.size == 0, (f"{tag}: {bad.size} blocks differ, first {bad[:8].tolist()}: gpu q={gq[bad[:4]].tolist()} "
                           f"oracle q={oq[bad[:4]].tolist()} gpu j0={None if gj is None else gj[bad[:4]].tolist()} "
                           f"oracle j0={oj[bad[:4]].tolist()}")


@pytest.mark.parametrize("n,budget", [(13, 2 ** 13), (32, 10 ** 4), (64, 10 ** 5), (127, 10 ** 5)])
def test_schedules_equal_oracle_order(gpu_device, n, budget):
    """Every offset with a schedule of its own (spot checks in the middle) and offsets
    above j0max, which share the last schedule, against the oracle's order for the
    offset itself: the prefix the decoder tests is the oracle's."""
    print(f"1-line schedules n={n} budget={budget}", flush=True)
    _, j0max = binding.orbg_schedule_export_1line(n, budget, 0, 0)
    assert j0max >= 1
    count = min(budget, 30000)
    js = sorted({-1, 0, 1, 2, 3, 5, 8, 13, j0max // 2, j0max - 1, j0max, j0max + 1, 3 * j0max + 7, (1 << 20) - 1})
    for j in js:
        got, jm = binding.orbg_schedule_export_1line(n, budget, j, count)
        assert jm == j0max
        want = O.order1_prefix_array(n, j, count)
        bad = np.nonzero((got.astype(np.int32) != want).any(axis=1))[0]
        assert bad.size == 0, f"j0={j}: first differing entry {bad[0]}: gpu {got[bad[0]]} oracle {want[bad[0]]}"
    # one schedule in full
    got, _ = binding.orbg_schedule_export_1line(n, budget, 1, budget)
    want = O.order1_prefix_array(n, 1, budget)
    assert (got.astype(np.int32) == want).all()


def test_rlc32_26_workload(gpu_device):
    print("1-line rlc32_26 4dB", flush=True)
    H, G = codes.code("rlc32_26")
    llr, _ = channel.awgn_llr(G, 10 ** 4, 4.0, seed=211)
    want = O.decode_1line(H, llr, 10 ** 4, THREADS)
    assert len(set(want[3].tolist())) >= 3
    _assert_same(_gpu(H, llr, 10 ** 4, gpu_device), want, "rlc32")
    got = _gpu(H, llr, 10 ** 4, gpu_device, j0=None)          # offsets not asked for: screening path
    _assert_same(got, want, "rlc32 no j0", check_j0=False)


@pytest.mark.parametrize("ebn0", [4.0, 5.5, 7.0])
def test_bch127_113_parity(gpu_device, ebn0):
    print(f"1-line bch127 {ebn0} dB", flush=True)
    H, G = codes.code("bch127_113")
    llr, _ = channel.awgn_llr(G, 3000, ebn0, seed=int(ebn0 * 10) + 500)
    want = O.decode_1line(H, llr, 10 ** 5, THREADS)
    _assert_same(_gpu(H, llr, 10 ** 5, gpu_device), want, "bch")
    _assert_same(_gpu(H, llr, 10 ** 5, gpu_device, j0=None), want, "bch no j0", check_j0=False)


@pytest.mark.parametrize("params", [
    dict(split_steps=0), dict(split_steps=1, heavy_waves=4), dict(split_steps=3, heavy_waves=16),
    dict(workgroups_per_cu=2, chunk=1, split_steps=8, heavy_waves=8, heavy_workgroups_per_cu=1)])
def test_launch_shapes(gpu_device, params):
    """Light pass alone, and heavy passes entered after 1, 3 and 8 steps: the same
    results (the heavy pass fits the offset again)."""
    print(f"1-line params {params}", flush=True)
    H, G = codes.code("bch127_113")
    llr, _ = channel.awgn_llr(G, 1500, 4.0, seed=77)
    want = O.decode_1line(H, llr, 10 ** 5, THREADS)
    p = binding.LaunchParams(**params)
    _assert_same(_gpu(H, llr, 10 ** 5, gpu_device, params=p), want, str(params))
    _assert_same(_gpu(H, llr, 10 ** 5, gpu_device, params=p, j0=None), want, f"{params} no j0", check_j0=False)


@pytest.mark.parametrize("n,k,budget,ebn0", [(8, 3, 2 ** 8, 1.0), (12, 5, 2 ** 12, 1.5), (63, 50, 20000, 2.5),
                                             (65, 52, 20000, 2.5), (100, 36, 3000, 2.5),
                                             (128, 80, 5000, 3.0), (200, 180, 256, 3.0), (300, 280, 256, 3.0),
                                             (1024, 1000, 200, 3.0)])
def test_shapes_and_ragged_lengths(gpu_device, n, k, budget, ebn0):
    """Ragged lengths, 1 to 16 keys per lane, 32- and 64-bit syndromes (n - k = 64
    for (100, 36)... and 48 for (128, 80)), and the largest budgets long codes allow."""
    print(f"1-line shape n={n} k={k} budget={budget}", flush=True)
    H = codes.rlc_H(n, k, seed=n * 5 + k)
    G = codes.generator_matrix(H)
    llr, _ = channel.awgn_llr(G, 300, ebn0, seed=n + 3 * k)
    want = O.decode_1line(H, llr, budget, THREADS)
    _assert_same(_gpu(H, llr, budget, gpu_device), want, f"n={n}")
    _assert_same(_gpu(H, llr, budget, gpu_device, j0=None), want, f"n={n} no j0", check_j0=False)


def test_special_values_and_fit_edges(gpu_device):
    """Zero, NaN and infinite LLRs, exact ties at the anchors, constant magnitudes
    (slope 0: J0 = 0), large offsets (far above j0max: clamped schedule) and the
    rounding boundary [x.5]."""
    print("1-line special values", flush=True)
    H, G = codes.code("rlc64_52")
    rng = np.random.default_rng(12)
    llr = rng.standard_normal((96, 64)).astype(np.float32)
    llr[0] = 0.0
    llr[1] = -0.0
    llr[2] = 0.75
    llr[3] = -0.75
    llr[4, ::3] = np.nan
    llr[5, :40] = np.inf
    llr[6, :10] = -np.inf
    llr[7] = np.round(llr[7])
    llr[8:16] = np.round(llr[8:16] * 4) / 4                   # many ties, also at ranks 1 and 32
    for b in range(16, 40):                                   # lines with large offsets
        off, slope = 10.0 ** rng.uniform(0, 3), 10.0 ** rng.uniform(-4, 0)
        mag = (off + slope * np.arange(1, 65)).astype(np.float32)
        llr[b] = (rng.permutation(mag) * rng.choice([-1, 1], 64)).astype(np.float32)
    for b in range(40, 48):                                   # L_1 / Q = j + 1/2 exactly: rounds up
        mag = np.concatenate([[2.5 + b - 40], 3.5 + b - 40 + np.arange(31), 100 + np.arange(32)]).astype(np.float32)
        llr[b] = (rng.permutation(mag) * rng.choice([-1, 1], 64)).astype(np.float32)
    book = channel.encode(G, rng.integers(0, 2, (8, 52), dtype=np.uint8))
    llr[48:56] = (2.0 * book - 1.0) * 5.0                     # codewords: q = 1
    want = O.decode_1line(H, llr, 5000, THREADS)
    assert want[3][16:40].max() > 300                         # above j0max (largest W of the prefix)
    _assert_same(_gpu(H, llr, 5000, gpu_device), want, "special")
    _assert_same(_gpu(H, llr, 5000, gpu_device, j0=None), want, "special no j0", check_j0=False)


def test_budget_edges(gpu_device):
    print("1-line budget edges", flush=True)
    H = codes.rlc_H(40, 20, seed=5)
    rng = np.random.default_rng(8)
    llr = rng.standard_normal((200, 40)).astype(np.float32)
    for budget in (1, 2, 63, 64, 65, 127, 4097, 30000):
        want = O.decode_1line(H, llr, budget, THREADS)
        _assert_same(_gpu(H, llr, budget, gpu_device), want, f"budget={budget}")
        _assert_same(_gpu(H, llr, budget, gpu_device, j0=None), want, f"budget={budget} no j0", check_j0=False)
    assert want[2].sum() > 0


def test_empty_batch_and_unsupported(gpu_device):
    H, _ = codes.code("rlc32_26")
    llr = torch.empty((0, 32), dtype=torch.float32, device=gpu_device)
    cw, q, ab, j0 = binding.orbg_decode_1line(H, llr, 100)
    torch.cuda.synchronize()
    assert cw.shape == (0, 32) and j0.shape == (0,)
    H600 = codes.rlc_H(600, 590, seed=3)
    llr = torch.zeros((4, 600), dtype=torch.float32, device=gpu_device)
    with pytest.raises(binding.OrbgError):                    # past the schedules and past n = 512
        binding.orbg_decode_1line(H600, llr, (1 << 22) + 1)


@pytest.mark.parametrize("name,ebn0,budget,N", [("rlc256_234", 5.0, 10 ** 5, 300), ("rlc256_240", 4.0, 1000, 400),
                                                ("bch127_113", 3.5, 4 * 10 ** 5, 200),
                                                ("rlc64_52", 2.0, 5 * 10 ** 6, 40)])
def test_beyond_the_schedules(gpu_device, name, ebn0, budget, N):
    """Orders the per-offset schedules cannot hold (n = 256 past a budget of 256,
    BCH(127,113) past about 2.86 x 10^5, any budget past 2^22) decode on the
    one-segment m-line kernel: codeword, queries, abandon flag and J0 against
    the oracle's 1-line decoder."""
    print(f"1-line beyond the schedules {name} budget={budget}", flush=True)
    H, G = codes.code(name)
    llr, _ = channel.awgn_llr(G, N, ebn0, seed=2561)
    want = O.decode_1line(H, llr, budget, THREADS)
    _assert_same(_gpu(H, llr, budget, gpu_device), want, name)
    _assert_same(_gpu(H, llr, budget, gpu_device, j0=None), want, name + " no j0", check_j0=False)
    assert (want[1] > 256).any()


def test_bch_full_size_sampled(gpu_device):
    """BCH(127,113), 10^6 blocks at 5 dB, budget 10^5, one launch: sampled blocks
    against the oracle, invariants on every block; the launch without offsets
    (patterns {1} and {2} tested before any sort) returns the same results."""
    print("1-line bch full size", flush=True)
    from paper_2202_13951_amd import autotune
    H, G = codes.code("bch127_113")
    N, budget = 10 ** 6, 10 ** 5
    llr, _ = channel.awgn_llr(G, N, 5.0, seed=5151)
    tuned = binding.LaunchParams(**autotune.load_tuned("bch127_1line"))      # the shape the benchmark times
    gcw, gq, gab, gj = _gpu(H, llr, budget, gpu_device, params=tuned)
    rng = np.random.default_rng(1)
    idx = np.sort(np.concatenate([rng.choice(N, 400, replace=False), np.argsort(gq)[-50:]]))
    want = O.decode_1line(H, llr[idx], budget, THREADS)
    _assert_same((gcw[idx], gq[idx], gab[idx], gj[idx]), want, "bch sampled")
    assert ((gq >= 1) & (gq <= budget)).all() and (gq[gab == 1] == budget).all() and (gj >= -1).all()
    Hf = torch.from_numpy(H.astype(np.float32)).to(gpu_device)
    ok = torch.from_numpy(gab == 0).to(gpu_device)
    syn = (torch.from_numpy(gcw).to(gpu_device).float() @ Hf.T).remainder(2)
    assert not syn[ok].any()
    ncw, nq, nab, _ = _gpu(H, llr, budget, gpu_device, j0=None, params=tuned)
    assert (ncw == gcw).all() and (nq == gq).all() and (nab == gab).all()


def test_hip_graph_replay(gpu_device):
    """The 1-line decode (counter reset, light pass with the offset fit, heavy
    pass) captured in a graph: every replay, with eager work in between, equals
    the eager result, offsets included."""
    print("1-line graph replay", flush=True)
    H, G = codes.code("bch127_113")
    llr, _ = channel.awgn_llr(G, 4000, 4.5, seed=808)
    x = torch.from_numpy(llr).to(gpu_device)
    budget = 10 ** 5
    params = binding.LaunchParams(split_steps=8)                # the heavy pass takes part
    eager = _gpu(H, llr, budget, gpu_device, params=params)
    N, n = llr.shape
    s = torch.cuda.Stream()
    cw = torch.zeros((N, n), dtype=torch.uint8, device=gpu_device)
    q = torch.zeros(N, dtype=torch.int64, device=gpu_device)
    ab = torch.zeros(N, dtype=torch.uint8, device=gpu_device)
    j0 = torch.zeros(N, dtype=torch.int32, device=gpu_device)
    with torch.cuda.stream(s):                                  # warm-up: schedules, work space
        binding.orbg_decode_1line(H, x, budget, j0=j0, params=params, out=(cw, q, ab), stream=s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        binding.orbg_decode_1line(H, x, budget, j0=j0, params=params, out=(cw, q, ab), stream=s)
    for rep in range(3):
        cw.fill_(7)
        q.fill_(-1)
        ab.fill_(9)
        j0.fill_(-9)
        _gpu(H, llr, budget, gpu_device, params=params)         # eager work between replays
        g.replay()
        torch.cuda.synchronize()
        got = (cw.cpu().numpy(), q.cpu().numpy().astype(np.uint64), ab.cpu().numpy(), j0.cpu().numpy())
        _assert_same(got, eager, f"replay {rep}")
    assert (eager[1] > 8 * 64).any()                            # some blocks reached the heavy pass
