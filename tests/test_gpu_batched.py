"""GPU: mixed-code persistent decodes, the heavy-block split and hipGraph replay.
Every result is checked bit for bit against the oracle or against the plain
single-code decode (itself parity-tested against the oracle)."""
import os

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2202_13951_amd import binding
from synth import codes, mixed

pytestmark = pytest.mark.gpu
THREADS = min(16, os.cpu_count() or 1)
NAMES = ["rlc64_52", "rlc128_116", "rlc256_240"]


def _setup(N, ebn0, seed, dev):
    HG = [codes.code(nm) for nm in NAMES]
    llr, sent, bc, ro = mixed.mixed_llr([G for _, G in HG], [1, 2, 1], N, ebn0, seed)
    ids = [binding.orbg_code_register(H) for H, _ in HG]
    t = dict(llr=torch.from_numpy(llr).to(dev), bc=torch.from_numpy(bc).to(dev), ro=torch.from_numpy(ro).to(dev))
    return HG, ids, llr, bc, ro, t


def _run_mixed(ids, t, N, budget, params=None):
    dev = t["llr"].device
    cw = torch.zeros(t["llr"].numel(), dtype=torch.uint8, device=dev)
    q = torch.zeros(N, dtype=torch.int64, device=dev)
    ab = torch.zeros(N, dtype=torch.uint8, device=dev)
    binding.orbg_decode_mixed(ids, t["bc"], t["ro"], t["llr"], budget, cw, q, ab, params=params)
    torch.cuda.synchronize()
    return cw.cpu().numpy(), q.cpu().numpy().astype(np.uint64), ab.cpu().numpy()


def _rows(flat, ro, n, idx):
    return flat[ro[idx][:, None] + np.arange(n)[None, :]]


def test_mixed_matches_oracle(gpu_device):
    print("mixed vs oracle", flush=True)
    N, budget = 2400, 10 ** 6
    HG, ids, llr, bc, ro, t = _setup(N, 4.0, 11, gpu_device)
    cw, q, ab = _run_mixed(ids, t, N, budget)
    for ci, (H, G) in enumerate(HG):
        n = H.shape[1]
        idx = np.nonzero(bc == ci)[0]
        if ci == 2:
            idx = idx[:300]
        ocw, oq, oab = O.decode(H, _rows(llr, ro, n, idx), budget, THREADS)
        assert (_rows(cw, ro, n, idx) == ocw).all(), NAMES[ci]
        assert (q[idx] == oq).all() and (ab[idx] == oab).all(), NAMES[ci]
    assert (q > 64 * 64).any()                      # the heavy pass took part


@pytest.mark.parametrize("params", [
    dict(split_steps=0), dict(split_steps=1), dict(split_steps=3, heavy_waves=4),
    dict(split_steps=64, heavy_waves=16, heavy_workgroups_per_cu=1), dict(workgroups_per_cu=1, chunk=7),
    dict(workgroups_per_cu=64, chunk=1, split_steps=8, heavy_waves=8, heavy_workgroups_per_cu=16),
    dict(one_block_per_workgroup=1)])
def test_schedule_invariance(gpu_device, params):
    """Any launch shape gives the same bits as the plain per-code decode."""
    print(f"invariance {params}", flush=True)
    N, budget = 6000, 10 ** 6
    HG, ids, llr, bc, ro, t = _setup(N, 3.5, 12, gpu_device)
    got = _run_mixed(ids, t, N, budget, binding.LaunchParams(**params))
    for ci, (H, G) in enumerate(HG):
        n = H.shape[1]
        idx = np.nonzero(bc == ci)[0]
        rows = torch.from_numpy(np.ascontiguousarray(_rows(llr, ro, n, idx))).to(gpu_device)
        pcw, pq, pab = binding.orbg_decode(H, rows, budget)
        torch.cuda.synchronize()
        assert (_rows(got[0], ro, n, idx) == pcw.cpu().numpy()).all()
        assert (got[1][idx] == pq.cpu().numpy().astype(np.uint64)).all()
        assert (got[2][idx] == pab.cpu().numpy()).all()


@pytest.mark.parametrize("split,waves", [(0, 8), (1, 4), (2, 16), (64, 8), (300, 4)])
def test_single_code_split_invariance(gpu_device, split, waves):
    print(f"single split {split} {waves}", flush=True)
    H, G = codes.code("bch127_113")
    from synth import channel
    llr, _ = channel.awgn_llr(G, 20000, 4.0, seed=77)
    x = torch.from_numpy(llr).to(gpu_device)
    ref = [v.cpu().numpy() for v in binding.orbg_decode_ex(H, x, 10 ** 5, params=binding.LaunchParams(split_steps=0))]
    got = [v.cpu().numpy() for v in binding.orbg_decode_ex(
        H, x, 10 ** 5, params=binding.LaunchParams(split_steps=split, heavy_waves=waves))]
    for a, b in zip(ref, got):
        assert (a == b).all()
    sample = np.arange(0, 20000, 40)
    ocw, oq, oab = O.decode(H, llr[sample], 10 ** 5, THREADS)
    assert (got[0][sample] == ocw).all() and (got[1][sample].astype(np.uint64) == oq).all()


def test_single_code_naive_launch(gpu_device):
    """One one-wave workgroup per block (no work counter, no split): the same bits
    as the persistent launch, and the oracle's on a sample."""
    print("single naive launch", flush=True)
    H, G = codes.code("bch127_113")
    from synth import channel
    llr, _ = channel.awgn_llr(G, 20000, 4.5, seed=78)
    x = torch.from_numpy(llr).to(gpu_device)
    ref = [v.cpu().numpy() for v in binding.orbg_decode_ex(H, x, 10 ** 5)]
    got = [v.cpu().numpy() for v in binding.orbg_decode_ex(
        H, x, 10 ** 5, params=binding.LaunchParams(one_block_per_workgroup=1))]
    for a, b in zip(ref, got):
        assert (a == b).all()
    sample = np.arange(0, 20000, 50)
    ocw, oq, oab = O.decode(H, llr[sample], 10 ** 5, THREADS)
    assert (got[0][sample] == ocw).all() and (got[1][sample].astype(np.uint64) == oq).all()


@pytest.mark.parametrize("N", [1, 7, 63, 64, 65, 511, 4097])
def test_work_slices_cover_every_block_once(gpu_device, N):
    """The persistent launch deals the blocks to 64 work slices in stripes;
    batches smaller than the slice count, ragged last stripes, chunks of any size
    and launches of few or many workgroups must write every block once with the
    same bits as one one-wave workgroup per block (no work counter).  Outputs
    start from a sentinel, so a block left out or written from another row
    shows."""
    print(f"work slices N={N}", flush=True)
    H, G = codes.code("bch127_113")
    from synth import channel
    llr, _ = channel.awgn_llr(G, N, 4.0, seed=300 + N)
    x = torch.from_numpy(llr).to(gpu_device)
    budget = 10 ** 4

    def run(params):
        cw = torch.full((N, H.shape[1]), 7, dtype=torch.uint8, device=gpu_device)
        q = torch.full((N,), -1, dtype=torch.int64, device=gpu_device)
        ab = torch.full((N,), 9, dtype=torch.uint8, device=gpu_device)
        binding.orbg_decode_ex(H, x, budget, params=params, out=(cw, q, ab))
        torch.cuda.synchronize()
        return [v.cpu().numpy() for v in (cw, q, ab)]

    ref = run(binding.LaunchParams(one_block_per_workgroup=1))
    assert (ref[1] > 0).all() and (ref[0] <= 1).all() and (ref[2] <= 1).all()
    for wgs, chunk in [(1, 1), (1, 5), (2, 64), (32, 32), (48, 3), (64, 1)]:
        got = run(binding.LaunchParams(workgroups_per_cu=wgs, chunk=chunk, split_steps=0))
        for a, b in zip(ref, got):
            assert (a == b).all(), (wgs, chunk)


def test_hip_graph_replay(gpu_device):
    """The mixed decode (counter reset, light pass, heavy pass) captured in a graph:
    every replay, with eager work in between, equals the eager result."""
    print("graph replay", flush=True)
    N, budget = 3000, 10 ** 6
    HG, ids, llr, bc, ro, t = _setup(N, 3.5, 13, gpu_device)
    eager = _run_mixed(ids, t, N, budget)
    s = torch.cuda.Stream()
    cw = torch.zeros(t["llr"].numel(), dtype=torch.uint8, device=gpu_device)
    q = torch.zeros(N, dtype=torch.int64, device=gpu_device)
    ab = torch.zeros(N, dtype=torch.uint8, device=gpu_device)
    with torch.cuda.stream(s):                        # warm-up: work space for this stream
        binding.orbg_decode_mixed(ids, t["bc"], t["ro"], t["llr"], budget, cw, q, ab)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        binding.orbg_decode_mixed(ids, t["bc"], t["ro"], t["llr"], budget, cw, q, ab)
    for rep in range(3):
        cw.fill_(7)
        q.fill_(-1)
        ab.fill_(9)
        _run_mixed(ids, t, N, budget)                 # eager work between replays
        g.replay()
        torch.cuda.synchronize()
        assert (cw.cpu().numpy() == eager[0]).all(), rep
        assert (q.cpu().numpy().astype(np.uint64) == eager[1]).all(), rep
        assert (ab.cpu().numpy() == eager[2]).all(), rep


def test_mixed_full_size_sampled(gpu_device):
    """The benchmark's mixed shape at its hardest point: 4 x 10^6 blocks of
    (64,52):(128,116):(256,240) = 1:2:1 at 3 dB, budget 10^6, one launch in the
    tuned launch shape the benchmark times.  Sampled blocks of every code (among
    them the 50 that needed most queries) against the oracle; on every block
    1 <= q <= budget, abandoned blocks at q = budget, and returned words with a
    zero syndrome."""
    print("mixed full size", flush=True)
    from paper_2202_13951_amd import autotune
    HG = [codes.code(nm) for nm in NAMES]
    N, budget = 4 * 10 ** 6, 10 ** 6
    llr, _, bc, ro = mixed.mixed_llr_torch([G for _, G in HG], [1, 2, 1], N, 3.0, seed=2030, device=gpu_device)
    ids = [binding.orbg_code_register(H) for H, _ in HG]
    cw = torch.zeros(llr.numel(), dtype=torch.uint8, device=gpu_device)
    q = torch.zeros(N, dtype=torch.int64, device=gpu_device)
    ab = torch.zeros(N, dtype=torch.uint8, device=gpu_device)
    params = binding.LaunchParams(**autotune.load_tuned("mixed"))
    binding.orbg_decode_mixed(ids, bc, ro, llr, budget, cw, q, ab, params=params)
    torch.cuda.synchronize()
    qn, abn, bcn, ron = q.cpu().numpy().astype(np.uint64), ab.cpu().numpy(), bc.cpu().numpy(), ro.cpu().numpy()
    assert ((qn >= 1) & (qn <= budget)).all() and (qn[abn == 1] == budget).all()
    rng = np.random.default_rng(3)
    for ci, (H, G) in enumerate(HG):
        n = H.shape[1]
        mine = np.nonzero(bcn == ci)[0]
        idx = np.unique(np.concatenate([rng.choice(mine, 120, replace=False), mine[np.argsort(qn[mine])[-17:]]]))
        pos = torch.from_numpy(ron[idx][:, None] + np.arange(n)[None, :]).to(gpu_device)
        rows = llr[pos].cpu().numpy()
        ocw, oq, oab = O.decode(H, rows, budget, THREADS)
        assert (cw[pos].cpu().numpy() == ocw).all(), NAMES[ci]
        assert (qn[idx] == oq).all() and (abn[idx] == oab).all(), NAMES[ci]
        # every returned word of this code has a zero syndrome (or is an abandoned hard decision)
        sel = torch.from_numpy(mine).to(gpu_device)
        allpos = ro[sel][:, None] + torch.arange(n, device=gpu_device)[None, :]
        words = cw[allpos].float()
        syn = (words @ torch.from_numpy(H.astype(np.float32)).to(gpu_device).T).remainder(2)
        ok = ab[sel] == 0
        assert not syn[ok].any(), NAMES[ci]
        del allpos, words, syn


STREAM_NAMES = ["rlc64_52", "bch127_113", "rlc128_116", "rlc256_240"]
_STREAM_CACHE = {}


def _stream_case(dev):
    """The request stream's code set (four codes, one of odd length) in one flat
    buffer, every block with its own Eb/N0 uniform in [3, 6] dB, budget 10^5."""
    if "case" not in _STREAM_CACHE:
        HG = [codes.code(nm) for nm in STREAM_NAMES]
        N = 40000
        llr, _, bc, ro, _ = mixed.mixed_llr_torch_snr_range([G for _, G in HG], [1, 1, 1, 1], N, 3.0, 6.0,
                                                            seed=5150, device=dev)
        _STREAM_CACHE["case"] = (HG, N, llr, bc, ro)
    return _STREAM_CACHE["case"]


@pytest.mark.parametrize("shape", ["stream", "mixed_tuned"])
def test_stream_code_set_matches_oracle(gpu_device, shape):
    """The request stream's four codes (RLC(64,52), BCH(127,113), RLC(128,116),
    RLC(256,240)) shuffled into one mixed launch, in the stream's launch shape
    (chunk 1, split after 16 steps, 16 heavy waves: the heavy pass on) and in the
    tuned bulk shape.  Sampled blocks of every code, among them each code's
    deepest searches, against the oracle element by element (codeword, queries,
    abandon flag)."""
    from paper_2202_13951_amd import autotune
    print(f"stream code set, {shape} shape", flush=True)
    HG, N, llr, bc, ro = _stream_case(gpu_device)
    budget = 10 ** 5
    if shape == "stream":
        params = binding.LaunchParams(workgroups_per_cu=32, chunk=1, split_steps=16, heavy_waves=16,
                                      heavy_workgroups_per_cu=2)
    else:
        params = binding.LaunchParams(**autotune.load_tuned("mixed"))
    ids = [binding.orbg_code_register(H) for H, _ in HG]
    cw = torch.zeros(llr.numel(), dtype=torch.uint8, device=gpu_device)
    q = torch.zeros(N, dtype=torch.int64, device=gpu_device)
    ab = torch.zeros(N, dtype=torch.uint8, device=gpu_device)
    binding.orbg_decode_mixed(ids, bc, ro, llr, budget, cw, q, ab, params=params)
    torch.cuda.synchronize()
    qn, abn, bcn, ron = q.cpu().numpy().astype(np.uint64), ab.cpu().numpy(), bc.cpu().numpy(), ro.cpu().numpy()
    cwn, llrn = cw.cpu().numpy(), llr.cpu().numpy()
    assert ((qn >= 1) & (qn <= budget)).all()
    if shape == "stream":
        assert (qn > 16 * 64).sum() >= 20                # the heavy pass took part
    rng = np.random.default_rng(17)
    for ci, (H, G) in enumerate(HG):
        n = H.shape[1]
        mine = np.nonzero(bcn == ci)[0]
        idx = np.unique(np.concatenate([rng.choice(mine, 300, replace=False), mine[np.argsort(qn[mine])[-12:]]]))
        key = (ci, idx.tobytes())
        if key not in _STREAM_CACHE:
            _STREAM_CACHE[key] = O.decode(H, _rows(llrn, ron, n, idx), budget, THREADS)
        ocw, oq, oab = _STREAM_CACHE[key]
        assert (_rows(cwn, ron, n, idx) == ocw).all(), STREAM_NAMES[ci]
        assert (qn[idx] == oq).all(), STREAM_NAMES[ci]
        assert (abn[idx] == oab).all(), STREAM_NAMES[ci]


def test_rows_outside_the_buffers_read_zeros_and_store_nothing(gpu_device):
    """A mixed decode bounds every row by the LLR and codeword lengths it is
    given: a row with a negative offset, or one that would run past either
    buffer, is decoded from zeros (query 1, not abandoned) and leaves the
    codeword buffer untouched; the other blocks decode as usual."""
    print("mixed rows outside the buffers", flush=True)
    N, budget = 600, 10 ** 4
    HG, ids, llr, bc, ro, t = _setup(N, 4.0, 21, gpu_device)
    bad = {5: -3, 17: llr.size - 10, 40: -(1 << 40), 41: (1 << 40)}
    ro_bad = ro.copy()
    for i, v in bad.items():
        ro_bad[i] = v
    t_bad = dict(t, ro=torch.from_numpy(ro_bad).to(gpu_device))
    ref = _run_mixed(ids, t, N, budget)
    dev = gpu_device
    cw = torch.full((llr.size,), 7, dtype=torch.uint8, device=dev)
    q = torch.zeros(N, dtype=torch.int64, device=dev)
    ab = torch.full((N,), 9, dtype=torch.uint8, device=dev)
    binding.orbg_decode_mixed(ids, t_bad["bc"], t_bad["ro"], t["llr"], budget, cw, q, ab)
    torch.cuda.synchronize()
    cwn, qn, abn = cw.cpu().numpy(), q.cpu().numpy(), ab.cpu().numpy()
    good = np.array([i for i in range(N) if i not in bad])
    for ci, (H, G) in enumerate(HG):
        n = H.shape[1]
        idx = good[bc[good] == ci]
        assert (_rows(cwn, ro, n, idx) == _rows(ref[0], ro, n, idx)).all()
    assert (qn[good].astype(np.uint64) == ref[1][good]).all() and (abn[good] == ref[2][good]).all()
    for i in bad:
        assert qn[i] == 1 and abn[i] == 0, i
    # every byte not inside a good block's row still holds the fill value
    touched = np.zeros(llr.size, dtype=bool)
    for i in good:
        touched[ro[i]:ro[i] + HG[bc[i]][0].shape[1]] = True
    assert (cwn[~touched] == 7).all()


def test_binding_rejects_bad_output_tensors(gpu_device):
    H, _ = codes.code("rlc32_26")
    llr = torch.zeros((4, 32), dtype=torch.float32, device=gpu_device)
    bad = [(torch.zeros((4, 32), dtype=torch.uint8, device=gpu_device), torch.zeros(4, dtype=torch.int32,
            device=gpu_device), torch.zeros(4, dtype=torch.uint8, device=gpu_device)),
           (torch.zeros((4, 31), dtype=torch.uint8, device=gpu_device), torch.zeros(4, dtype=torch.int64,
            device=gpu_device), torch.zeros(4, dtype=torch.uint8, device=gpu_device)),
           (torch.zeros((4, 32), dtype=torch.uint8), torch.zeros(4, dtype=torch.int64),
            torch.zeros(4, dtype=torch.uint8))]
    for out in bad:
        with pytest.raises(ValueError):
            binding.orbg_decode(H, llr, 100, out=out)
