"""GPU: the allocation-free mixed decode (orbg_decode_mixed_noalloc) against
orbg_decode_mixed, called through the C-ABI: two calls in a row, the second on
a smaller input, with and without the heavy pass; then its refusals (batch above
the scratch array's limit, a code whose schedule has not been built)."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2202_13951_amd import binding
from synth import codes, mixed

pytestmark = pytest.mark.gpu
NAMES = ["rlc64_52", "bch127_113", "rlc128_116", "rlc256_240"]


def _case(N, seed, dev):
    HG = [codes.code(nm) for nm in NAMES]
    llr, _, bc, ro, _ = mixed.mixed_llr_torch_snr_range([G for _, G in HG], [1, 1, 1, 1], N, 3.0, 6.0, seed=seed,
                                                        device=dev)
    return HG, llr, bc, ro


def _outs(llr, N, dev):
    return (torch.full((llr.numel(),), 5, dtype=torch.uint8, device=dev),
            torch.full((N,), -1, dtype=torch.int64, device=dev),
            torch.full((N,), 7, dtype=torch.uint8, device=dev))


@pytest.mark.parametrize("params", [None, dict(split_steps=2, heavy_waves=8, heavy_workgroups_per_cu=2)])
def test_noalloc_equals_mixed_decode_twice(gpu_device, params):
    dev = gpu_device
    budget = 10 ** 5
    p = binding.LaunchParams(**params) if params else None
    for call, (N, seed) in enumerate([(30000, 601), (7000, 602)]):
        print(f"no-alloc call {call}: {N} blocks, params {params}", flush=True)
        HG, llr, bc, ro = _case(N, seed, dev)
        ids = [binding.orbg_code_register(H) for H, _ in HG]
        ref = _outs(llr, N, dev)
        binding.orbg_decode_mixed(ids, bc, ro, llr, budget, *ref, params=p)     # builds the schedules
        got = _outs(llr, N, dev)
        binding.orbg_decode_mixed_noalloc(ids, bc, ro, llr, budget, *got, params=p)
        torch.cuda.synchronize()
        for a, b in zip(ref, got):
            assert torch.equal(a, b), call
        assert int(ref[1].min()) >= 1
        for i in ids:
            binding.orbg_code_release(i)


def test_noalloc_refusals(gpu_device):
    dev = gpu_device
    L = binding.load()
    H, _ = codes.code("rlc64_52")
    cid = binding.orbg_code_register(H)
    ids = (ctypes.c_int * 1)(cid)
    p = ctypes.c_void_p(8)
    big = binding.ORBG_NOALLOC_BATCH_MAX + 1
    rc = L.orbg_decode_mixed_noalloc(ids, 1, p, p, p, 1 << 30, big, 100, p, 1 << 30, p, p, None, None)
    assert rc == -1 and "above 262144" in L.orbg_last_error().decode()
    # a code of a length no other call uses: its schedule does not exist yet
    rng = np.random.default_rng(5)
    H77 = np.concatenate([rng.integers(0, 2, (17, 60)), np.eye(17, dtype=np.int64)], axis=1).astype(np.uint8)
    cid77 = binding.orbg_code_register(H77)
    N = 10
    llr = torch.ones(N * 77, dtype=torch.float32, device=dev)
    bc = torch.zeros(N, dtype=torch.uint8, device=dev)
    ro = torch.arange(N, dtype=torch.int64, device=dev) * 77
    outs = _outs(llr, N, dev)
    with pytest.raises(binding.OrbgError, match="no query schedule"):
        binding.orbg_decode_mixed_noalloc([cid77], bc, ro, llr, 12345, *outs)
    binding.orbg_decode_mixed([cid77], bc, ro, llr, 12345, *outs)
    outs2 = _outs(llr, N, dev)
    binding.orbg_decode_mixed_noalloc([cid77], bc, ro, llr, 12345, *outs2)
    torch.cuda.synchronize()
    for a, b in zip(outs, outs2):
        assert torch.equal(a, b)
    binding.orbg_code_release(cid)
    binding.orbg_code_release(cid77)
