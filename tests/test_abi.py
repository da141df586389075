"""CPU checks of the C-ABI library: it loads, exports every symbol the public
header declares, and rejects bad arguments before touching the device."""
import ctypes

import numpy as np
import pytest

from paper_2202_13951_amd import binding


def test_library_exports_header_symbols():
    L = binding.load()
    syms = binding.header_symbols()
    assert {"orbg_decode", "orbg_decode_ordered", "orbg_schedule_export", "orbg_last_error"} <= set(syms)
    for s in syms:
        assert hasattr(L, s), s


@pytest.mark.parametrize("n,k,budget,Hval,msg", [
    (0, 0, 10, 0, "n = 0"),
    (1025, 1000, 10, 0, "n = 1025"),
    (100, 30, 10, 0, "n - k = 70"),
    (32, 32, 10, 0, "n - k = 0"),
    (32, 26, 0, 0, "budget = 0"),
    (32, 26, (1 << 28) + 1, 0, "budget"),
    (32, 26, 10, 2, "is not 0 or 1"),
])
def test_argument_errors_are_einval(n, k, budget, Hval, msg):
    L = binding.load()
    m = max(n - k, 1)
    H = np.zeros((m, max(n, 1)), dtype=np.uint8)
    H[0, 0] = Hval
    rc = L.orbg_decode(H.ctypes.data_as(ctypes.c_void_p), None, n, k, budget, 4, None, None, None, None)
    assert rc == -1
    assert msg in L.orbg_last_error().decode()


def test_ordered_needs_n_at_least_12():
    L = binding.load()
    H = np.zeros((3, 10), dtype=np.uint8)
    rc = L.orbg_decode_ordered(H.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(8), 10, 7, 100, 1,
                               ctypes.c_void_p(8), ctypes.c_void_p(8), ctypes.c_void_p(8),
                               ctypes.c_void_p(8), None)
    assert rc == -1 and "n >= 12" in L.orbg_last_error().decode()


@pytest.mark.parametrize("field,value,msg", [
    ("workgroups_per_cu", 65, "workgroups_per_cu"), ("chunk", 65, "chunk"), ("split_steps", -2, "split_steps"),
    ("heavy_waves", 5, "heavy_waves"), ("heavy_workgroups_per_cu", 17, "heavy_workgroups_per_cu")])
def test_launch_params_are_checked(field, value, msg):
    L = binding.load()
    H = np.zeros((6, 32), dtype=np.uint8)
    p = binding.LaunchParams()
    setattr(p, field, value)
    rc = L.orbg_decode_ex(H.ctypes.data_as(ctypes.c_void_p), None, 32, 26, 100, 4, None, None, None, None,
                          ctypes.byref(p), None)
    assert rc == -1 and msg in L.orbg_last_error().decode()


def test_mixed_rejects_unregistered_and_bad_counts():
    L = binding.load()
    ids = (ctypes.c_int * 1)(12345)
    p = ctypes.c_void_p(8)
    rc = L.orbg_decode_mixed(ids, 1, p, p, p, 1000, 1, 100, p, 1000, p, p, None, None)
    assert rc == -1 and "not registered" in L.orbg_last_error().decode()
    rc = L.orbg_decode_mixed(ids, 9, None, None, None, 0, 0, 100, None, 0, None, None, None, None)
    assert rc == -1 and "ncodes" in L.orbg_last_error().decode()
    assert L.orbg_code_release(777) == -1


@pytest.mark.parametrize("llr_len,cw_len", [(-1, 100), (100, -5), (-1, -1)])
def test_mixed_rejects_negative_buffer_lengths(llr_len, cw_len):
    """The mixed decode bounds every row by the two buffer lengths it is given;
    negative lengths are rejected before anything is looked up or launched."""
    L = binding.load()
    ids = (ctypes.c_int * 1)(0)
    p = ctypes.c_void_p(8)
    rc = L.orbg_decode_mixed(ids, 1, p, p, p, llr_len, 1, 100, p, cw_len, p, p, None, None)
    assert rc == -1 and "must not be negative" in L.orbg_last_error().decode()


def _cpu(shape, dtype):
    import torch
    return torch.zeros(shape, dtype=dtype)


@pytest.mark.parametrize("case,msg", [
    ("block_code_dtype", "block_code must be torch.uint8"),
    ("row_offset_dtype", "row_offset must be torch.int64"),
    ("row_offset_len", "row_offset has shape"),
    ("llr_dtype", "llr must be torch.float32"),
    ("llr_rank", "llr must have 1 dimension"),
    ("codeword_dtype", "codeword must be torch.uint8"),
    ("queries_dtype", "queries must be torch.int64"),
    ("abandoned_len", "abandoned has shape"),
    ("host_tensors", "must be on a CUDA device"),
])
def test_binding_mixed_rejects_bad_tensors(case, msg):
    """The binding checks dtype, rank, shape, contiguity and device of every tensor
    (ValueError, independent of python -O) before it calls the library."""
    import torch
    N = 4
    t = dict(block_code=_cpu(N, torch.uint8), row_offset=_cpu(N, torch.int64), llr=_cpu(64, torch.float32),
             codeword=_cpu(64, torch.uint8), queries=_cpu(N, torch.int64), abandoned=_cpu(N, torch.uint8))
    field, what = case.rsplit("_", 1) if case != "host_tensors" else ("", "")
    if what == "dtype":
        t[field] = t[field].to(torch.int32 if t[field].dtype != torch.int32 else torch.int64)
    elif what == "len":
        t[field] = t[field][:N - 1]
    elif what == "rank":
        t[field] = t[field].reshape(8, 8)
    with pytest.raises(ValueError, match=msg):
        binding.orbg_decode_mixed([0], t["block_code"], t["row_offset"], t["llr"], 100, t["codeword"], t["queries"],
                                  t["abandoned"])


@pytest.mark.parametrize("case,msg", [
    ("llr_dtype", "llr must be torch.float32"), ("llr_width", r"llr has shape \(4, 31\), expected \(4, 32\)"),
    ("llr_rank", "llr must be a 2-D"), ("host", "must be on a CUDA device")])
def test_binding_decode_rejects_bad_tensors(case, msg):
    import torch
    H = np.zeros((6, 32), dtype=np.uint8)
    llr = _cpu((4, 32), torch.float32)
    if case == "llr_dtype":
        llr = llr.double()
    elif case == "llr_width":
        llr = _cpu((4, 31), torch.float32)
    elif case == "llr_rank":
        llr = _cpu(128, torch.float32)
    with pytest.raises(ValueError, match=msg):
        binding.orbg_decode(H, llr, 100)


@pytest.mark.parametrize("n,k,budget,bufs,msg", [
    (0, 0, 10, True, "n = 0"),
    (100, 30, 10, True, "n - k = 70"),
    (32, 26, 0, True, "budget = 0"),
    (32, 26, 5 * 10 ** 6 + 1, True, "budget = 5000001"),
    (600, 590, (1 << 22) + 1, True, "above 2^22"),
    (32, 26, 100, False, "device buffer is NULL"),
])
def test_1line_argument_errors(n, k, budget, bufs, msg):
    L = binding.load()
    m = max(n - k, 1)
    H = np.zeros((m, max(n, 1)), dtype=np.uint8)
    p = ctypes.c_void_p(8) if bufs else None
    rc = L.orbg_decode_1line(H.ctypes.data_as(ctypes.c_void_p), p, n, k, budget, 4, p, p, p, None, None, None)
    assert rc == -1 and msg in L.orbg_last_error().decode()


@pytest.mark.parametrize("n,budget,j0,count,msg", [
    (0, 100, 0, 10, "n = 0"),
    (32, 0, 0, 10, "budget"),
    (8, 300, 0, 10, "budget"),            # more than 2^n patterns
    (32, 100, 0, 101, "above the budget"),
    (32, 100, -2, 10, "j0 = -2"),
    (32, 100, 1 << 20, 10, "j0 = 1048576"),
])
def test_1line_export_argument_errors(n, budget, j0, count, msg):
    L = binding.load()
    out = np.zeros((max(count, 1), 16), dtype=np.uint8)
    jm = ctypes.c_int(0)
    rc = L.orbg_schedule_export_1line(n, budget, j0, count, out.ctypes.data_as(ctypes.c_void_p), ctypes.byref(jm),
                                      None)
    assert rc == -1 and msg in L.orbg_last_error().decode()


@pytest.mark.parametrize("n,k,budget,seg,jdiv,bufs,msg", [
    (0, 0, 10, 2, 0, True, "n = 0"),
    (513, 500, 10, 2, 0, True, "n = 513"),
    (100, 30, 10, 2, 0, True, "n - k = 70"),
    (32, 26, 10, 0, 0, True, "segments = 0"),
    (32, 26, 10, 5, 0, True, "segments = 5"),
    (32, 26, 10, 2, 2, True, "jdiv = 2"),
    (32, 26, 0, 2, 0, True, "budget = 0"),
    (32, 26, 5 * 10 ** 6 + 1, 2, 0, True, "budget = 5000001"),
    (32, 26, 100, 2, 0, False, "device buffer is NULL"),
])
def test_mline_argument_errors(n, k, budget, seg, jdiv, bufs, msg):
    L = binding.load()
    m = max(n - k, 1)
    H = np.zeros((m, max(n, 1)), dtype=np.uint8)
    p = ctypes.c_void_p(8) if bufs else None
    rc = L.orbg_decode_mline(H.ctypes.data_as(ctypes.c_void_p), p, n, k, budget, 4, seg, jdiv, p, p, p, None, None)
    assert rc == -1 and msg in L.orbg_last_error().decode()


@pytest.mark.parametrize("case,msg", [
    ("negative_batch", "batch = -1"),
    ("no_output", "no output"),
    ("no_input", "device buffer is NULL"),
    ("negative_rows", "llr_rows = -3"),
    ("pin0", "pin0 = 2"),
])
def test_mlp_infer_argument_errors(case, msg):
    """The fused inference entry point's checks (no device work is reached)."""
    L = binding.load()
    p = ctypes.c_void_p(8)
    args = dict(w=p, wb=p, llr=p, rows=4, ids=None, x=None, batch=4, logits=p, order=None, pin0=0)
    if case == "negative_batch":
        args["batch"] = -1
    elif case == "no_output":
        args["logits"] = None
    elif case == "no_input":
        args["llr"] = None
    elif case == "negative_rows":
        args["rows"] = -3
    elif case == "pin0":
        args["pin0"] = 2
    rc = L.orbg_mlp_infer(args["w"], args["wb"], args["llr"], args["rows"], args["ids"], args["x"], args["batch"],
                          args["logits"], args["order"], args["pin0"], None)
    assert rc == -1 and msg in L.orbg_last_error().decode()
