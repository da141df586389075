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
    rc = L.orbg_decode_mixed(ids, 1, ctypes.c_void_p(8), ctypes.c_void_p(8), ctypes.c_void_p(8), 1, 100,
                             ctypes.c_void_p(8), ctypes.c_void_p(8), ctypes.c_void_p(8), None, None)
    assert rc == -1 and "not registered" in L.orbg_last_error().decode()
    rc = L.orbg_decode_mixed(ids, 9, None, None, None, 0, 100, None, None, None, None, None)
    assert rc == -1 and "ncodes" in L.orbg_last_error().decode()
    assert L.orbg_code_release(777) == -1


@pytest.mark.parametrize("n,k,budget,bufs,msg", [
    (0, 0, 10, True, "n = 0"),
    (100, 30, 10, True, "n - k = 70"),
    (32, 26, 0, True, "budget = 0"),
    (32, 26, (1 << 22) + 1, True, "budget"),
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
    (257, 240, 10, 2, 0, True, "n = 257"),
    (100, 30, 10, 2, 0, True, "n - k = 70"),
    (32, 26, 10, 0, 0, True, "segments = 0"),
    (32, 26, 10, 5, 0, True, "segments = 5"),
    (32, 26, 10, 2, 2, True, "jdiv = 2"),
    (32, 26, 0, 2, 0, True, "budget = 0"),
    (32, 26, (1 << 20) + 1, 2, 0, True, "budget = 1048577"),
    (32, 26, 100, 2, 0, False, "device buffer is NULL"),
])
def test_mline_argument_errors(n, k, budget, seg, jdiv, bufs, msg):
    L = binding.load()
    m = max(n - k, 1)
    H = np.zeros((m, max(n, 1)), dtype=np.uint8)
    p = ctypes.c_void_p(8) if bufs else None
    rc = L.orbg_decode_mline(H.ctypes.data_as(ctypes.c_void_p), p, n, k, budget, 4, seg, jdiv, p, p, p, None, None)
    assert rc == -1 and msg in L.orbg_last_error().decode()
