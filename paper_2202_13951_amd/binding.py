"""ctypes binding of liborbgrand (argument marshalling only).

Every computation happens in the HIP library; torch supplies device memory and
the current stream.  Importing this module never falls back to anything: if the
library is missing, load() raises.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liborbgrand.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "orbgrand.h")

ORBG_OK = 0
ORBG_NOALLOC_BATCH_MAX = 262144     # largest batch of orbg_decode_mixed_noalloc
_lib = None


class LaunchParams(ctypes.Structure):
    """orbg_launch_params: 0 fields take the library defaults (split_steps: -1)."""
    _fields_ = [("workgroups_per_cu", ctypes.c_int), ("chunk", ctypes.c_int), ("split_steps", ctypes.c_int),
                ("heavy_waves", ctypes.c_int), ("heavy_workgroups_per_cu", ctypes.c_int),
                ("one_block_per_workgroup", ctypes.c_int)]

    def __init__(self, workgroups_per_cu=0, chunk=0, split_steps=-1, heavy_waves=0, heavy_workgroups_per_cu=0,
                 one_block_per_workgroup=0):
        super().__init__(workgroups_per_cu, chunk, split_steps, heavy_waves, heavy_workgroups_per_cu,
                         one_block_per_workgroup)

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class OrbgError(RuntimeError):
    def __init__(self, fn: str, code: int, msg: str):
        super().__init__(f"{fn} returned {code}: {msg}")
        self.code = code


def load():
    """Load liborbgrand.so (built in-tree by build.py); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"liborbgrand.so is not built ({LIB_PATH}); run __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, u64, i64, ci = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int
    L.orbg_decode.argtypes = [vp, vp, ci, ci, u64, i64, vp, vp, vp, vp]
    L.orbg_decode.restype = ci
    L.orbg_decode_ordered.argtypes = [vp, vp, ci, ci, u64, i64, vp, vp, vp, vp, vp]
    L.orbg_decode_ordered.restype = ci
    L.orbg_decode_ex.argtypes = [vp, vp, ci, ci, u64, i64, vp, vp, vp, vp, vp, vp]
    L.orbg_decode_ex.restype = ci
    L.orbg_code_register.argtypes = [vp, ci, ci, ctypes.POINTER(ci)]
    L.orbg_code_register.restype = ci
    L.orbg_code_release.argtypes = [ci]
    L.orbg_code_release.restype = ci
    L.orbg_decode_mixed.argtypes = [vp, ci, vp, vp, vp, i64, i64, u64, vp, i64, vp, vp, vp, vp]
    L.orbg_decode_mixed.restype = ci
    L.orbg_decode_mixed_noalloc.argtypes = [vp, ci, vp, vp, vp, i64, i64, u64, vp, i64, vp, vp, vp, vp]
    L.orbg_decode_mixed_noalloc.restype = ci
    L.orbg_mlp_workspace_bytes.argtypes = [i64]
    L.orbg_mlp_workspace_bytes.restype = i64
    L.orbg_mlp_features.argtypes = [vp, ci, i64, vp, vp]
    L.orbg_mlp_features.restype = ci
    L.orbg_mlp_prepare.argtypes = [vp, vp, vp, vp]
    L.orbg_mlp_prepare.restype = ci
    L.orbg_mlp_forward.argtypes = [vp, vp, vp, i64, vp, vp, i64, vp]
    L.orbg_mlp_forward.restype = ci
    L.orbg_mlp_backward.argtypes = [vp, vp, vp, vp, vp, i64, vp, vp, vp, i64, vp]
    L.orbg_mlp_backward.restype = ci
    L.orbg_mlp_adam.argtypes = [vp, vp, vp, vp, ctypes.c_float, ci, vp, vp, vp]
    L.orbg_mlp_adam.restype = ci
    L.orbg_mlp_order.argtypes = [vp, i64, vp, vp]
    L.orbg_mlp_order.restype = ci
    L.orbg_mlp_infer.argtypes = [vp, vp, vp, i64, vp, vp, i64, vp, vp, ci, vp]
    L.orbg_mlp_infer.restype = ci
    L.orbg_schedule_export.argtypes = [ci, u64, vp, vp]
    L.orbg_schedule_export.restype = ci
    L.orbg_decode_1line.argtypes = [vp, vp, ci, ci, u64, i64, vp, vp, vp, vp, vp, vp]
    L.orbg_decode_1line.restype = ci
    L.orbg_schedule_export_1line.argtypes = [ci, u64, ci, u64, vp, ctypes.POINTER(ci), vp]
    L.orbg_schedule_export_1line.restype = ci
    L.orbg_decode_mline.argtypes = [vp, vp, ci, ci, u64, i64, ci, ci, vp, vp, vp, vp, vp]
    L.orbg_decode_mline.restype = ci
    L.orbg_learned_workspace_bytes.argtypes = [i64]
    L.orbg_learned_workspace_bytes.restype = i64
    L.orbg_decode_learned.argtypes = [vp, vp, ci, ci, u64, i64, vp, vp, vp, i64, vp, vp, vp, vp,
                                      ctypes.POINTER(i64), vp, vp]
    L.orbg_decode_learned.restype = ci
    L.orbg_last_error.argtypes = []
    L.orbg_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def header_symbols() -> list[str]:
    """Function names the public header declares."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(orbg_[a-z_0-9]+)\s*\(", txt)))


def _check(fn: str, rc: int):
    if rc != ORBG_OK:
        raise OrbgError(fn, rc, load().orbg_last_error().decode())


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _host_H(H) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(H), dtype=np.uint8)


def _need(cond: bool, msg):
    """Argument check that survives python -O (raises ValueError).  msg: the
    message, or a function that makes it (formatted only when the check fails,
    so a passing check costs no string formatting)."""
    if not cond:
        raise ValueError(msg() if callable(msg) else msg)


def _tensor_spec(t, name: str, dtype, shape=None, ndim=None):
    """t must be a contiguous torch tensor of this dtype (and shape / rank)."""
    import torch
    _need(isinstance(t, torch.Tensor), lambda: f"{name} must be a torch tensor")
    _need(t.dtype == dtype, lambda: f"{name} must be {dtype} (got {t.dtype})")
    if ndim is not None:
        _need(t.dim() == ndim, lambda: f"{name} must have {ndim} dimension(s)")
    if shape is not None:
        _need(tuple(t.shape) == tuple(shape),
              lambda: f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    _need(t.is_contiguous(), lambda: f"{name} must be contiguous")


def _on_device(t, name: str, device=None):
    _need(t.is_cuda, lambda: f"{name} must be on a CUDA device")
    if device is not None:
        _need(t.device == device, lambda: f"{name} is on {t.device}, expected {device}")


def _dev_tensor(t, name: str, dtype, shape=None, device=None, ndim=None):
    """t must be a contiguous CUDA tensor of this dtype (and shape / device / rank)."""
    _tensor_spec(t, name, dtype, shape, ndim)
    _on_device(t, name, device)


def _llr_rows(llr, n: int):
    """llr must be a CUDA float32 [N, n] tensor; returns N."""
    import torch
    _need(isinstance(llr, torch.Tensor) and llr.dim() == 2, "llr must be a 2-D torch tensor")
    _dev_tensor(llr, "llr", torch.float32, shape=(llr.shape[0], n))
    return llr.shape[0]


def _outputs(N, n, device, out):
    import torch
    if out is not None:
        _need(len(out) == 3, "out must be (codeword, queries, abandoned)")
        cw, q, ab = out
        _dev_tensor(cw, "codeword", torch.uint8, (N, n), device)
        _dev_tensor(q, "queries", torch.int64, (N,), device)
        _dev_tensor(ab, "abandoned", torch.uint8, (N,), device)
        return out
    return (torch.empty((N, n), dtype=torch.uint8, device=device),
            torch.empty((N,), dtype=torch.int64, device=device),
            torch.empty((N,), dtype=torch.uint8, device=device))


def orbg_decode(H, llr, budget: int, out=None, stream=None):
    """Plain basic-ORBGRAND decode.  H: host (n-k) x n 0/1 array; llr: CUDA float32
    tensor [N, n].  Returns (codeword u8 [N, n], queries int64 [N], abandoned u8 [N])
    on the same device (queries holds the u64 counts)."""
    Hn = _host_H(H)
    m, n = Hn.shape
    N = _llr_rows(llr, n)
    cw, q, ab = _outputs(N, n, llr.device, out)
    rc = load().orbg_decode(Hn.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(llr.data_ptr()), n, n - m,
                            int(budget), N, ctypes.c_void_p(cw.data_ptr()), ctypes.c_void_p(q.data_ptr()),
                            ctypes.c_void_p(ab.data_ptr()), _stream_ptr(stream))
    _check("orbg_decode", rc)
    return cw, q, ab


def orbg_decode_ordered(H, llr, budget: int, order, out=None, stream=None):
    """Decode with a per-block order of the first 64 batches; order: CUDA uint8 [N, 64]."""
    import torch
    Hn = _host_H(H)
    m, n = Hn.shape
    N = _llr_rows(llr, n)
    _dev_tensor(order, "order", torch.uint8, (N, 64), llr.device)
    cw, q, ab = _outputs(N, n, llr.device, out)
    rc = load().orbg_decode_ordered(Hn.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(llr.data_ptr()), n,
                                    n - m, int(budget), N, ctypes.c_void_p(order.data_ptr()),
                                    ctypes.c_void_p(cw.data_ptr()), ctypes.c_void_p(q.data_ptr()),
                                    ctypes.c_void_p(ab.data_ptr()), _stream_ptr(stream))
    _check("orbg_decode_ordered", rc)
    return cw, q, ab


def _params_ptr(params):
    return ctypes.byref(params) if params is not None else None


def orbg_decode_ex(H, llr, budget: int, order=None, params: LaunchParams | None = None, out=None, stream=None):
    """orbg_decode (order None) or orbg_decode_ordered with an explicit launch shape."""
    import torch
    Hn = _host_H(H)
    m, n = Hn.shape
    N = _llr_rows(llr, n)
    if order is not None:
        _dev_tensor(order, "order", torch.uint8, (N, 64), llr.device)
    cw, q, ab = _outputs(N, n, llr.device, out)
    rc = load().orbg_decode_ex(Hn.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(llr.data_ptr()), n, n - m,
                               int(budget), N, ctypes.c_void_p(order.data_ptr()) if order is not None else None,
                               ctypes.c_void_p(cw.data_ptr()), ctypes.c_void_p(q.data_ptr()),
                               ctypes.c_void_p(ab.data_ptr()), _params_ptr(params), _stream_ptr(stream))
    _check("orbg_decode_ex", rc)
    return cw, q, ab


def orbg_decode_1line(H, llr, budget: int, j0=True, params: LaunchParams | None = None, out=None, stream=None):
    """1-line ORBGRAND decode.  j0: True (allocate), a CUDA int32 [N] tensor, or None/False
    (offsets not reported).  Returns (codeword, queries, abandoned, j0 or None)."""
    import torch
    Hn = _host_H(H)
    m, n = Hn.shape
    N = _llr_rows(llr, n)
    cw, q, ab = _outputs(N, n, llr.device, out)
    if j0 is True:
        j0 = torch.empty((N,), dtype=torch.int32, device=llr.device)
    elif j0 is False:
        j0 = None
    if j0 is not None:
        _dev_tensor(j0, "j0", torch.int32, (N,), llr.device)
    rc = load().orbg_decode_1line(Hn.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(llr.data_ptr()), n, n - m,
                                  int(budget), N, ctypes.c_void_p(cw.data_ptr()), ctypes.c_void_p(q.data_ptr()),
                                  ctypes.c_void_p(ab.data_ptr()), _p(j0), _params_ptr(params),
                                  _stream_ptr(stream))
    _check("orbg_decode_1line", rc)
    return cw, q, ab, j0


def orbg_decode_mline(H, llr, budget: int, segments: int, jdiv: bool = False, segments_out=True, out=None,
                      stream=None):
    """Full m-line ORBGRAND decode.  segments_out: True (allocate), a CUDA int32 [N] tensor,
    or None/False.  Returns (codeword, queries, abandoned, segments_out or None)."""
    import torch
    Hn = _host_H(H)
    m, n = Hn.shape
    N = _llr_rows(llr, n)
    cw, q, ab = _outputs(N, n, llr.device, out)
    if segments_out is True:
        segments_out = torch.empty((N,), dtype=torch.int32, device=llr.device)
    elif segments_out is False:
        segments_out = None
    if segments_out is not None:
        _dev_tensor(segments_out, "segments_out", torch.int32, (N,), llr.device)
    rc = load().orbg_decode_mline(Hn.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(llr.data_ptr()), n, n - m,
                                  int(budget), N, int(segments), int(bool(jdiv)), ctypes.c_void_p(cw.data_ptr()),
                                  ctypes.c_void_p(q.data_ptr()), ctypes.c_void_p(ab.data_ptr()), _p(segments_out),
                                  _stream_ptr(stream))
    _check("orbg_decode_mline", rc)
    return cw, q, ab, segments_out


def orbg_code_register(H) -> int:
    """Registers a parity-check matrix for mixed decodes; returns its id."""
    Hn = _host_H(H)
    m, n = Hn.shape
    cid = ctypes.c_int(-1)
    rc = load().orbg_code_register(Hn.ctypes.data_as(ctypes.c_void_p), n, n - m, ctypes.byref(cid))
    _check("orbg_code_register", rc)
    return cid.value


def orbg_code_release(code_id: int) -> None:
    _check("orbg_code_release", load().orbg_code_release(int(code_id)))


def orbg_decode_mixed(code_ids, block_code, row_offset, llr, budget: int, codeword, queries, abandoned,
                      params: LaunchParams | None = None, stream=None):
    """Mixed-code decode.  code_ids: registered ids; block_code: CUDA uint8 [N] index into
    code_ids; row_offset: CUDA int64 [N] element offset of each row in llr (float32, 1-D) and
    codeword (uint8, 1-D); queries: CUDA int64 [N]; abandoned: CUDA uint8 [N].  The library
    bounds every row by the lengths of llr and codeword (a row outside them reads zeros and
    its codeword stores are dropped)."""
    import torch
    ids = (ctypes.c_int * len(code_ids))(*[int(c) for c in code_ids])
    _tensor_spec(block_code, "block_code", torch.uint8, ndim=1)
    N = block_code.shape[0]
    spec = [(row_offset, "row_offset", torch.int64, (N,), None), (llr, "llr", torch.float32, None, 1),
            (codeword, "codeword", torch.uint8, None, 1), (queries, "queries", torch.int64, (N,), None),
            (abandoned, "abandoned", torch.uint8, (N,), None)]
    for t, name, dt, shape, nd in spec:
        _tensor_spec(t, name, dt, shape, nd)
    dev = block_code.device
    _on_device(block_code, "block_code")
    for t, name, *_ in spec:
        _on_device(t, name, dev)
    rc = load().orbg_decode_mixed(ids, len(code_ids), ctypes.c_void_p(block_code.data_ptr()),
                                  ctypes.c_void_p(row_offset.data_ptr()), ctypes.c_void_p(llr.data_ptr()),
                                  llr.numel(), N, int(budget), ctypes.c_void_p(codeword.data_ptr()),
                                  codeword.numel(), ctypes.c_void_p(queries.data_ptr()),
                                  ctypes.c_void_p(abandoned.data_ptr()), _params_ptr(params), _stream_ptr(stream))
    _check("orbg_decode_mixed", rc)


def orbg_decode_mixed_noalloc(code_ids, block_code, row_offset, llr, budget: int, codeword, queries, abandoned,
                              params: LaunchParams | None = None, stream=None):
    """orbg_decode_mixed without any device allocation (batch <= 262144; the codes'
    schedules for this budget must exist; calls overlapping on one device race)."""
    import torch
    ids = (ctypes.c_int * len(code_ids))(*[int(c) for c in code_ids])
    _tensor_spec(block_code, "block_code", torch.uint8, ndim=1)
    N = block_code.shape[0]
    spec = [(row_offset, "row_offset", torch.int64, (N,), None), (llr, "llr", torch.float32, None, 1),
            (codeword, "codeword", torch.uint8, None, 1), (queries, "queries", torch.int64, (N,), None),
            (abandoned, "abandoned", torch.uint8, (N,), None)]
    for t, name, dt, shape, nd in spec:
        _tensor_spec(t, name, dt, shape, nd)
    _on_device(block_code, "block_code")
    for t, name, *_ in spec:
        _on_device(t, name, block_code.device)
    rc = load().orbg_decode_mixed_noalloc(ids, len(code_ids), ctypes.c_void_p(block_code.data_ptr()),
                                          ctypes.c_void_p(row_offset.data_ptr()), ctypes.c_void_p(llr.data_ptr()),
                                          llr.numel(), N, int(budget), ctypes.c_void_p(codeword.data_ptr()),
                                          codeword.numel(), ctypes.c_void_p(queries.data_ptr()),
                                          ctypes.c_void_p(abandoned.data_ptr()), _params_ptr(params),
                                          _stream_ptr(stream))
    _check("orbg_decode_mixed_noalloc", rc)


def orbg_schedule_export(n: int, count: int, stream=None) -> np.ndarray:
    """The first `count` schedule entries for length n: uint8 [count, 16] of ranks."""
    out = np.zeros((count, 16), dtype=np.uint8)
    rc = load().orbg_schedule_export(int(n), int(count), out.ctypes.data_as(ctypes.c_void_p),
                                     _stream_ptr(stream))
    _check("orbg_schedule_export", rc)
    return out


def orbg_schedule_export_1line(n: int, budget: int, j0: int, count: int, stream=None):
    """The first `count` entries of the 1-line schedule of offset j0 used with this budget:
    (uint8 [count, 16] of ranks, j0max)."""
    out = np.zeros((max(count, 1), 16), dtype=np.uint8)
    jm = ctypes.c_int(-2)
    rc = load().orbg_schedule_export_1line(int(n), int(budget), int(j0), int(count),
                                           out.ctypes.data_as(ctypes.c_void_p), ctypes.byref(jm),
                                           _stream_ptr(stream))
    _check("orbg_schedule_export_1line", rc)
    return out[:count], jm.value


# ---------------------------------------------------------------------------
# learned batch-order proposal (tensors: torch CUDA, contiguous)
# ---------------------------------------------------------------------------
MLP_PARAMS = 115264
MLP_TPARAMS = 114688


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def orbg_mlp_workspace_bytes(batch: int) -> int:
    return int(load().orbg_mlp_workspace_bytes(int(batch)))


def orbg_mlp_features(llr, x, stream=None):
    """x (int16 [N,128], BF16 bits) <- sorted |llr| / 8 of llr (float32 [N,128])."""
    N, n = llr.shape
    _check("orbg_mlp_features", load().orbg_mlp_features(_p(llr), n, N, _p(x), _stream_ptr(stream)))


def orbg_mlp_prepare(w, wb, wt, stream=None):
    _check("orbg_mlp_prepare", load().orbg_mlp_prepare(_p(w), _p(wb), _p(wt), _stream_ptr(stream)))


def orbg_mlp_forward(w, wb, x, logits, workspace, stream=None):
    _check("orbg_mlp_forward", load().orbg_mlp_forward(_p(w), _p(wb), _p(x), x.shape[0], _p(logits), _p(workspace),
                                                       workspace.numel(), _stream_ptr(stream)))


def orbg_mlp_backward(w, wb, wt, x, labels, grads, loss, workspace, stream=None):
    _check("orbg_mlp_backward", load().orbg_mlp_backward(_p(w), _p(wb), _p(wt), _p(x), _p(labels), x.shape[0],
                                                         _p(grads), _p(loss), _p(workspace), workspace.numel(),
                                                         _stream_ptr(stream)))


def orbg_mlp_adam(w, m, v, grads, lr: float, step: int, wb, wt, stream=None):
    _check("orbg_mlp_adam", load().orbg_mlp_adam(_p(w), _p(m), _p(v), _p(grads), float(lr), int(step), _p(wb),
                                                 _p(wt), _stream_ptr(stream)))


def orbg_mlp_order(logits, order, stream=None):
    _check("orbg_mlp_order", load().orbg_mlp_order(_p(logits), logits.shape[0], _p(order), _stream_ptr(stream)))


def orbg_mlp_infer(w, wb, llr=None, ids=None, x=None, logits=None, order=None, pin0: bool = False, stream=None):
    """Fused inference: features of llr rows (row ids[b], or b) or the given
    features x, the three layers, then logits [N, 64] f32 and/or the batch order
    [N, 64] u8 (pass the output tensors to fill)."""
    import torch
    if (llr is None) == (x is None):
        raise ValueError("orbg_mlp_infer takes exactly one of llr and x")
    rows = 0
    if llr is not None:
        rows = _llr_rows(llr, 128)
        N = rows if ids is None else int(ids.numel())
        dev = llr.device
        if ids is not None:
            _dev_tensor(ids, "ids", torch.int64, (N,), dev)
    else:
        _dev_tensor(x, "x", torch.int16, (x.shape[0], 128), x.device)
        N, dev = x.shape[0], x.device
    if logits is None and order is None:
        raise ValueError("orbg_mlp_infer needs logits or order")
    if logits is not None:
        _dev_tensor(logits, "logits", torch.float32, (N, 64), dev)
    if order is not None:
        _dev_tensor(order, "order", torch.uint8, (N, 64), dev)
    _check("orbg_mlp_infer", load().orbg_mlp_infer(_p(w), _p(wb), _p(llr), rows, _p(ids), _p(x), N, _p(logits),
                                                   _p(order), int(bool(pin0)), _stream_ptr(stream)))
    return logits, order


def orbg_learned_workspace_bytes(batch: int) -> int:
    return int(load().orbg_learned_workspace_bytes(int(batch)))


def orbg_decode_learned(H, llr, budget: int, w, wb, workspace, out=None, order_out=None,
                        params: LaunchParams | None = None, stream=None):
    """Gated learned decode (n = 128): batch 0 for every block, the network and the
    ordered search only for the blocks batch 0 does not decide.  Returns
    (codeword, queries, abandoned, listed block count)."""
    import torch
    Hn = _host_H(H)
    m, n = Hn.shape
    N = _llr_rows(llr, n)
    cw, q, ab = _outputs(N, n, llr.device, out)
    _dev_tensor(w, "w", torch.float32, (MLP_PARAMS,), llr.device)
    _dev_tensor(wb, "wb", torch.int16, (MLP_PARAMS,), llr.device)
    _dev_tensor(workspace, "workspace", torch.uint8, device=llr.device, ndim=1)
    if order_out is not None:
        _dev_tensor(order_out, "order_out", torch.uint8, (N, 64), llr.device)
    rest = ctypes.c_int64(-1)
    rc = load().orbg_decode_learned(Hn.ctypes.data_as(ctypes.c_void_p), _p(llr), n, n - m, int(budget), N, _p(w),
                                    _p(wb), _p(workspace), workspace.numel(), _p(cw), _p(q), _p(ab), _p(order_out),
                                    ctypes.byref(rest), _params_ptr(params), _stream_ptr(stream))
    _check("orbg_decode_learned", rc)
    return cw, q, ab, rest.value
