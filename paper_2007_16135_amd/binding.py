"""Thin Python binding of libtwed (ctypes).  Argument marshalling only: every
step of the distance computation runs in the HIP library.

Tensors are PyTorch device tensors (PyTorch supplies device memory and the
current stream); the functions keep the C names of include/twed.h.  The
library must have been built (``python -m paper_2007_16135_amd.build``):
a missing library raises, there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libtwed.so")

TWED_OK, TWED_ERR_INVALID, TWED_ERR_UNSUPPORTED, TWED_ERR_WORKSPACE, TWED_ERR_DEVICE = range(5)
PRECISIONS = {"f64": 0, "f32": 1, "f32_acc64": 2, "auto": 3}
ALGOS = {"auto": 0, "wavefront": 1, "diagonal": 2}
EXPORTS = [
    "twed_params_default", "twed_pair_workspace_size", "twed_pair", "twed_pair_noalloc", "twed_pair_matrix",
    "twed_batch_workspace_size", "twed_batch", "twed_batch_max_short_length",
    "twed_batch_plan_create", "twed_batch_plan_run", "twed_batch_plan_destroy", "twed_batch_plan_stage_y",
    "twed_batch_plan_tune", "twed_batch_plan_config", "twed_tune_save", "twed_tune_load",
    "twed_status_string", "twed_last_error", "twed_stream_check", "twed_version",
    "twed_pair_tune", "twed_tune_clear", "twed_pair_config",
    "twed_pair_tile_workspace_size", "twed_pair_tile", "twed_pair_path_workspace_size", "twed_pair_path",
    "twed_dp_workspace_size", "twed_dp", "twed_dp_path_workspace_size", "twed_dp_path",
    "twed_embed_param_count", "twed_embed_max_length", "twed_embed_set_limits", "twed_embed_workspace_size",
    "twed_embed_forward",
    "twed_embed_loss_grad", "twed_embed_adamw", "twed_knn_index_storage_size", "twed_knn_index_create",
    "twed_knn_index_build_workspace_size", "twed_knn_index_build", "twed_knn_workspace_size", "twed_knn",
    "twed_knn_index_destroy", "twed_probe_valu",
]
EMBED_DIM = 128


class TwedParams(ctypes.Structure):
    _fields_ = [("nu", ctypes.c_double), ("lambda_", ctypes.c_double), ("p", ctypes.c_double),
                ("dim", ctypes.c_int32), ("precision", ctypes.c_int32), ("algo", ctypes.c_int32),
                ("strip_k", ctypes.c_int32), ("acc64_threshold", ctypes.c_int64)]


class TwedError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libtwed status {status}: {msg}")
        self.status = status


_lib = None
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i64p = ctypes.POINTER(ctypes.c_int64)
_pp = ctypes.POINTER(TwedParams)


def load_library(path: str = LIB_PATH):
    """Loads libtwed.so and declares its signatures (no GPU needed)."""
    global _lib
    if _lib is not None and path == LIB_PATH:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libtwed not built: {path} is missing "
                           "(run python -m paper_2007_16135_amd.build)")
    L = ctypes.CDLL(path)
    L.twed_params_default.argtypes = [_pp]
    L.twed_params_default.restype = None
    L.twed_pair_workspace_size.argtypes = [_i64, _i64, _pp]
    L.twed_pair_workspace_size.restype = ctypes.c_size_t
    L.twed_pair.argtypes = [_vp, _vp, _i64, _vp, _vp, _i64, _pp, _vp, _vp, ctypes.c_size_t, _vp]
    L.twed_pair.restype = ctypes.c_int
    L.twed_pair_noalloc.argtypes = [_vp, _vp, _i64, _vp, _vp, _i64, _pp, _vp, _vp]
    L.twed_pair_noalloc.restype = ctypes.c_int
    L.twed_pair_matrix.argtypes = [_vp, _vp, _i64, _vp, _vp, _i64, _pp, _vp, _vp, _vp, ctypes.c_size_t, _vp]
    L.twed_pair_matrix.restype = ctypes.c_int
    L.twed_batch_workspace_size.argtypes = [_i64p, _i64, _i64p, _i64, _pp]
    L.twed_batch_workspace_size.restype = ctypes.c_size_t
    L.twed_batch.argtypes = [_vp, _vp, _i64p, _i64, _vp, _vp, _i64p, _i64, _vp, _i64, _pp, _vp, _vp,
                             ctypes.c_size_t, _vp]
    L.twed_batch.restype = ctypes.c_int
    L.twed_batch_plan_create.argtypes = [_i64p, _i64, _i64p, _i64, _i64, _pp, _vp, ctypes.c_size_t,
                                         ctypes.POINTER(_vp)]
    L.twed_batch_plan_create.restype = ctypes.c_int
    L.twed_batch_plan_run.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
    L.twed_batch_plan_run.restype = ctypes.c_int
    L.twed_batch_plan_stage_y.argtypes = [_vp, _vp, _vp, _vp]
    L.twed_batch_plan_stage_y.restype = ctypes.c_int
    L.twed_batch_plan_destroy.argtypes = [_vp]
    L.twed_batch_plan_destroy.restype = None
    _i32p = ctypes.POINTER(ctypes.c_int32)
    L.twed_batch_plan_tune.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i32p, _i32p, _i32p]
    L.twed_batch_plan_tune.restype = ctypes.c_int
    L.twed_batch_plan_config.argtypes = [_vp, _i32p, _i32p, _i32p]
    L.twed_batch_plan_config.restype = ctypes.c_int
    L.twed_tune_save.argtypes = [ctypes.c_char_p]
    L.twed_tune_save.restype = ctypes.c_int
    L.twed_tune_load.argtypes = [ctypes.c_char_p]
    L.twed_tune_load.restype = ctypes.c_int
    L.twed_pair_tune.argtypes = [_vp, _vp, _i64, _vp, _vp, _i64, _pp, _vp, ctypes.c_size_t, _vp,
                                 ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
    L.twed_pair_tune.restype = ctypes.c_int
    L.twed_tune_clear.argtypes = []
    L.twed_pair_config.argtypes = [_i64, _i64, _pp, _i32p, _i32p, _i64p, _i64p]
    L.twed_pair_config.restype = ctypes.c_int
    L.twed_pair_tile_workspace_size.argtypes = [_i64, _i64, _pp]
    L.twed_pair_tile_workspace_size.restype = ctypes.c_size_t
    L.twed_pair_tile.argtypes = [_vp, _vp, _i64, _vp, _vp, _i64, _pp, _i64, _i64, _i64, _i64, _vp, _vp, _vp, _vp,
                                 _vp, _vp, ctypes.c_size_t, _vp]
    L.twed_pair_tile.restype = ctypes.c_int
    L.twed_pair_path_workspace_size.argtypes = [_i64, _i64, _pp, _i64]
    L.twed_pair_path_workspace_size.restype = ctypes.c_size_t
    L.twed_pair_path.argtypes = [_vp, _vp, _i64, _vp, _vp, _i64, _pp, _i64, _vp, _vp, _vp, _vp, ctypes.c_size_t,
                                 _vp]
    L.twed_pair_path.restype = ctypes.c_int
    L.twed_dp_workspace_size.argtypes = [ctypes.c_int32, _i64, _i64, _pp]
    L.twed_dp_workspace_size.restype = ctypes.c_size_t
    L.twed_dp.argtypes = [ctypes.c_int32, _vp, _i64, _vp, _i64, _pp, _vp, _vp, ctypes.c_size_t, _vp]
    L.twed_dp.restype = ctypes.c_int
    L.twed_dp_path_workspace_size.argtypes = [ctypes.c_int32, _i64, _i64, _pp, _i64]
    L.twed_dp_path_workspace_size.restype = ctypes.c_size_t
    L.twed_dp_path.argtypes = [ctypes.c_int32, _vp, _i64, _vp, _i64, _pp, _i64, _vp, _vp, _vp, _vp,
                               ctypes.c_size_t, _vp]
    L.twed_dp_path.restype = ctypes.c_int
    L.twed_tune_clear.restype = None
    L.twed_batch_max_short_length.argtypes = [ctypes.c_int32]
    L.twed_batch_max_short_length.restype = ctypes.c_int64
    L.twed_status_string.argtypes = [ctypes.c_int]
    L.twed_status_string.restype = ctypes.c_char_p
    L.twed_last_error.argtypes = []
    L.twed_last_error.restype = ctypes.c_char_p
    L.twed_stream_check.argtypes = [_vp]
    L.twed_stream_check.restype = ctypes.c_int
    L.twed_version.argtypes = []
    L.twed_version.restype = ctypes.c_char_p
    L.twed_probe_valu.argtypes = [ctypes.c_int32, _i64, _i64, _vp, ctypes.POINTER(ctypes.c_double), _vp]
    L.twed_probe_valu.restype = ctypes.c_int
    # embedding network and k-NN index (include/twed_knn.h)
    _sz = ctypes.c_size_t
    L.twed_embed_param_count.argtypes = []
    L.twed_embed_param_count.restype = _i64
    L.twed_embed_max_length.argtypes = []
    L.twed_embed_max_length.restype = _i64
    L.twed_embed_set_limits.argtypes = [_i64, _i64]
    L.twed_embed_set_limits.restype = None
    L.twed_embed_workspace_size.argtypes = [_i64p, _i64, _i64]
    L.twed_embed_workspace_size.restype = _sz
    L.twed_embed_forward.argtypes = [_vp, _vp, _i64p, _i64, _vp, _vp, _sz, _vp]
    L.twed_embed_forward.restype = ctypes.c_int
    L.twed_embed_loss_grad.argtypes = [_vp, _vp, _i64p, _i64, _vp, _vp, _i64, _vp, _vp, _vp, _vp, _sz, _vp]
    L.twed_embed_loss_grad.restype = ctypes.c_int
    L.twed_embed_adamw.argtypes = [_vp, _vp, _vp, _vp, _i64, ctypes.c_float, ctypes.c_float, _vp]
    L.twed_embed_adamw.restype = ctypes.c_int
    L.twed_knn_index_storage_size.argtypes = [_i64p, _i64, _pp]
    L.twed_knn_index_storage_size.restype = _sz
    L.twed_knn_index_create.argtypes = [_vp, _vp, _i64p, _i64, _vp, _pp, _vp, _sz, ctypes.POINTER(_vp)]
    L.twed_knn_index_create.restype = ctypes.c_int
    L.twed_knn_index_build_workspace_size.argtypes = [_vp]
    L.twed_knn_index_build_workspace_size.restype = _sz
    L.twed_knn_index_build.argtypes = [_vp, _vp, _sz, _vp]
    L.twed_knn_index_build.restype = ctypes.c_int
    L.twed_knn_workspace_size.argtypes = [_vp, _i64p, _i64, ctypes.c_int32, ctypes.c_int32]
    L.twed_knn_workspace_size.restype = _sz
    L.twed_knn.argtypes = [_vp, _vp, _vp, _i64p, _i64, ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp, _sz, _vp]
    L.twed_knn.restype = ctypes.c_int
    L.twed_knn_index_destroy.argtypes = [_vp]
    L.twed_knn_index_destroy.restype = None
    if path == LIB_PATH:
        _lib = L
    return L


def make_params(nu=1e-3, lam=1.0, p=1.0, dim=1, precision="f64", algo="auto", strip_k=0,
                acc64_threshold=0) -> TwedParams:
    prm = TwedParams()
    load_library().twed_params_default(ctypes.byref(prm))
    prm.nu, prm.lambda_, prm.p, prm.dim = float(nu), float(lam), float(p), int(dim)
    prm.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    prm.algo = ALGOS[algo] if isinstance(algo, str) else int(algo)
    prm.strip_k = int(strip_k)
    prm.acc64_threshold = int(acc64_threshold)
    return prm


def _check(status: int):
    if status != TWED_OK:
        L = load_library()
        raise TwedError(status, L.twed_last_error().decode() or L.twed_status_string(status).decode())


def _torch():
    import torch
    return torch


def _stream(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def input_dtype(precision):
    torch = _torch()
    return torch.float64 if precision in ("f64", 0) else torch.float32


def output_dtype(precision):
    torch = _torch()
    return torch.float32 if precision in ("f32", 1) else torch.float64


def _dev(t, dtype, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous")
    return t


def _workspace(nbytes, device, workspace=None):
    torch = _torch()
    nbytes = max(int(nbytes), 256)
    if workspace is not None and workspace.numel() >= nbytes:
        return workspace
    ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
    assert ws.data_ptr() % 256 == 0
    return ws


def twed_pair_workspace_size(nA, nB, prm: TwedParams) -> int:
    return load_library().twed_pair_workspace_size(int(nA), int(nB), ctypes.byref(prm))


def twed_pair(A, TA, B, TB, nu=1e-3, lam=1.0, p=1.0, precision="f64", algo="auto", strip_k=0,
              acc64_threshold=0, out=None, workspace=None, stream=None):
    """TWED of one pair of device series.  A: (nA, dim) or (nA,), TA: (nA,).
    Returns a one-element device tensor (float32 for "f32", float64 otherwise)."""
    torch = _torch()
    dt = input_dtype(precision)
    A2 = A if A.dim() == 2 else A.reshape(-1, 1)
    B2 = B if B.dim() == 2 else B.reshape(-1, 1)
    _dev(A2, dt, "A"); _dev(B2, dt, "B"); _dev(TA, dt, "TA"); _dev(TB, dt, "TB")
    nA, dim = A2.shape
    nB = B2.shape[0]
    if B2.shape[1] != dim or TA.numel() != nA or TB.numel() != nB:
        raise ValueError("shape mismatch")
    prm = make_params(nu, lam, p, dim, precision, algo, strip_k, acc64_threshold)
    L = load_library()
    need = L.twed_pair_workspace_size(nA, nB, ctypes.byref(prm))
    ws = _workspace(need, A2.device, workspace)
    if out is None:
        out = torch.empty(1, dtype=output_dtype(precision), device=A2.device)
    _check(L.twed_pair(A2.data_ptr(), TA.data_ptr(), nA, B2.data_ptr(), TB.data_ptr(), nB,
                       ctypes.byref(prm), out.data_ptr(), ws.data_ptr(), ws.numel(), _stream(stream)))
    return out


def twed_pair_noalloc(A, TA, B, TB, nu=1e-3, lam=1.0, p=1.0, precision="f64", algo="auto", strip_k=0,
                      acc64_threshold=0, out=None, stream=None):
    """twed_pair without a workspace: the library's fixed per-device scratch
    array (TWED_PAIR_NOALLOC_SCRATCH_BYTES) serves as one; calls that overlap
    on one GPU race.  `out` (one element, float32 for "f32", float64
    otherwise) is allocated here only when not given."""
    torch = _torch()
    A2, B2, nA, nB, dim = _pair_operands(A, TA, B, TB, precision)
    prm = make_params(nu, lam, p, dim, precision, algo, strip_k, acc64_threshold)
    if out is None:
        out = torch.empty(1, dtype=output_dtype(precision), device=A2.device)
    _check(load_library().twed_pair_noalloc(A2.data_ptr(), TA.data_ptr(), nA, B2.data_ptr(), TB.data_ptr(), nB,
                                            ctypes.byref(prm), out.data_ptr(), _stream(stream)))
    return out


def _pair_operands(A, TA, B, TB, precision):
    dt = input_dtype(precision)
    A2 = A if A.dim() == 2 else A.reshape(-1, 1)
    B2 = B if B.dim() == 2 else B.reshape(-1, 1)
    _dev(A2, dt, "A"); _dev(B2, dt, "B"); _dev(TA, dt, "TA"); _dev(TB, dt, "TB")
    nA, dim = A2.shape
    nB = B2.shape[0]
    if B2.shape[1] != dim or TA.numel() != nA or TB.numel() != nB:
        raise ValueError("shape mismatch")
    return A2, B2, nA, nB, dim


def _ptr(t):
    return None if t is None else t.data_ptr()


def twed_pair_tile(A, TA, B, TB, r0, r1, c0, c1, top=None, left=None, nu=1e-3, lam=1.0, p=1.0,
                   precision="f64", strip_k=0, bottom=True, right=True, workspace=None, stream=None):
    """Sweeps rows r0+1..r1, columns c0+1..c1 of the DP matrix of (A, B) from
    its top row and left column: float64 device tensors of (DP, X) cells,
    shapes (c1-c0+1, 2) and (r1-r0+1, 2), None for the pad row / column.
    Returns (corner, bottom, right): DP(r1, c1) as a one-element tensor and
    the (DP, X) cells of row r1 and column c1 (None where not asked for)."""
    torch = _torch()
    A2, B2, nA, nB, dim = _pair_operands(A, TA, B, TB, precision)
    for t, name, n in ((top, "top", c1 - c0 + 1), (left, "left", r1 - r0 + 1)):
        if t is not None:
            _dev(t, torch.float64, name)
            if tuple(t.shape) != (n, 2):
                raise ValueError(f"{name} must have shape ({n}, 2)")
    prm = make_params(nu, lam, p, dim, precision, "auto", strip_k)
    L = load_library()
    ws = _workspace(L.twed_pair_tile_workspace_size(int(r1 - r0), int(c1 - c0), ctypes.byref(prm)), A2.device,
                    workspace)
    dev = A2.device
    corner = torch.empty(1, dtype=torch.float64, device=dev)
    bot = torch.empty((c1 - c0 + 1, 2), dtype=torch.float64, device=dev) if bottom else None
    rig = torch.empty((r1 - r0 + 1, 2), dtype=torch.float64, device=dev) if right else None
    _check(L.twed_pair_tile(A2.data_ptr(), TA.data_ptr(), nA, B2.data_ptr(), TB.data_ptr(), nB,
                            ctypes.byref(prm), int(r0), int(r1), int(c0), int(c1), _ptr(top), _ptr(left),
                            _ptr(bot), _ptr(rig), corner.data_ptr(), ws.data_ptr(), ws.numel(), _stream(stream)))
    return corner, bot, rig


def twed_dp_workspace_size(kind, nA, nB, prm: TwedParams) -> int:
    k = DP_KINDS[kind] if isinstance(kind, str) else int(kind)
    return load_library().twed_dp_workspace_size(k, int(nA), int(nB), ctypes.byref(prm))


def twed_pair_path_workspace_size(nA, nB, prm: TwedParams, block=0) -> int:
    return load_library().twed_pair_path_workspace_size(int(nA), int(nB), ctypes.byref(prm), int(block))


def twed_pair_tile_workspace_size(rows, cols, prm: TwedParams) -> int:
    return load_library().twed_pair_tile_workspace_size(int(rows), int(cols), ctypes.byref(prm))


def twed_pair_path(A, TA, B, TB, nu=1e-3, lam=1.0, p=1.0, precision="f64", block=0, strip_k=0,
                   workspace=None, stream=None):
    """(distance, path): a one-element float64 tensor and an (L, 2) int64
    device tensor of the cells (i, j) of one optimal alignment path from
    (0, 0) to (nA, nB).  Synchronises the stream."""
    torch = _torch()
    A2, B2, nA, nB, dim = _pair_operands(A, TA, B, TB, precision)
    prm = make_params(nu, lam, p, dim, precision, "auto", strip_k)
    L = load_library()
    ws = _workspace(L.twed_pair_path_workspace_size(nA, nB, ctypes.byref(prm), int(block)), A2.device, workspace)
    dev = A2.device
    out = torch.empty(1, dtype=torch.float64, device=dev)
    path = torch.empty((nA + nB + 1, 2), dtype=torch.int64, device=dev)
    n = torch.zeros(1, dtype=torch.int64, device=dev)
    _check(L.twed_pair_path(A2.data_ptr(), TA.data_ptr(), nA, B2.data_ptr(), TB.data_ptr(), nB,
                            ctypes.byref(prm), int(block), out.data_ptr(), path.data_ptr(), n.data_ptr(),
                            ws.data_ptr(), ws.numel(), _stream(stream)))
    return out, path[: int(n.item())]


DP_KINDS = {"dtw": 1, "edit": 2, "lcs": 3}


def _dp_operands(A, B, precision):
    dt = input_dtype(precision)
    A2 = A if A.dim() == 2 else A.reshape(-1, 1)
    B2 = B if B.dim() == 2 else B.reshape(-1, 1)
    _dev(A2, dt, "A"); _dev(B2, dt, "B")
    if A2.shape[1] != B2.shape[1]:
        raise ValueError("shape mismatch")
    return A2, B2, A2.shape[0], B2.shape[0], A2.shape[1]


def twed_dp(kind, A, B, p=1.0, precision="f64", strip_k=0, workspace=None, stream=None):
    """DTW distance ("dtw", Lp point distance), edit distance ("edit") or LCS
    length ("lcs") of two device series, as a one-element float64 tensor."""
    torch = _torch()
    k = DP_KINDS[kind] if isinstance(kind, str) else int(kind)
    A2, B2, nA, nB, dim = _dp_operands(A, B, precision)
    prm = make_params(0.0, 0.0, p, dim, precision, "auto", strip_k)
    L = load_library()
    ws = _workspace(L.twed_dp_workspace_size(k, nA, nB, ctypes.byref(prm)), A2.device, workspace)
    out = torch.empty(1, dtype=torch.float64, device=A2.device)
    _check(L.twed_dp(k, A2.data_ptr(), nA, B2.data_ptr(), nB, ctypes.byref(prm), out.data_ptr(), ws.data_ptr(),
                     ws.numel(), _stream(stream)))
    return out


def twed_dp_path(kind, A, B, p=1.0, precision="f64", block=0, strip_k=0, workspace=None, stream=None):
    """(value, path) for a twed_dp kind; path as twed_pair_path."""
    torch = _torch()
    k = DP_KINDS[kind] if isinstance(kind, str) else int(kind)
    A2, B2, nA, nB, dim = _dp_operands(A, B, precision)
    prm = make_params(0.0, 0.0, p, dim, precision, "auto", strip_k)
    L = load_library()
    ws = _workspace(L.twed_dp_path_workspace_size(k, nA, nB, ctypes.byref(prm), int(block)), A2.device, workspace)
    out = torch.empty(1, dtype=torch.float64, device=A2.device)
    path = torch.empty((nA + nB + 1, 2), dtype=torch.int64, device=A2.device)
    n = torch.zeros(1, dtype=torch.int64, device=A2.device)
    _check(L.twed_dp_path(k, A2.data_ptr(), nA, B2.data_ptr(), nB, ctypes.byref(prm), int(block), out.data_ptr(),
                          path.data_ptr(), n.data_ptr(), ws.data_ptr(), ws.numel(), _stream(stream)))
    return out, path[: int(n.item())]


def twed_pair_matrix(A, TA, B, TB, nu=1e-3, lam=1.0, p=1.0, precision="f64", algo="auto", strip_k=0,
                     stream=None):
    """Like twed_pair, and also returns every DP cell as an (nA+1, nB+1) tensor."""
    torch = _torch()
    dt = input_dtype(precision)
    A2 = A if A.dim() == 2 else A.reshape(-1, 1)
    B2 = B if B.dim() == 2 else B.reshape(-1, 1)
    _dev(A2, dt, "A"); _dev(B2, dt, "B"); _dev(TA, dt, "TA"); _dev(TB, dt, "TB")
    nA, dim = A2.shape
    nB = B2.shape[0]
    prm = make_params(nu, lam, p, dim, precision, algo, strip_k)
    L = load_library()
    ws = _workspace(L.twed_pair_workspace_size(nA, nB, ctypes.byref(prm)), A2.device)
    out = torch.empty(1, dtype=output_dtype(precision), device=A2.device)
    dp = torch.empty((nA + 1, nB + 1), dtype=output_dtype(precision), device=A2.device)
    _check(L.twed_pair_matrix(A2.data_ptr(), TA.data_ptr(), nA, B2.data_ptr(), TB.data_ptr(), nB,
                              ctypes.byref(prm), out.data_ptr(), dp.data_ptr(), ws.data_ptr(), ws.numel(),
                              _stream(stream)))
    return out, dp


def twed_pair_tune(A, TA, B, TB, nu=1e-3, lam=1.0, p=1.0, precision="f64", acc64_threshold=0, workspace=None,
                   stream=None):
    """Times the single-pair sweep configurations on this pair and caches the
    fastest for later twed_pair calls (strip_k=0).  Returns (strip_k, group)."""
    dt = input_dtype(precision)
    A2 = A if A.dim() == 2 else A.reshape(-1, 1)
    B2 = B if B.dim() == 2 else B.reshape(-1, 1)
    _dev(A2, dt, "A"); _dev(B2, dt, "B"); _dev(TA, dt, "TA"); _dev(TB, dt, "TB")
    nA, dim = A2.shape
    nB = B2.shape[0]
    prm = make_params(nu, lam, p, dim, precision, "auto", 0, acc64_threshold)
    L = load_library()
    ws = _workspace(L.twed_pair_workspace_size(nA, nB, ctypes.byref(prm)), A2.device, workspace)
    k, g = ctypes.c_int32(0), ctypes.c_int32(0)
    _check(L.twed_pair_tune(A2.data_ptr(), TA.data_ptr(), nA, B2.data_ptr(), TB.data_ptr(), nB, ctypes.byref(prm),
                            ws.data_ptr(), ws.numel(), _stream(stream), ctypes.byref(k), ctypes.byref(g)))
    return int(k.value), int(g.value)


def twed_pair_config(nA, nB, dim=1, nu=1e-3, lam=1.0, p=1.0, precision="f64", strip_k=0, acc64_threshold=0):
    """The strip layout twed_pair would sweep for these arguments, as a dict:
    strip_k (columns per lane), group (strips per workgroup), wide_strips (the
    strips of strip_k columns before those of strip_k - 1 in a two-width
    sweep, 0 for uniform strips) and strips.  Needs a current GPU; launches
    nothing."""
    prm = make_params(nu, lam, p, dim, precision, "auto", strip_k, acc64_threshold)
    L = load_library()
    k, g = ctypes.c_int32(0), ctypes.c_int32(0)
    w, n = ctypes.c_int64(0), ctypes.c_int64(0)
    _check(L.twed_pair_config(int(nA), int(nB), ctypes.byref(prm), ctypes.byref(k), ctypes.byref(g),
                              ctypes.byref(w), ctypes.byref(n)))
    return {"strip_k": int(k.value), "group": int(g.value), "wide_strips": int(w.value), "strips": int(n.value)}


def twed_tune_clear():
    load_library().twed_tune_clear()


def _offsets(off):
    off = np.ascontiguousarray(np.asarray(off, dtype=np.int64))
    return off, off.ctypes.data_as(_i64p)


def twed_batch_workspace_size(offX, offY, prm: TwedParams) -> int:
    offX, px = _offsets(offX)
    if offY is None:
        return load_library().twed_batch_workspace_size(px, len(offX) - 1, None, 0, ctypes.byref(prm))
    offY, py = _offsets(offY)
    return load_library().twed_batch_workspace_size(px, len(offX) - 1, py, len(offY) - 1, ctypes.byref(prm))


def twed_batch(X, TX, offX, Y=None, TY=None, offY=None, pairs=None, nu=1e-3, lam=1.0, p=1.0,
               precision="f32", D=None, workspace=None, stream=None):
    """Distances between packed collections (offsets are host int64 arrays).

    Y is None: symmetric nX x nX matrix (upper triangle swept).  pairs (device
    int64 (P, 2)) given: D[k] = TWED(X_i, Y_j) for the listed pairs.
    """
    torch = _torch()
    dt = input_dtype(precision)
    X2 = X if X.dim() == 2 else X.reshape(-1, 1)
    _dev(X2, dt, "X"); _dev(TX, dt, "TX")
    dim = X2.shape[1]
    offX, px = _offsets(offX)
    nX = len(offX) - 1
    if Y is None:
        Yp = TYp = None
        py, nY = None, nX
        offYa = None
    else:
        Y2 = Y if Y.dim() == 2 else Y.reshape(-1, 1)
        _dev(Y2, dt, "Y"); _dev(TY, dt, "TY")
        offYa, py = _offsets(offY)
        nY = len(offYa) - 1
        Yp, TYp = Y2.data_ptr(), TY.data_ptr()
    prm = make_params(nu, lam, p, dim, precision)
    L = load_library()
    need = L.twed_batch_workspace_size(px, nX, py, nY if Y is not None else 0, ctypes.byref(prm))
    ws = _workspace(need, X2.device, workspace)
    if pairs is not None:
        _dev(pairs, torch.int64, "pairs")
        nP = pairs.shape[0]
        if D is None:
            D = torch.empty(nP, dtype=output_dtype(precision), device=X2.device)
        if nP == 0:
            return D
        pp = pairs.data_ptr()
    else:
        nP = 0
        pp = None
        if D is None:
            D = torch.empty((nX, nY), dtype=output_dtype(precision), device=X2.device)
    _check(L.twed_batch(X2.data_ptr(), TX.data_ptr(), px, nX, Yp, TYp, py, nY, pp, nP,
                        ctypes.byref(prm), D.data_ptr(), ws.data_ptr(), ws.numel(), _stream(stream)))
    return D


class BatchPlan:
    """A batch of fixed shape planned once (offsets checked and uploaded, the
    workspace laid out) and run many times; run() only enqueues kernels, so
    it can be captured in a torch CUDA graph and replayed.  The plan keeps
    its workspace tensor alive; runs on one plan must not overlap."""

    def __init__(self, offX, offY=None, n_pairs=0, dim=1, nu=1e-3, lam=1.0, p=1.0, precision="f32",
                 device="cuda"):
        torch = _torch()
        offX, px = _offsets(offX)
        self.nX = len(offX) - 1
        self.sym = offY is None
        if self.sym:
            py, self.nY = None, self.nX
        else:
            offYa, py = _offsets(offY)
            self.nY = len(offYa) - 1
        self.n_pairs = int(n_pairs)
        self.precision = precision
        self.dim = dim
        self.prm = make_params(nu, lam, p, dim, precision)
        L = load_library()
        need = L.twed_batch_workspace_size(px, self.nX, py, 0 if self.sym else self.nY, ctypes.byref(self.prm))
        self.ws = _workspace(need, torch.device(device))
        h = _vp()
        self._h = None
        _check(L.twed_batch_plan_create(px, self.nX, py, 0 if self.sym else self.nY, self.n_pairs,
                                        ctypes.byref(self.prm), self.ws.data_ptr(), self.ws.numel(),
                                        ctypes.byref(h)))
        self._h = h

    def output(self):
        torch = _torch()
        shape = (self.n_pairs,) if self.n_pairs > 0 else (self.nX, self.nY)
        return torch.empty(shape, dtype=output_dtype(self.precision), device=self.ws.device)

    def stage_y(self, Y, TY, stream=None):
        """Packs the second collection once; run() without Y then reuses it."""
        dt = input_dtype(self.precision)
        Y2 = Y if Y.dim() == 2 else Y.reshape(-1, 1)
        _dev(Y2, dt, "Y"); _dev(TY, dt, "TY")
        if Y2.shape[1] != self.dim:
            raise ValueError("Y has a different dimension than the plan")
        _check(load_library().twed_batch_plan_stage_y(self._h, Y2.data_ptr(), TY.data_ptr(), _stream(stream)))

    def run(self, X, TX, Y=None, TY=None, pairs=None, D=None, stream=None):
        torch = _torch()
        dt = input_dtype(self.precision)
        X2 = X if X.dim() == 2 else X.reshape(-1, 1)
        _dev(X2, dt, "X"); _dev(TX, dt, "TX")
        if X2.shape[1] != self.dim:
            raise ValueError("X has a different dimension than the plan")
        Yp = TYp = None
        if Y is not None:
            Y2 = Y if Y.dim() == 2 else Y.reshape(-1, 1)
            _dev(Y2, dt, "Y"); _dev(TY, dt, "TY")
            Yp, TYp = Y2.data_ptr(), TY.data_ptr()
        pp = None
        if pairs is not None:
            _dev(pairs, torch.int64, "pairs")
            pp = pairs.data_ptr()
        if D is None:
            D = self.output()
        _check(load_library().twed_batch_plan_run(self._h, X2.data_ptr(), TX.data_ptr(), Yp, TYp, pp,
                                                  D.data_ptr(), _stream(stream)))
        return D

    def _args(self, X, TX, Y, TY, pairs):
        torch = _torch()
        dt = input_dtype(self.precision)
        X2 = X if X.dim() == 2 else X.reshape(-1, 1)
        _dev(X2, dt, "X"); _dev(TX, dt, "TX")
        if X2.shape[1] != self.dim:
            raise ValueError("X has a different dimension than the plan")
        Yp = TYp = None
        if Y is not None:
            Y2 = Y if Y.dim() == 2 else Y.reshape(-1, 1)
            _dev(Y2, dt, "Y"); _dev(TY, dt, "TY")
            Yp, TYp = Y2.data_ptr(), TY.data_ptr()
        pp = None
        if pairs is not None:
            _dev(pairs, torch.int64, "pairs")
            pp = pairs.data_ptr()
        return X2.data_ptr(), TX.data_ptr(), Yp, TYp, pp

    def tune(self, X, TX, Y=None, TY=None, pairs=None, D=None, stream=None):
        """Measures the batch configurations on these inputs (twed_batch_plan_tune);
        returns the chosen (chunk, waves_per_cu, lane_mode)."""
        if D is None:
            D = self.output()
        c, w, l = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(load_library().twed_batch_plan_tune(self._h, *self._args(X, TX, Y, TY, pairs), D.data_ptr(),
                                                   _stream(stream), ctypes.byref(c), ctypes.byref(w),
                                                   ctypes.byref(l)))
        return c.value, w.value, l.value

    def config(self):
        """(chunk, waves_per_cu, lane_mode) this plan runs with (0 / 0 / -1: the rules)."""
        c, w, l = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(load_library().twed_batch_plan_config(self._h, ctypes.byref(c), ctypes.byref(w), ctypes.byref(l)))
        return c.value, w.value, l.value

    def close(self):
        if self._h is not None:
            load_library().twed_batch_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def twed_tune_save(path) -> None:
    """Writes the tuning cache (single-pair and batch choices) to a file."""
    _check(load_library().twed_tune_save(os.fsencode(path)))


def twed_tune_load(path) -> None:
    """Merges a tuning cache file written by twed_tune_save."""
    _check(load_library().twed_tune_load(os.fsencode(path)))


def twed_stream_check(stream=None):
    _check(load_library().twed_stream_check(_stream(stream)))


def twed_version() -> str:
    return load_library().twed_version().decode()


def twed_host(A, TA, B, TB, nu=1e-3, lam=1.0, p=1.0, precision="f64", device="cuda", **kw) -> float:
    """Host-array convenience (the paper's managed call): copies numpy inputs
    to the device, runs twed_pair and returns the value as a Python float."""
    torch = _torch()
    dt = input_dtype(precision)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=device)
    A = np.asarray(A)
    B = np.asarray(B)
    out = twed_pair(t(A.reshape(len(A), -1)), t(TA), t(B.reshape(len(B), -1)), t(TB), nu, lam, p,
                    precision, **kw)
    return float(out.item())


# ---- embedding network and learned k-NN (include/twed_knn.h) -----------------------

def twed_embed_param_count() -> int:
    return int(load_library().twed_embed_param_count())


def twed_embed_max_length() -> int:
    return int(load_library().twed_embed_max_length())


def twed_embed_set_limits(chunk_rows: int = 0, score_bytes: int = 0) -> None:
    """Forward-pass chunk (samples) and k-NN score-chunk (bytes) limits;
    0 restores the defaults (twed_embed_set_limits in twed_knn.h)."""
    load_library().twed_embed_set_limits(int(chunk_rows), int(score_bytes))


def twed_embed_forward(params, X, off, emb=None, workspace=None, stream=None):
    """Embeddings (nSeries, 128) float32 of packed 1-D series X (float32
    device values) with host offsets `off`; params: the flat float32 vector."""
    torch = _torch()
    _dev(params, torch.float32, "params"); _dev(X, torch.float32, "X")
    off, po = _offsets(off)
    n = len(off) - 1
    L = load_library()
    ws = _workspace(L.twed_embed_workspace_size(po, n, 0), X.device, workspace)
    if emb is None:
        emb = torch.empty((n, EMBED_DIM), dtype=torch.float32, device=X.device)
    _check(L.twed_embed_forward(params.data_ptr(), X.data_ptr(), po, n, emb.data_ptr(), ws.data_ptr(),
                                ws.numel(), _stream(stream)))
    return emb


def twed_embed_loss_grad(params, X, off, pairs, target, grad=None, loss=None, emb=None, workspace=None,
                         stream=None):
    """Mean pair loss and its gradient.  pairs: int32 device (P, 2) indices
    into the collection; target: float32 device (P,) TWED values.  Returns
    (loss (1,), grad (param_count,), emb or None)."""
    torch = _torch()
    _dev(params, torch.float32, "params"); _dev(X, torch.float32, "X")
    _dev(pairs, torch.int32, "pairs"); _dev(target, torch.float32, "target")
    off, po = _offsets(off)
    n = len(off) - 1
    P = int(pairs.shape[0])
    L = load_library()
    ws = _workspace(L.twed_embed_workspace_size(po, n, P), X.device, workspace)
    if grad is None:
        grad = torch.empty(twed_embed_param_count(), dtype=torch.float32, device=X.device)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=X.device)
    _check(L.twed_embed_loss_grad(params.data_ptr(), X.data_ptr(), po, n, pairs.data_ptr(), target.data_ptr(),
                                  P, loss.data_ptr(), grad.data_ptr(), emb.data_ptr() if emb is not None else None,
                                  ws.data_ptr(), ws.numel(), _stream(stream)))
    return loss, grad, emb


def twed_embed_adamw(params, m, v, grad, step, lr, weight_decay=0.0, stream=None):
    _check(load_library().twed_embed_adamw(params.data_ptr(), m.data_ptr(), v.data_ptr(), grad.data_ptr(),
                                           int(step), float(lr), float(weight_decay), _stream(stream)))


class KnnIndex:
    """Learned k-NN index over packed 1-D FP32 series (twed_knn_index_*).
    Keeps references to DB, TDB and params (the C index does not copy them)."""

    def __init__(self, DB, TDB, offDB, params, nu=1e-3, lam=1.0, stream=None):
        torch = _torch()
        _dev(DB, torch.float32, "DB"); _dev(TDB, torch.float32, "TDB"); _dev(params, torch.float32, "params")
        self.DB, self.TDB, self.params = DB, TDB, params
        self.off, po = _offsets(offDB)
        self.nDB = len(self.off) - 1
        self.prm = make_params(nu, lam, 1.0, 1, "f32")
        L = load_library()
        need = L.twed_knn_index_storage_size(po, self.nDB, ctypes.byref(self.prm))
        if need == 0:
            _check(TWED_ERR_INVALID if L.twed_last_error() == b"" else TWED_ERR_UNSUPPORTED)
        self.storage = _workspace(need, DB.device)
        self._h = ctypes.c_void_p()
        _check(L.twed_knn_index_create(DB.data_ptr(), TDB.data_ptr(), po, self.nDB, params.data_ptr(),
                                       ctypes.byref(self.prm), self.storage.data_ptr(), self.storage.numel(),
                                       ctypes.byref(self._h)))
        # scratch returned to torch's caching allocator right away: later work
        # that reuses it is ordered after the build on the same stream
        ws = _workspace(L.twed_knn_index_build_workspace_size(self._h), DB.device)
        _check(L.twed_knn_index_build(self._h, ws.data_ptr(), ws.numel(), _stream(stream)))

    def workspace_size(self, offQ, k, n_cand) -> int:
        offQ, pq = _offsets(offQ)
        return int(load_library().twed_knn_workspace_size(self._h, pq, len(offQ) - 1, int(k), int(n_cand)))

    def query(self, Q, TQ, offQ, k=10, n_cand=200, ids=None, dist=None, workspace=None, stream=None):
        """(ids int64 (nQ, k), dist float32 (nQ, k)) of the k nearest series."""
        torch = _torch()
        _dev(Q, torch.float32, "Q"); _dev(TQ, torch.float32, "TQ")
        offQ, pq = _offsets(offQ)
        nQ = len(offQ) - 1
        L = load_library()
        ws = _workspace(L.twed_knn_workspace_size(self._h, pq, nQ, int(k), int(n_cand)), Q.device, workspace)
        if ids is None:
            ids = torch.empty((nQ, k), dtype=torch.int64, device=Q.device)
        if dist is None:
            dist = torch.empty((nQ, k), dtype=torch.float32, device=Q.device)
        _check(L.twed_knn(self._h, Q.data_ptr(), TQ.data_ptr(), pq, nQ, int(k), int(n_cand), ids.data_ptr(),
                          dist.data_ptr(), ws.data_ptr(), ws.numel(), _stream(stream)))
        return ids, dist

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _torch().cuda.synchronize()
            load_library().twed_knn_index_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
