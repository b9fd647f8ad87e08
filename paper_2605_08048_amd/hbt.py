"""Python binding of ``libhbt.so`` (include/hbt.h): argument marshalling only.

Every step of the test runs in the HIP kernels behind the C ABI; this module
turns torch tensors into device pointers, sizes and allocates the workspace
with torch (the library allocates nothing), passes torch's current stream,
and copies the per-pair ``hbt_result`` back.  There is no fallback: without
the built library every call raises.
"""
from __future__ import annotations

import ctypes as C
import os
from pathlib import Path

import numpy as np

# HBT_LIBRARY names another build of the same library (for A/B timing)
LIB_PATH = Path(os.environ.get("HBT_LIBRARY") or Path(__file__).resolve().parent / "libhbt.so")

OK, ERR_ARG, ERR_SIZE, ERR_DTYPE, ERR_WORKSPACE, ERR_DEGENERATE, ERR_MASK, ERR_DEVICE, \
    ERR_UNSUPPORTED, ERR_INTERNAL, ERR_NOT_UNIT = range(11)
PRECISION = {"f64": 0, "f32": 1, "bf16x2": 2, "i8x3": 3, "bf16e4m3": 4, "bf16lazy": 5}
DTYPE = {"f32": 0, "f64": 1}
GD = {"banerjee": 0, "identity": 1}
ALT = {"greater": 0, "two-sided": 1}
FLAG_NO_RECHECK = 1
FLAG_T_OUT_F64 = 2
FLAG_T_OUT_NORMS = 4
MAX_N, MAX_D = 65536, 8192


class HbtResult(C.Structure):
    _fields_ = [("t_obs", C.c_double), ("r_x", C.c_double), ("r_y", C.c_double), ("p", C.c_double),
                ("tau", C.c_double), ("mu_cos", C.c_double), ("t_mean", C.c_double), ("t_sd", C.c_double),
                ("count", C.c_int64), ("B", C.c_int64), ("n_recheck", C.c_int64), ("n", C.c_int64),
                ("m", C.c_int64), ("status", C.c_int32), ("h_identity", C.c_int32)]


class HbtPermParams(C.Structure):
    _fields_ = [("n", C.c_int64), ("m", C.c_int64), ("d", C.c_int64), ("B", C.c_int64),
                ("seed", C.c_uint64), ("perm_offset", C.c_uint64), ("pair_index", C.c_uint32),
                ("precision", C.c_int32), ("input_dtype", C.c_int32), ("gd", C.c_int32),
                ("alternative", C.c_int32), ("align", C.c_int32), ("stat_route", C.c_int32),
                ("flags", C.c_int32), ("block_perms", C.c_int64), ("masks", C.c_void_p)]


class HbtTuneEntry(C.Structure):
    _fields_ = [("cost", C.c_double * 2), ("grid_wide", C.c_int32), ("grid_narrow", C.c_int32),
                ("split_cap", C.c_int32), ("chunks", C.c_int32), ("tuned", C.c_int32), ("_pad", C.c_int32)]


TUNE_FIELDS = ("cost", "grid_wide", "grid_narrow", "split_cap", "chunks", "tuned")
RESULT_BYTES = 112
assert C.sizeof(HbtResult) == RESULT_BYTES and C.sizeof(HbtPermParams) == 96 and C.sizeof(HbtTuneEntry) == 40

RESULT_DTYPE = np.dtype([("t_obs", "f8"), ("r_x", "f8"), ("r_y", "f8"), ("p", "f8"), ("tau", "f8"),
                         ("mu_cos", "f8"), ("t_mean", "f8"), ("t_sd", "f8"),
                         ("count", "i8"), ("B", "i8"), ("n_recheck", "i8"), ("n", "i8"), ("m", "i8"),
                         ("status", "i4"), ("h_identity", "i4")])
assert RESULT_DTYPE.itemsize == RESULT_BYTES


class HbtError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"hbt status {status}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load libhbt.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2605_08048_amd.build`")
        L = C.CDLL(str(LIB_PATH))
        P, i64, i32, sz = C.c_void_p, C.c_int64, C.c_int32, C.c_size_t
        L.hbt_abi_version.restype = i32
        L.hbt_status_string.argtypes = [i32]
        L.hbt_status_string.restype = C.c_char_p
        L.hbt_last_error.restype = C.c_char_p
        L.hbt_align_workspace_size.argtypes = [i64, i64, i64]
        L.hbt_align_workspace_size.restype = sz
        L.hbt_align.argtypes = [i32, P, i64, P, i64, i64, i32, i32, P, P, P, P, sz, P]
        L.hbt_align.restype = i32
        L.hbt_perm_test_workspace_size.argtypes = [C.POINTER(HbtPermParams)]
        L.hbt_perm_test_workspace_size.restype = sz
        L.hbt_perm_test.argtypes = [P, P, C.POINTER(HbtPermParams), P, P, P, P, sz, P]
        L.hbt_perm_test.restype = i32
        L.hbt_perm_test_batched_workspace_size.argtypes = [i64, P, P, P, i64, C.POINTER(HbtPermParams)]
        L.hbt_perm_test_batched_workspace_size.restype = sz
        L.hbt_perm_test_batched.argtypes = [i64, P, P, P, P, P, P, i64, C.POINTER(HbtPermParams), P, P,
                                            sz, P]
        L.hbt_perm_test_batched.restype = i32
        L.hbt_stage_timing.argtypes = [i32]
        L.hbt_stage_timing.restype = i32
        L.hbt_stage_times.argtypes = [P, P]
        L.hbt_stage_times.restype = i32
        dbl, flt = C.c_double, C.c_float
        L.hbt_tune_batched.argtypes = [i64, P, P, P, P, P, P, i64, C.POINTER(HbtPermParams), P, P, sz, P]
        L.hbt_tune_get.argtypes = [i64, P, P]
        L.hbt_tune_set.argtypes = [i64, P]
        L.hbt_tune_entry_get.argtypes = [i32, i64, C.POINTER(HbtTuneEntry)]
        L.hbt_tune_entry_set.argtypes = [i32, i64, C.POINTER(HbtTuneEntry)]
        L.hbt_tune_save.argtypes = [C.c_char_p]
        L.hbt_tune_load.argtypes = [C.c_char_p]
        for f in ["hbt_tune_entry_get", "hbt_tune_entry_set", "hbt_tune_save", "hbt_tune_load"]:
            getattr(L, f).restype = i32
        L.hbt_tile_widths.argtypes = [i64, P, i64, P]
        L.hbt_recheck_band.argtypes = [i32, i32, i32, i64, i64, i64, dbl, dbl, P]
        L.hbt_perm_test_static.argtypes = [P, P, C.POINTER(HbtPermParams), P, P, P, P]
        L.hbt_perm_test_clouds_workspace_size.argtypes = [i64, P, i64, P, P, P, i64, C.POINTER(HbtPermParams)]
        L.hbt_perm_test_clouds_workspace_size.restype = sz
        L.hbt_perm_test_clouds.argtypes = [i64, P, P, P, i64, P, P, P, P, i64, C.POINTER(HbtPermParams), P, P,
                                           sz, P]
        L.hbt_perm_test_clouds.restype = i32
        L.hbt_pipeline_chunks.argtypes = [i32, P]
        L.hbt_pipeline_chunks.restype = i32
        L.hbt_perm_test_static.restype = i32
        for f in ["hbt_tune_batched", "hbt_tune_get", "hbt_tune_set", "hbt_tile_widths", "hbt_recheck_band"]:
            getattr(L, f).restype = i32
        L.hbt_budget_features.argtypes = [i64, P, i64, i32, P, P]
        L.hbt_feature_norm.argtypes = [i64, P, P, P]
        L.hbt_target_norm.argtypes = [i64, P, P, P]
        L.hbt_null_targets.argtypes = [i64, P, P, P]
        L.hbt_mlp_forward.argtypes = [i64, P, P, P, P]
        L.hbt_mlp_grad_workspace_size.argtypes = [i64]
        L.hbt_mlp_grad_workspace_size.restype = sz
        L.hbt_mlp_grad.argtypes = [i64, P, P, P, P, P, P, sz, P]
        L.hbt_mlp_adam.argtypes = [P, P, P, P, i64, flt, flt, flt, flt, P]
        L.hbt_budgets.argtypes = [i64, P, P, dbl, dbl, i64, i64, dbl, P, P]
        L.hbt_budgets_min_cost.argtypes = [i64, P, P, dbl, dbl, i64, i64, P, P]
        L.hbt_budgets_min_cost.restype = i32
        for f in ["hbt_budget_features", "hbt_null_targets", "hbt_feature_norm", "hbt_target_norm", "hbt_mlp_forward", "hbt_mlp_grad",
                  "hbt_mlp_adam", "hbt_budgets"]:
            getattr(L, f).restype = i32
        _lib = L
    return _lib


def _check(status):
    if status != OK:
        L = lib()
        raise HbtError(status, (L.hbt_last_error() or L.hbt_status_string(status)).decode())


def _torch():
    import torch
    return torch


def _stream(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


_ws = {}


def workspace(nbytes, device):
    """A cached device byte buffer of at least ``nbytes`` (allocated by torch)."""
    torch = _torch()
    key = str(device)
    buf = _ws.get(key)
    if buf is None or buf.numel() < nbytes:
        _ws[key] = buf = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
    return buf


def _dev_tensor(a, dtype, device):
    torch = _torch()
    if isinstance(a, torch.Tensor):
        t = a.to(device=device, dtype=dtype)
    else:
        t = torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=device)
    return t.contiguous()


def _on_device(name, t, device=None):
    """Raise unless ``t`` is a tensor in GPU memory (on ``device`` if given):
    the library dereferences every pointer it is handed on the GPU."""
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise HbtError(ERR_ARG, f"{name} must be a GPU tensor")
    if device is not None and t.device != device:
        raise HbtError(ERR_ARG, f"{name} is on {t.device}, the call runs on {device}")


def _pair_operands(X, Y):
    """Shape checks shared by the one-pair calls: X (n, d), Y (m, d), one device."""
    if X.dim() != 2 or Y.dim() != 2 or X.shape[1] != Y.shape[1]:
        raise HbtError(ERR_SIZE, f"X {tuple(X.shape)} and Y {tuple(Y.shape)} must be (n, d) and (m, d)")
    _on_device("X", X)
    _on_device("Y", Y, X.device)


def _input_dtype(X):
    torch = _torch()
    if X.dtype == torch.float64:
        return DTYPE["f64"]
    if X.dtype == torch.float32:
        return DTYPE["f32"]
    raise HbtError(ERR_DTYPE, f"inputs must be float32 or float64, got {X.dtype}")


def results_to_numpy(res_tensor):
    raw = res_tensor.cpu().numpy().tobytes()
    return np.frombuffer(raw, dtype=RESULT_DTYPE).copy()


def _result_dict(row):
    return {k: (row[k].item()) for k in RESULT_DTYPE.names}


def make_params(n, m, d, B, *, seed=0, perm_offset=0, pair_index=0, precision="f32", input_dtype=0,
                gd="banerjee", alternative="greater", align=True, stat_route=0, recheck=True,
                block_perms=0, masks_ptr=None):
    return HbtPermParams(n=n, m=m, d=d, B=B, seed=seed, perm_offset=perm_offset, pair_index=pair_index,
                         precision=PRECISION[precision], input_dtype=input_dtype, gd=GD[gd],
                         alternative=ALT[alternative], align=1 if align else 0, stat_route=stat_route,
                         flags=0 if recheck else FLAG_NO_RECHECK, block_perms=block_perms,
                         masks=masks_ptr)


def align(X, Y, *, align=True, gd="banerjee", out=None, stream=None):
    """Householder alignment of X onto Y's mean direction (Algorithm 1, Steps 1-4)."""
    torch = _torch()
    _pair_operands(X, Y)
    n, d = X.shape
    m = Y.shape[0]
    dev = X.device
    Y = Y.to(dtype=X.dtype).contiguous()
    X = X.contiguous()
    if out is not None:
        _on_device("out", out, dev)
        if out.shape != X.shape or out.dtype != X.dtype or not out.is_contiguous():
            raise HbtError(ERR_ARG, f"out must be a contiguous {X.dtype} tensor of shape {tuple(X.shape)}")
    Xo = out if out is not None else torch.empty_like(X)
    v = torch.empty(d, dtype=torch.float64, device=dev)
    res = torch.zeros(RESULT_BYTES, dtype=torch.uint8, device=dev)
    L = lib()
    need = L.hbt_align_workspace_size(n, m, d)
    ws = workspace(need, dev)
    _check(L.hbt_align(_input_dtype(X), C.c_void_p(X.data_ptr()), n, C.c_void_p(Y.data_ptr()), m, d,
                       1 if align else 0, GD[gd], C.c_void_p(Xo.data_ptr()), C.c_void_p(v.data_ptr()),
                       C.c_void_p(res.data_ptr()), C.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream)))
    r = _result_dict(results_to_numpy(res)[0])
    r.update(X_out=Xo, v=v)
    return r


def perm_test(X, Y, B, *, seed=0, perm_offset=0, pair_index=0, precision="f32", gd="banerjee",
              alternative="greater", align=True, recheck=True, block_perms=0, masks=None,
              stat_route=0, want_T=False, want_masks=False, stream=None, sync=True,
              static_scratch=False):
    """The whole test for one pair.  Returns a dict of the hbt_result fields,
    plus ``T`` (B floats; doubles with want_T="f64"; B x 3 doubles (T_b,
    |sigma_1|^2, |sigma_2|^2) with want_T="norms") and ``masks``
    (B x ceil(N/32) words) when asked.  ``static_scratch``: call
    hbt_perm_test_static, which uses the library's own device scratch
    instead of a workspace allocated here."""
    torch = _torch()
    _pair_operands(X, Y)
    n, d = X.shape
    m = Y.shape[0]
    dev = X.device
    X = X.contiguous()
    Y = Y.to(dtype=X.dtype).contiguous()
    W = (n + m + 31) // 32
    mk = None
    if masks is not None:
        mk = _dev_tensor(np.asarray(masks, dtype=np.uint32).view(np.int32).reshape(B, W)
                         if not isinstance(masks, torch.Tensor) else masks, torch.int32, dev)
        if mk.numel() != B * W:
            raise HbtError(ERR_SIZE, f"masks hold {mk.numel()} words, B x ceil((n+m)/32) = {B * W}")
    prm = make_params(n, m, d, B, seed=seed, perm_offset=perm_offset, pair_index=pair_index,
                      precision=precision, input_dtype=_input_dtype(X), gd=gd, alternative=alternative,
                      align=align, recheck=recheck, block_perms=block_perms, stat_route=stat_route,
                      masks_ptr=None if mk is None else mk.data_ptr())
    t64 = want_T in ("f64", "norms")
    if want_T == "f64":
        prm.flags |= FLAG_T_OUT_F64
    if want_T == "norms":
        prm.flags |= FLAG_T_OUT_NORMS
    L = lib()
    res = torch.zeros(RESULT_BYTES, dtype=torch.uint8, device=dev)
    T = torch.empty((B, 3) if want_T == "norms" else B, dtype=torch.float64 if t64 else torch.float32,
                    device=dev) if want_T else None
    mo = torch.empty((B, W), dtype=torch.int32, device=dev) if want_masks else None
    outs = (C.c_void_p(res.data_ptr()), None if T is None else C.c_void_p(T.data_ptr()),
            None if mo is None else C.c_void_p(mo.data_ptr()))
    if static_scratch:
        _check(L.hbt_perm_test_static(C.c_void_p(X.data_ptr()), C.c_void_p(Y.data_ptr()), C.byref(prm),
                                      *outs, _stream(stream)))
    else:
        need = L.hbt_perm_test_workspace_size(C.byref(prm))
        if need == 0:
            need = 256
        ws = workspace(need, dev)
        _check(L.hbt_perm_test(C.c_void_p(X.data_ptr()), C.c_void_p(Y.data_ptr()), C.byref(prm), *outs,
                               C.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream)))
    if not sync:
        return dict(result=res, T=T, masks=mo)
    r = _result_dict(results_to_numpy(res)[0])
    if T is not None:
        r["T"] = T.cpu().numpy()
    if mo is not None:
        r["masks"] = mo.cpu().numpy().view(np.uint32)
    return r


def pipeline_chunks(chunks):
    """Set the number of pipeline chunks of later batched calls (0 = default);
    returns the previous setting."""
    prev = C.c_int32()
    _check(lib().hbt_pipeline_chunks(int(chunks), C.byref(prev)))
    return prev.value


def recheck_band(precision, n, m, d, r1, r2, *, stat_route=0, gd="banerjee"):
    """Half-width of the FP64 recheck band for splits with permuted mean
    resultant lengths r1, r2 (arrays or scalars); a host call of the library."""
    L = lib()
    r1 = np.broadcast_to(np.asarray(r1, dtype=np.float64), np.broadcast(r1, r2).shape)
    r2 = np.broadcast_to(np.asarray(r2, dtype=np.float64), r1.shape)
    out = np.empty(r1.shape, dtype=np.float64)
    e = C.c_double()
    for idx in np.ndindex(r1.shape):
        _check(L.hbt_recheck_band(PRECISION[precision], stat_route, GD[gd], n, m, d,
                                  float(r1[idx]), float(r2[idx]), C.byref(e)))
        out[idx] = e.value
    return out if out.shape else float(out)


def batched_workspace_size(row_offset, n, m, B, d, *, precision="bf16x2", input_dtype="f32", stat_route=0):
    """Workspace bytes of one ``perm_test_batched`` call of these shapes."""
    P = len(n)
    nn = np.ascontiguousarray(n, dtype=np.int64)
    mm = np.ascontiguousarray(m, dtype=np.int64)
    BB = np.ascontiguousarray(np.broadcast_to(np.asarray(B, dtype=np.int64), (P,)))
    prm = make_params(0, 0, d, 0, precision=precision, input_dtype={"f32": 0, "f64": 1}[input_dtype],
                      stat_route=stat_route)
    ptr = lambda a: a.ctypes.data_as(C.c_void_p)
    return int(lib().hbt_perm_test_batched_workspace_size(P, ptr(nn), ptr(mm), ptr(BB), d, C.byref(prm)))


def _batch_tables(Z_all, row_offset, n, m, B, pair_index):
    """Host tables of a batched call, checked: Z_all (rows, d) on the GPU, one
    entry per pair (row_offset may carry more, e.g. a cumulative table, whose
    first P count), and every pair's rows inside Z_all, whose length the
    library cannot see."""
    if Z_all.dim() != 2:
        raise HbtError(ERR_SIZE, f"Z_all must be (rows, d), got {tuple(Z_all.shape)}")
    P = len(n)
    off = np.ascontiguousarray(np.asarray(row_offset, dtype=np.int64)[:P])
    nn = np.ascontiguousarray(n, dtype=np.int64)
    mm = np.ascontiguousarray(m, dtype=np.int64)
    BB = np.ascontiguousarray(np.broadcast_to(np.asarray(B, dtype=np.int64), (P,)))
    ids = None if pair_index is None else np.ascontiguousarray(pair_index, dtype=np.uint32)
    if off.shape != (P,) or mm.shape != (P,) or (ids is not None and ids.shape != (P,)):
        raise HbtError(ERR_SIZE, "row_offset, n, m and pair_index need one entry per pair")
    outside = (off < 0) | (off + nn + mm > Z_all.shape[0])
    if np.any(outside):
        k = int(np.flatnonzero(outside)[0])
        raise HbtError(ERR_SIZE, f"pair {k}: rows [{off[k]}, {off[k] + nn[k] + mm[k]}) "
                                 f"outside Z_all's {Z_all.shape[0]} rows")
    _on_device("Z_all", Z_all)
    return P, off, nn, mm, BB, ids


def perm_test_batched(Z_all, row_offset, n, m, B, *, seed=0, perm_offset=0, pair_index=None,
                      precision="bf16x2", gd="banerjee", alternative="greater", align=True, recheck=True,
                      stream=None, sync=True, results=None, workspace=None, stat_route=0):
    """Many pairs in one call.  Z_all (device tensor) holds rows X_0, Y_0, X_1, ...;
    row_offset/n/m/B are host integer arrays.  ``pair_index`` (host, one Philox
    counter word per pair; default 0, 1, 2, ...): pairs with equal n, m, B and
    index get identical splits, drawn once.  Returns a numpy structured array
    of hbt_result (or, with sync=False, the device result tensor).  A caller
    that captures the call into a graph passes its own ``workspace`` (a uint8
    device tensor that outlives the graph) instead of the shared cached one."""
    torch = _torch()
    dev = Z_all.device
    P, off, nn, mm, BB, ids = _batch_tables(Z_all, row_offset, n, m, B, pair_index)
    if results is not None:
        _on_device("results", results, dev)
        if results.dtype != torch.uint8 or results.numel() < RESULT_BYTES * P or not results.is_contiguous():
            raise HbtError(ERR_SIZE, f"results must be a contiguous uint8 tensor of {RESULT_BYTES * P} bytes")
    if workspace is not None:
        _on_device("workspace", workspace, dev)
        if workspace.dtype != torch.uint8 or not workspace.is_contiguous():
            raise HbtError(ERR_ARG, "workspace must be a contiguous uint8 tensor")
    Z_all = Z_all.contiguous()
    d = Z_all.shape[1]
    prm = make_params(0, 0, d, 0, seed=seed, perm_offset=perm_offset, precision=precision,
                      input_dtype=_input_dtype(Z_all), gd=gd, alternative=alternative, align=align,
                      recheck=recheck, stat_route=stat_route)
    L = lib()
    ptr = lambda a: a.ctypes.data_as(C.c_void_p)
    need = L.hbt_perm_test_batched_workspace_size(P, ptr(nn), ptr(mm), ptr(BB), d, C.byref(prm))
    if workspace is None:
        ws = globals()["workspace"](max(need, 256), dev)
    else:
        ws = workspace
        if ws.numel() < need:
            raise ValueError(f"workspace of {ws.numel()} bytes, the call needs {need}")
    res = results if results is not None else torch.zeros(RESULT_BYTES * P, dtype=torch.uint8, device=dev)
    _check(L.hbt_perm_test_batched(P, C.c_void_p(Z_all.data_ptr()), ptr(off), ptr(nn), ptr(mm), ptr(BB),
                                   None if ids is None else ptr(ids), d, C.byref(prm),
                                   C.c_void_p(res.data_ptr()), C.c_void_p(ws.data_ptr()), ws.numel(),
                                   _stream(stream)))
    if not sync:
        return res
    return results_to_numpy(res)


def perm_test_clouds(Z_all, cloud_offset, cloud_rows, pair_x, pair_y, B, *, seed=0, perm_offset=0,
                     pair_index=None, gd="banerjee", alternative="greater", align=True, recheck=True,
                     stream=None, sync=True, results=None, workspace=None):
    """Many pairs over shared clouds, each cloud stored once (split BF16, the
    Householder reflection folded into the statistic).  Z_all (device FP32
    tensor) holds the clouds' rows: cloud c is ``cloud_rows[c]`` rows from row
    ``cloud_offset[c]``; pair p tests cloud ``pair_x[p]`` (X) against cloud
    ``pair_y[p]`` (Y) with ``B[p]`` splits.  Returns a numpy structured array
    of hbt_result (or, with sync=False, the device result tensor)."""
    torch = _torch()
    dev = Z_all.device
    _on_device("Z_all", Z_all, dev)
    if Z_all.dtype != torch.float32 or Z_all.dim() != 2:
        raise HbtError(ERR_DTYPE, "Z_all must be a 2-D float32 tensor")
    Z_all = Z_all.contiguous()
    d = Z_all.shape[1]
    off = np.ascontiguousarray(cloud_offset, dtype=np.int64).ravel()
    rows = np.ascontiguousarray(cloud_rows, dtype=np.int64).ravel()
    px = np.ascontiguousarray(pair_x, dtype=np.int64).ravel()
    py = np.ascontiguousarray(pair_y, dtype=np.int64).ravel()
    P = px.size
    BB = np.ascontiguousarray(np.broadcast_to(np.asarray(B, dtype=np.int64), (P,)))
    if off.size != rows.size or py.size != P:
        raise HbtError(ERR_SIZE, "cloud_offset / cloud_rows and pair_x / pair_y must have equal lengths")
    if np.any(off < 0) or np.any(off + rows > Z_all.shape[0]):
        raise HbtError(ERR_SIZE, "a cloud's rows lie outside Z_all")
    ids = None if pair_index is None else np.ascontiguousarray(pair_index, dtype=np.uint32).ravel()
    if ids is not None and ids.size != P:
        raise HbtError(ERR_SIZE, "pair_index needs one entry per pair")
    prm = make_params(0, 0, d, 0, seed=seed, perm_offset=perm_offset, precision="bf16x2", input_dtype=0, gd=gd,
                      alternative=alternative, align=align, recheck=recheck)
    L = lib()
    ptr = lambda a: a.ctypes.data_as(C.c_void_p)
    need = L.hbt_perm_test_clouds_workspace_size(rows.size, ptr(rows), P, ptr(px), ptr(py), ptr(BB), d,
                                                 C.byref(prm))
    if need == 0:
        need = 256
    ws = workspace if workspace is not None else globals()["workspace"](need, dev)
    if results is not None:
        _on_device("results", results, dev)
        if results.dtype != torch.uint8 or results.numel() < RESULT_BYTES * P or not results.is_contiguous():
            raise HbtError(ERR_SIZE, f"results must be a contiguous uint8 tensor of {RESULT_BYTES * P} bytes")
    res = results if results is not None else torch.zeros(RESULT_BYTES * P, dtype=torch.uint8, device=dev)
    _check(L.hbt_perm_test_clouds(rows.size, C.c_void_p(Z_all.data_ptr()), ptr(off), ptr(rows), P, ptr(px),
                                  ptr(py), ptr(BB), None if ids is None else ptr(ids), d, C.byref(prm),
                                  C.c_void_p(res.data_ptr()), C.c_void_p(ws.data_ptr()), ws.numel(),
                                  _stream(stream)))
    if not sync:
        return res
    return results_to_numpy(res)


# ------------------------------------------------------------------ allocator kernels

MLP_FEATURES, MLP_PARAMS, MLP_TRAINABLE_OFFSET = 12, 5150, 28
GD = {"banerjee": 0, "identity": 1}


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _need(name, t, dtype, *, cols=None, numel=None, device=None):
    """Raise unless ``t`` is a contiguous GPU tensor of ``dtype`` with ``cols``
    columns (2-D) or ``numel`` elements: the kernels index it by those sizes."""
    _on_device(name, t, device)
    if t.dtype != dtype or not t.is_contiguous():
        raise HbtError(ERR_ARG, f"{name} must be a contiguous {dtype} tensor, got {t.dtype}")
    if cols is not None and (t.dim() != 2 or t.shape[1] != cols):
        raise HbtError(ERR_SIZE, f"{name} must be (rows, {cols}), got {tuple(t.shape)}")
    if numel is not None and t.numel() != numel:
        raise HbtError(ERR_SIZE, f"{name} must hold {numel} elements, got {t.numel()}")


def _results_records(results, device=None):
    """Number of hbt_result records in a uint8 device tensor (checked)."""
    torch = _torch()
    _need("results", results, torch.uint8, device=device)
    if results.numel() % RESULT_BYTES:
        raise HbtError(ERR_SIZE, f"results hold {results.numel()} bytes, not a multiple of {RESULT_BYTES}")
    return results.numel() // RESULT_BYTES


def budget_features(results, d, gd="banerjee", stream=None):
    """(npairs, 12) float32 device tensor of allocator inputs from a device
    tensor of hbt_result records (as returned with sync=False)."""
    torch = _torch()
    P = _results_records(results)
    out = torch.empty((P, MLP_FEATURES), dtype=torch.float32, device=results.device)
    _check(lib().hbt_budget_features(P, _ptr(results), d, GD[gd], _ptr(out), _stream(stream)))
    return out


def null_targets(results, stream=None):
    """(npairs, 2) float32 device tensor (t_mean, log t_sd) of hbt_result records."""
    torch = _torch()
    P = _results_records(results)
    out = torch.empty((P, 2), dtype=torch.float32, device=results.device)
    _check(lib().hbt_null_targets(P, _ptr(results), _ptr(out), _stream(stream)))
    return out


def feature_norm(features, theta, stream=None):
    """Write the per-feature standardisation (mean, 1/sd) into theta[0:24]."""
    torch = _torch()
    _need("features", features, torch.float32, cols=MLP_FEATURES)
    _need("theta", theta, torch.float32, numel=MLP_PARAMS, device=features.device)
    _check(lib().hbt_feature_norm(features.shape[0], _ptr(features), _ptr(theta), _stream(stream)))


def target_norm(targets, theta, stream=None):
    """Write the output standardisation (mean, sd of the targets) into theta[24:28]."""
    torch = _torch()
    _need("targets", targets, torch.float32, cols=2)
    _need("theta", theta, torch.float32, numel=MLP_PARAMS, device=targets.device)
    _check(lib().hbt_target_norm(targets.shape[0], _ptr(targets), _ptr(theta), _stream(stream)))


def mlp_forward(features, theta, stream=None):
    torch = _torch()
    _need("features", features, torch.float32, cols=MLP_FEATURES)
    _need("theta", theta, torch.float32, numel=MLP_PARAMS, device=features.device)
    out = torch.empty((features.shape[0], 2), dtype=torch.float32, device=features.device)
    _check(lib().hbt_mlp_forward(features.shape[0], _ptr(features), _ptr(theta), _ptr(out), _stream(stream)))
    return out


def mlp_grad(features, targets, theta, grad=None, loss=None, stream=None):
    """(grad, loss): float32 gradient of the mean half squared error and the
    FP64 loss, both device tensors."""
    torch = _torch()
    _need("features", features, torch.float32, cols=MLP_FEATURES)
    R = features.shape[0]
    dev = features.device
    _need("targets", targets, torch.float32, cols=2, device=dev)
    if targets.shape[0] != R:
        raise HbtError(ERR_SIZE, f"{R} feature rows but {targets.shape[0]} target rows")
    _need("theta", theta, torch.float32, numel=MLP_PARAMS, device=dev)
    grad = grad if grad is not None else torch.zeros(MLP_PARAMS, dtype=torch.float32, device=dev)
    loss = loss if loss is not None else torch.zeros(1, dtype=torch.float64, device=dev)
    _need("grad", grad, torch.float32, numel=MLP_PARAMS, device=dev)
    _need("loss", loss, torch.float64, numel=1, device=dev)
    L = lib()
    ws = workspace(L.hbt_mlp_grad_workspace_size(R), dev)
    _check(L.hbt_mlp_grad(R, _ptr(features), _ptr(targets), _ptr(theta), _ptr(grad), _ptr(loss), _ptr(ws),
                          ws.numel(), _stream(stream)))
    return grad, loss


def mlp_adam(theta, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    torch = _torch()
    for name, t in (("theta", theta), ("grad", grad), ("m", m), ("v", v)):
        _need(name, t, torch.float32, numel=MLP_PARAMS, device=theta.device)
    _check(lib().hbt_mlp_adam(_ptr(theta), _ptr(grad), _ptr(m), _ptr(v), step, lr, beta1, beta2, eps,
                              _stream(stream)))


def budgets(mlp_out, results, p_lo, p_hi, b_min, b_max, zq=2.3263478740408408, stream=None):
    """int64 device tensor of permutation budgets per pair."""
    torch = _torch()
    _need("mlp_out", mlp_out, torch.float32, cols=2)
    P = mlp_out.shape[0]
    if _results_records(results, mlp_out.device) < P:
        raise HbtError(ERR_SIZE, f"{P} predictions but fewer hbt_result records")
    out = torch.empty(P, dtype=torch.int64, device=mlp_out.device)
    _check(lib().hbt_budgets(P, _ptr(mlp_out), _ptr(results), p_lo, p_hi, b_min, b_max, zq, _ptr(out),
                             _stream(stream)))
    return out


def budgets_min_cost(mlp_out, results, p_lo, p_hi, b_min, b_max, stream=None):
    """int64 device tensor of permutation budgets per pair by expected cost."""
    torch = _torch()
    _need("mlp_out", mlp_out, torch.float32, cols=2)
    P = mlp_out.shape[0]
    if _results_records(results, mlp_out.device) < P:
        raise HbtError(ERR_SIZE, f"{P} predictions but fewer hbt_result records")
    out = torch.empty(P, dtype=torch.int64, device=mlp_out.device)
    _check(lib().hbt_budgets_min_cost(P, _ptr(mlp_out), _ptr(results), p_lo, p_hi, b_min, b_max, _ptr(out),
                                      _stream(stream)))
    return out


# ------------------------------------------------------------------ tile-width tuning

def tune_batched(Z_all, row_offset, n, m, B, *, seed=0, pair_index=None, gd="banerjee", workspace=None,
                 precision="bf16x2"):
    """Measure the launch parameters of this batch's precision and dimension
    (tile widths, persistent grids, split work-groups per CU, pipeline
    chunks) and install them; returns the split-BF16 costs (cost_1024,
    cost_256) for d (see tune_entry_get for the rest)."""
    torch = _torch()
    dev = Z_all.device
    P, off, nn, mm, BB, ids = _batch_tables(Z_all, row_offset, n, m, B, pair_index)
    if workspace is not None:
        _on_device("workspace", workspace, dev)
        if workspace.dtype != torch.uint8 or not workspace.is_contiguous():
            raise HbtError(ERR_ARG, "workspace must be a contiguous uint8 tensor")
    Z_all = Z_all.contiguous()
    d = Z_all.shape[1]
    prm = make_params(0, 0, d, 0, seed=seed, precision=precision, input_dtype=_input_dtype(Z_all), gd=gd)
    L = lib()
    ptr = lambda a: a.ctypes.data_as(C.c_void_p)
    need = L.hbt_perm_test_batched_workspace_size(P, ptr(nn), ptr(mm), ptr(BB), d, C.byref(prm))
    ws = workspace if workspace is not None else globals()["workspace"](max(need, 256), dev)
    res = torch.zeros(RESULT_BYTES * P, dtype=torch.uint8, device=dev)
    _check(L.hbt_tune_batched(P, C.c_void_p(Z_all.data_ptr()), ptr(off), ptr(nn), ptr(mm), ptr(BB),
                              None if ids is None else ptr(ids), d, C.byref(prm), C.c_void_p(res.data_ptr()),
                              C.c_void_p(ws.data_ptr()), ws.numel(), _stream(None)))
    return tune_get(d)[0]


def tune_get(d):
    """((cost_1024, cost_256), tuned) for dimension d."""
    c = (C.c_double * 2)()
    t = C.c_int32()
    _check(lib().hbt_tune_get(d, c, C.byref(t)))
    return (c[0], c[1]), bool(t.value)


def tune_set(d, costs):
    c = (C.c_double * 2)(*[float(x) for x in costs])
    _check(lib().hbt_tune_set(d, c))


def tile_widths(B, d):
    BB = np.ascontiguousarray(np.asarray(B, dtype=np.int64).ravel())
    out = np.zeros(BB.size, dtype=np.int32)
    _check(lib().hbt_tile_widths(BB.size, BB.ctypes.data_as(C.c_void_p), d, out.ctypes.data_as(C.c_void_p)))
    return out


def tune_entry_get(precision, d):
    """The tuned launch parameters of (precision, d) as a dict."""
    e = HbtTuneEntry()
    _check(lib().hbt_tune_entry_get(PRECISION[precision], d, C.byref(e)))
    return {"cost": (e.cost[0], e.cost[1]), "grid_wide": e.grid_wide, "grid_narrow": e.grid_narrow,
            "split_cap": e.split_cap, "chunks": e.chunks, "tuned": bool(e.tuned)}


def tune_entry_set(precision, d, entry):
    e = HbtTuneEntry()
    e.cost[0], e.cost[1] = (float(x) for x in entry["cost"])
    for k in ("grid_wide", "grid_narrow", "split_cap", "chunks"):
        setattr(e, k, int(entry[k]))
    _check(lib().hbt_tune_entry_set(PRECISION[precision], d, C.byref(e)))


def save_tuning(path):
    """Write every tuned entry to a JSON file (the library's format, also the
    HBT_TUNE_CACHE file)."""
    _check(lib().hbt_tune_save(os.fsencode(str(path))))


def load_tuning(path):
    """Load entries written by save_tuning into the library's table."""
    _check(lib().hbt_tune_load(os.fsencode(str(path))))

