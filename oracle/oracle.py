"""ctypes front end of the FP64 CPU oracle (``hbt_oracle.c``).

TEST INFRASTRUCTURE ONLY: used by ``tests/``, the smoke check and the
benchmark's CPU-baseline leg.  The product library never imports it.

All arrays are passed as float64 (float32 inputs are widened exactly).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from pathlib import Path

import numpy as np

HERE = Path(__file__).resolve().parent
SRC = HERE / "hbt_oracle.c"
LIB = HERE / "libhbt_oracle.so"

GD_BANERJEE, GD_IDENTITY = 0, 1
ALT_GREATER, ALT_TWO_SIDED = 0, 1
OK, ERR_ARG, ERR_SIZE, ERR_DEGENERATE, ERR_MASK, ERR_NOT_UNIT = 0, 1, 2, 5, 6, 10


def build(force: bool = False) -> Path:
    """Compile the oracle with gcc (-O2, OpenMP); plain C, no BLAS."""
    if force or not LIB.exists() or LIB.stat().st_mtime < SRC.stat().st_mtime:
        tmp = LIB.with_suffix(".so.tmp")
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", str(SRC), "-o", str(tmp), "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(str(LIB))
        P = C.c_void_p
        i64, u64, u32, i32, dbl = C.c_int64, C.c_uint64, C.c_uint32, C.c_int, C.c_double
        L.oracle_philox4x32.argtypes = [P, P, i32, P]
        L.oracle_philox4x64.argtypes = [P, P, i32, P]
        L.oracle_split_keys.argtypes = [u64, u32, u32, i64, P, P]
        L.oracle_split_mask.argtypes = [u64, u32, u32, i64, i64, P]
        L.oracle_log_g.argtypes = [dbl, i64, i32]
        L.oracle_log_g.restype = dbl
        L.oracle_mrl.argtypes = [P, i64, i64]
        L.oracle_mrl.restype = dbl
        L.oracle_align.argtypes = [P, i64, P, i64, i64, i32, i32, P, P, P, P, P]
        L.oracle_align.restype = i32
        L.oracle_split_stat.argtypes = [P, i64, i64, i64, P, i32, P, P]
        L.oracle_split_stat.restype = dbl
        L.oracle_perm_test.argtypes = [P, i64, P, i64, i64, i64, u64, u32, u64, i32, i32, i32, P, P, P, P, i32]
        L.oracle_perm_test.restype = i32
        L.oracle_perm_stats_at.argtypes = [P, i64, P, i64, i64, u64, u32, i32, i32, P, i64, P, P, P, P, i32]
        L.oracle_perm_stats_at.restype = i32
        L.oracle_exhaustive.argtypes = [P, i64, P, i64, i64, i32, i32, i32, P, P, i64]
        L.oracle_exhaustive.restype = i32
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def philox4x32(ctr, key, rounds=10):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox4x32(_p(c), _p(k), rounds, _p(out))
    return out


def philox4x64(ctr, key, rounds=10):
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().oracle_philox4x64(_p(c), _p(k), rounds, _p(out))
    return out


def split_keys(seed, pair, b, N):
    P = np.zeros(N, dtype=np.uint8)
    S = np.zeros(N, dtype=np.uint32)
    lib().oracle_split_keys(seed, pair, b, N, _p(P), _p(S))
    return P, S


def n_words(N):
    return (N + 31) // 32


def split_mask(seed, pair, b, N, n):
    w = np.zeros(n_words(N), dtype=np.uint32)
    lib().oracle_split_mask(seed, pair, b, N, n, _p(w))
    return w


def mask_to_bool(words, N):
    w = np.ascontiguousarray(words, dtype="<u4")
    one = w.ndim == 1
    w2 = w.reshape(1, -1) if one else w
    bits = np.unpackbits(w2.view(np.uint8), axis=1, bitorder="little")[:, :N].astype(bool)
    return bits[0] if one else bits


def bool_to_mask(sel):
    sel = np.atleast_2d(np.asarray(sel, dtype=bool))
    N = sel.shape[1]
    W = n_words(N)
    pad = np.zeros((sel.shape[0], W * 32), dtype=np.uint8)
    pad[:, :N] = sel
    return np.packbits(pad, axis=1, bitorder="little").view("<u4").reshape(sel.shape[0], W)


def log_g(r, d, gd=GD_BANERJEE):
    return lib().oracle_log_g(float(r), int(d), int(gd))


def mrl(A):
    A = _f64(A)
    return lib().oracle_mrl(_p(A), A.shape[0], A.shape[1])


def align(X, Y, align=1, gd=GD_BANERJEE):
    X, Y = _f64(X), _f64(Y)
    n, d = X.shape
    m = Y.shape[0]
    Xp = np.zeros_like(X)
    mux, muy, v = np.zeros(d), np.zeros(d), np.zeros(d)
    info = np.zeros(8)
    st = lib().oracle_align(_p(X), n, _p(Y), m, d, align, gd, _p(Xp), _p(mux), _p(muy), _p(v), _p(info))
    return dict(status=st, Xp=Xp, mu_x=mux, mu_y=muy, v=v, r_x=info[0], r_y=info[1], t_obs=info[2],
                h_identity=int(info[3]), vv=info[4], tau=info[5], f_x=info[6], f_y=info[7])


def split_stat(Z, n, m, mask, gd=GD_BANERJEE):
    Z = _f64(Z)
    mk = np.ascontiguousarray(mask, dtype=np.uint32)
    r1, r2 = C.c_double(), C.c_double()
    T = lib().oracle_split_stat(_p(Z), n, m, Z.shape[1], _p(mk), gd, C.byref(r1), C.byref(r2))
    return T, r1.value, r2.value


def perm_test(X, Y, B, seed=0, pair=0, perm_offset=0, align=1, gd=GD_BANERJEE, alternative=ALT_GREATER,
              masks=None, want_T=False, want_masks=False, nthreads=0):
    X, Y = _f64(X), _f64(Y)
    n, d = X.shape
    m = Y.shape[0]
    W = n_words(n + m)
    out = np.zeros(8)
    T = np.zeros(B) if want_T else None
    mo = np.zeros((B, W), dtype=np.uint32) if want_masks else None
    mk = None if masks is None else np.ascontiguousarray(masks, dtype=np.uint32).reshape(B, W)
    st = lib().oracle_perm_test(_p(X), n, _p(Y), m, d, B, seed, pair, perm_offset, align, gd, alternative,
                                _p(mk), _p(out), _p(T), _p(mo), nthreads)
    return dict(status=st, t_obs=out[0], r_x=out[1], r_y=out[2], p=out[3], count=int(out[4]),
                h_identity=int(out[5]), tau=out[6], vv=out[7], T=T, masks=mo, B=B)


def perm_stats_at(X, Y, blist, seed=0, pair=0, align=1, gd=GD_BANERJEE, want_masks=False, nthreads=0):
    X, Y = _f64(X), _f64(Y)
    n, d = X.shape
    m = Y.shape[0]
    bl = np.ascontiguousarray(blist, dtype=np.uint64)
    T, r1, r2 = np.zeros(bl.size), np.zeros(bl.size), np.zeros(bl.size)
    mo = np.zeros((bl.size, n_words(n + m)), dtype=np.uint32) if want_masks else None
    st = lib().oracle_perm_stats_at(_p(X), n, _p(Y), m, d, seed, pair, align, gd, _p(bl), bl.size,
                                    _p(T), _p(r1), _p(r2), _p(mo), nthreads)
    return dict(status=st, T=T, r1=r1, r2=r2, masks=mo)


def exhaustive(X, Y, align=1, gd=GD_BANERJEE, alternative=ALT_GREATER, want_T=False):
    from math import comb
    X, Y = _f64(X), _f64(Y)
    n, d = X.shape
    m = Y.shape[0]
    total = comb(n + m, n)
    out = np.zeros(9)
    T = np.zeros(total) if want_T else None
    st = lib().oracle_exhaustive(_p(X), n, _p(Y), m, d, align, gd, alternative, _p(out), _p(T),
                                 total if want_T else 0)
    return dict(status=st, t_obs=out[0], r_x=out[1], r_y=out[2], p=out[3], count=int(out[4]),
                h_identity=int(out[5]), tau=out[6], total=int(out[8]), T=T)
