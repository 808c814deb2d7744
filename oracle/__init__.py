"""Oracle for batched multi-precision division -- TEST INFRASTRUCTURE ONLY.

A plain CPU implementation (``mpref.c``) of what the GPU path computes:
schoolbook multiplication, Knuth's Algorithm D for (q, r), and the shifted
inverse floor(B^h / v) by its definition (Definition 1 of the paper, Sec. 2.1).
Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package; the product path never does.

Arrays are numpy uint32 of shape [batch, limbs], little-endian limbs
(limb i has weight 2^(32 i)).
"""
import ctypes
import os

import numpy as np

from . import build as _build

REF_OK, REF_DIVZERO, REF_QWIDTH = 0, 1, 2

_lib = None
_u32p = ctypes.POINTER(ctypes.c_uint32)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i32 = ctypes.c_int32


def lib():
    """Load (building first if absent) the oracle library."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        L.ref_mul_batch.argtypes = [_u32p, _i32, _u32p, _i32, _u32p, _i32, _i32]
        L.ref_divrem_batch.argtypes = [_u32p, _i32, _u32p, _i32, _u32p, _i32,
                                       _u32p, _i32, _i32p, _i32, _i32]
        L.ref_shinv_batch.argtypes = [_u32p, _i32, _i32, _u32p, _i32, _i32p, _i32, _i32]
        for f in (L.ref_mul_batch, L.ref_divrem_batch, L.ref_shinv_batch):
            f.restype = _i32
        _lib = L
    return _lib


def _c(x):
    x = np.ascontiguousarray(x, dtype=np.uint32)
    if x.ndim == 1:
        x = x[None, :]
    return x


def _p(x, t=_u32p):
    return x.ctypes.data_as(t)


def mul(a, b, nthreads=0):
    """c = a * b per instance; c has na + nb limbs."""
    a, b = _c(a), _c(b)
    batch, na = a.shape
    nb = b.shape[1]
    assert b.shape[0] == batch
    c = np.zeros((batch, na + nb), dtype=np.uint32)
    lib().ref_mul_batch(_p(a), na, _p(b), nb, _p(c), batch, nthreads)
    return c


def divrem(u, v, nq=None, nr=None, nthreads=0):
    """(q, r, status) per instance with u = q v + r, 0 <= r < v."""
    u, v = _c(u), _c(v)
    batch, nu = u.shape
    nv = v.shape[1]
    assert v.shape[0] == batch
    nq = nu if nq is None else nq
    nr = nv if nr is None else nr
    q = np.zeros((batch, nq), dtype=np.uint32)
    r = np.zeros((batch, nr), dtype=np.uint32)
    st = np.zeros(batch, dtype=np.int32)
    lib().ref_divrem_batch(_p(u), nu, _p(v), nv, _p(q), nq, _p(r), nr,
                           _p(st, _i32p), batch, nthreads)
    return q, r, st


def divrem_threads(u, v, nq, nr, nthreads=0):
    """Like divrem, also returning the number of threads the batch used."""
    u, v = _c(u), _c(v)
    batch, nu = u.shape
    nv = v.shape[1]
    q = np.zeros((batch, nq), dtype=np.uint32)
    r = np.zeros((batch, nr), dtype=np.uint32)
    st = np.zeros(batch, dtype=np.int32)
    used = lib().ref_divrem_batch(_p(u), nu, _p(v), nv, _p(q), nq, _p(r), nr,
                                  _p(st, _i32p), batch, nthreads)
    return q, r, st, used


def shinv(v, h, nw=None, nthreads=0):
    """(w, status) with w = floor(B^h / v) per instance."""
    v = _c(v)
    batch, nv = v.shape
    nw = h + 1 if nw is None else nw
    w = np.zeros((batch, nw), dtype=np.uint32)
    st = np.zeros(batch, dtype=np.int32)
    lib().ref_shinv_batch(_p(v), nv, h, _p(w), nw, _p(st, _i32p), batch, nthreads)
    return w, st
