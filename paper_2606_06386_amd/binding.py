"""Python binding of libmpdiv (include/mpdiv.h): argument marshalling only.

Every operation runs in the HIP kernels of libmpdiv.so; PyTorch provides the
device memory and the stream.  Numbers are torch tensors of shape
[batch, limbs] with dtype int32 or uint32 holding little-endian 32-bit limbs,
contiguous, on the GPU.  There is no CPU fallback: without the built library
or a GPU these calls raise.
"""
import ctypes
import os

import torch

from . import build as _build

MP_OK, MP_ERR_ARG, MP_ERR_SIZE, MP_ERR_LAUNCH, MP_ERR_DEVICE, MP_ERR_COUNT = range(6)
MP_STATIC_MAX_COUNT = 65536
MP_INST_OK, MP_INST_DIVZERO, MP_INST_QWIDTH, MP_INST_INTERNAL, MP_INST_BADDESC = range(5)

# every entry point declared in include/mpdiv.h
EXPORTS = ("mp_mul_batch", "mp_shinv_batch", "mp_divrem_batch", "mp_divrem_ragged", "mp_divrem_ragged_static",
           "mp_ragged_workspace_bytes",
           "mp_ragged_config", "mp_set_knob", "mp_get_knob", "mp_lds_bytes", "mp_status_str", "mp_max_limbs")
MP_KNOB_MFMA_MIN, MP_KNOB_SMALL_LIMIT = 0, 1
MP_SMALL_LIMIT_AUTO = -2          # the head limit chosen per launch
MP_OP_MUL, MP_OP_DIVREM, MP_OP_SHINV = 0, 1, 2

_lib = None
_vp, _i32 = ctypes.c_void_p, ctypes.c_int32


class MPError(RuntimeError):
    """A libmpdiv call returned an error status."""


def lib():
    """The loaded libmpdiv.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            raise RuntimeError(f"{_build.LIB} is not built: run paper_2606_06386_amd/build.py "
                               "(or __graft_entry__.build()) first")
        L = ctypes.CDLL(_build.LIB)
        L.mp_mul_batch.argtypes = [_vp, _i32, _vp, _i32, _vp, _i32, _vp]
        L.mp_shinv_batch.argtypes = [_vp, _i32, _i32, _vp, _i32, _vp, _i32, _vp]
        L.mp_divrem_batch.argtypes = [_vp, _i32, _vp, _i32, _vp, _i32, _vp, _vp, _i32, _vp]
        for f in (L.mp_mul_batch, L.mp_shinv_batch, L.mp_divrem_batch, L.mp_max_limbs):
            f.restype = _i32
        _i64 = ctypes.c_int64
        L.mp_divrem_ragged.argtypes = [_vp, _i64, _vp, _i64, _vp, _vp, _i64, _vp, _i64, _vp, _i32, _vp, _vp]
        L.mp_divrem_ragged.restype = _i32
        L.mp_divrem_ragged_static.argtypes = [_vp, _i64, _vp, _i64, _vp, _vp, _i64, _vp, _i64, _vp, _i32, _vp]
        L.mp_divrem_ragged_static.restype = _i32
        L.mp_ragged_workspace_bytes.argtypes = [_i32]
        L.mp_ragged_workspace_bytes.restype = _i64
        L.mp_ragged_config.argtypes = [_i32, _i32, _i32]
        L.mp_ragged_config.restype = _i32
        L.mp_set_knob.argtypes = [_i32, _i32]
        L.mp_set_knob.restype = _i32
        L.mp_get_knob.argtypes = [_i32]
        L.mp_get_knob.restype = _i32
        L.mp_lds_bytes.argtypes = [_i32, _i32, _i32]
        L.mp_lds_bytes.restype = _i64
        L.mp_max_limbs.argtypes = []
        L.mp_status_str.argtypes = [_i32]
        L.mp_status_str.restype = ctypes.c_char_p
        _lib = L
    return _lib


def max_limbs() -> int:
    return int(lib().mp_max_limbs())


def _limbs(t, name):
    if not isinstance(t, torch.Tensor) or t.dtype not in (torch.int32, torch.uint32):
        raise TypeError(f"{name}: expected an int32/uint32 torch tensor of limbs")
    if t.dim() == 1:
        t = t.unsqueeze(0)
    if t.dim() != 2 or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name}: expected a contiguous [batch, limbs] tensor on the GPU")
    return t


def _stream(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _raise(code, what):
    if code != MP_OK:
        raise MPError(f"{what}: {lib().mp_status_str(code).decode()}")


def mul(a, b, stream=None):
    """c = a * b per instance (c has na + nb limbs)."""
    a, b = _limbs(a, "a"), _limbs(b, "b")
    if a.shape[0] != b.shape[0]:
        raise ValueError("a and b must have the same batch size")
    c = torch.empty((a.shape[0], a.shape[1] + b.shape[1]), dtype=torch.int32, device=a.device)
    _raise(lib().mp_mul_batch(a.data_ptr(), a.shape[1], b.data_ptr(), b.shape[1], c.data_ptr(),
                              a.shape[0], _stream(stream)), "mp_mul_batch")
    return c


def shinv(v, h, nw=None, stream=None):
    """(w, status): w = floor(B^h / v) per instance, nw limbs (default h + 1)."""
    v = _limbs(v, "v")
    nw = h + 1 if nw is None else nw
    w = torch.empty((v.shape[0], nw), dtype=torch.int32, device=v.device)
    st = torch.empty(v.shape[0], dtype=torch.int32, device=v.device)
    _raise(lib().mp_shinv_batch(v.data_ptr(), v.shape[1], h, w.data_ptr(), nw, st.data_ptr(),
                                v.shape[0], _stream(stream)), "mp_shinv_batch")
    return w, st


def divrem(u, v, nq=None, out=None, stream=None):
    """(q, r, status) with u = q v + r, 0 <= r < v per instance.

    q has nq limbs (default: u's width), r has v's width.  ``out`` may supply
    preallocated (q, r, status) tensors."""
    u, v = _limbs(u, "u"), _limbs(v, "v")
    if u.shape[0] != v.shape[0]:
        raise ValueError("u and v must have the same batch size")
    batch = u.shape[0]
    if out is None:
        nq = u.shape[1] if nq is None else nq
        q = torch.empty((batch, nq), dtype=torch.int32, device=u.device)
        r = torch.empty((batch, v.shape[1]), dtype=torch.int32, device=u.device)
        st = torch.empty(batch, dtype=torch.int32, device=u.device)
    else:
        q, r, st = out
        nq = q.shape[1]
    _raise(lib().mp_divrem_batch(u.data_ptr(), u.shape[1], v.data_ptr(), v.shape[1], q.data_ptr(), nq,
                                 r.data_ptr(), st.data_ptr(), batch, _stream(stream)), "mp_divrem_batch")
    return q, r, st


class Ragged:
    """Device-resident ragged batch (pools, descriptors, outputs, workspace)
    built from ragged.pack(); run() launches mp_divrem_ragged."""

    def __init__(self, packed, device="cuda"):
        import numpy as np
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).to(device)
        self.count = len(packed["desc"])
        self.u = t(packed["u_pool"])
        self.v = t(packed["v_pool"])
        self.desc = torch.from_numpy(packed["desc"].view(np.uint8).copy()).to(device)
        self.q = torch.zeros(packed["q_limbs"], dtype=torch.int32, device=device)
        self.r = torch.zeros(packed["r_limbs"], dtype=torch.int32, device=device)
        self.status = torch.zeros(self.count, dtype=torch.int32, device=device)
        nb = int(lib().mp_ragged_workspace_bytes(self.count))
        self.ws = torch.zeros((nb + 3) // 4, dtype=torch.int32, device=device)

    def run(self, stream=None):
        _raise(lib().mp_divrem_ragged(self.u.data_ptr(), self.u.numel(), self.v.data_ptr(), self.v.numel(),
                                      self.desc.data_ptr(), self.q.data_ptr(), self.q.numel(), self.r.data_ptr(),
                                      self.r.numel(), self.status.data_ptr(), self.count, self.ws.data_ptr(),
                                      _stream(stream)), "mp_divrem_ragged")

    def run_static(self, stream=None):
        """The same batch through mp_divrem_ragged_static (no workspace)."""
        _raise(lib().mp_divrem_ragged_static(self.u.data_ptr(), self.u.numel(), self.v.data_ptr(), self.v.numel(),
                                             self.desc.data_ptr(), self.q.data_ptr(), self.q.numel(),
                                             self.r.data_ptr(), self.r.numel(), self.status.data_ptr(), self.count,
                                             _stream(stream)), "mp_divrem_ragged_static")


def set_knob(knob, value):
    """Set a run-time tuning knob (see mp_set_knob)."""
    _raise(lib().mp_set_knob(knob, value), "mp_set_knob")


def get_knob(knob):
    return int(lib().mp_get_knob(knob))


def lds_bytes(op, n1, n2):
    """Dynamic LDS bytes per workgroup of a launch (see mp_lds_bytes)."""
    return int(lib().mp_lds_bytes(op, n1, n2))


def ragged_config(cls, threads, wgs_per_cu):
    """Launch configuration of width class cls (see mp_ragged_config)."""
    _raise(lib().mp_ragged_config(cls, threads, wgs_per_cu), "mp_ragged_config")
