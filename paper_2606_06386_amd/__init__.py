"""Batched exact multi-precision integer division on MI355X (gfx950).

The shifted-inverse Newton division of the paper (Algorithms 1-3): quotient
and remainder of u by v over little-endian 32-bit limbs, computed by
hand-written HIP kernels behind a C ABI (include/mpdiv.h).  This package is
the thin Python binding over that library; see ``binding`` for the calls.
"""
__all__ = ["mul", "shinv", "divrem", "max_limbs"]


def __getattr__(name):
    # The binding (and with it the HIP library) loads on first use, so that
    # ``paper_2606_06386_amd.inputs`` can be imported without a GPU library.
    if name in __all__:
        from . import binding
        return getattr(binding, name)
    raise AttributeError(name)
