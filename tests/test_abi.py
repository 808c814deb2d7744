"""The C-ABI library (CPU only: no compute call is made here).

It loads, exports every entry point include/mpdiv.h declares, and rejects
invalid arguments on the host before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "mpdiv.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mp_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    from paper_2606_06386_amd import binding
    return binding.lib()


def test_exports_every_declared_symbol(L):
    names = _declared()
    assert set(names) == {"mp_mul_batch", "mp_shinv_batch", "mp_divrem_batch", "mp_divrem_ragged",
                          "mp_divrem_ragged_static",
                          "mp_ragged_workspace_bytes", "mp_ragged_config", "mp_set_knob", "mp_get_knob",
                          "mp_lds_bytes", "mp_status_str", "mp_max_limbs"}
    for n in names:
        assert hasattr(L, n), n
    from paper_2606_06386_amd import binding
    assert set(binding.EXPORTS) == set(names)


def test_limits_and_status_strings(L):
    assert L.mp_max_limbs() == 8192
    for code in range(6):
        assert L.mp_status_str(code).decode().startswith("MP_")


def test_host_argument_errors(L):
    from paper_2606_06386_amd.binding import MP_ERR_ARG, MP_ERR_SIZE, MP_OK
    p = ctypes.c_void_p(16)   # never dereferenced: every call below returns before a launch
    assert L.mp_divrem_batch(None, 4, p, 4, p, 4, p, None, 1, None) == MP_ERR_ARG
    assert L.mp_divrem_batch(p, 0, p, 4, p, 4, p, None, 1, None) == MP_ERR_ARG
    assert L.mp_divrem_batch(p, 4, p, 4, p, 0, p, None, 1, None) == MP_ERR_ARG
    assert L.mp_divrem_batch(p, 4, p, 4, p, 4, p, None, -1, None) == MP_ERR_ARG
    assert L.mp_divrem_batch(p, 8193, p, 4, p, 4, p, None, 1, None) == MP_ERR_SIZE
    assert L.mp_divrem_batch(p, 4, p, 4, p, 4, p, None, 0, None) == MP_OK
    assert L.mp_mul_batch(p, 4, None, 4, p, 1, None) == MP_ERR_ARG
    assert L.mp_mul_batch(p, 9000, p, 4, p, 1, None) == MP_ERR_SIZE
    assert L.mp_mul_batch(p, 4, p, 4, p, 0, None) == MP_OK
    assert L.mp_shinv_batch(p, 4, -1, p, 4, None, 1, None) == MP_ERR_ARG
    assert L.mp_shinv_batch(p, 4, 8193, p, 4, None, 1, None) == MP_ERR_SIZE
    assert L.mp_shinv_batch(p, 4, 10, p, 11, None, 0, None) == MP_OK
    # ragged batch: pointers and count are checked on the host
    assert L.mp_divrem_ragged(None, 4, p, 4, p, p, 4, p, 4, p, 1, p, None) == MP_ERR_ARG
    assert L.mp_divrem_ragged(p, 4, p, 4, p, p, 4, p, 4, None, 1, p, None) == MP_ERR_ARG
    assert L.mp_divrem_ragged(p, 4, p, 4, p, p, 4, p, 4, p, 1, None, None) == MP_ERR_ARG
    assert L.mp_divrem_ragged(p, 4, p, 4, p, p, 4, p, 4, p, -1, p, None) == MP_ERR_ARG
    assert L.mp_divrem_ragged(p, 4, p, 4, p, p, 4, p, 4, p, 0, p, None) == MP_OK
    # the no-allocation variant: same checks, and count beyond its static work queue
    from paper_2606_06386_amd.binding import MP_ERR_COUNT, MP_STATIC_MAX_COUNT
    assert L.mp_divrem_ragged_static(None, 4, p, 4, p, p, 4, p, 4, p, 1, None) == MP_ERR_ARG
    assert L.mp_divrem_ragged_static(p, 4, p, 4, p, p, 4, p, 4, None, 1, None) == MP_ERR_ARG
    assert L.mp_divrem_ragged_static(p, 4, p, 4, p, p, 4, p, 4, p, -1, None) == MP_ERR_ARG
    assert L.mp_divrem_ragged_static(p, 4, p, 4, p, p, 4, p, 4, p, MP_STATIC_MAX_COUNT + 1, None) == MP_ERR_COUNT
    assert L.mp_divrem_ragged_static(p, 4, p, 4, p, p, 4, p, 4, p, 0, None) == MP_OK
    assert L.mp_ragged_workspace_bytes(MP_STATIC_MAX_COUNT) == 4 * (16 + 4 * MP_STATIC_MAX_COUNT)
    assert L.mp_ragged_workspace_bytes(0) > 0
    assert L.mp_ragged_workspace_bytes(1000) >= 4 * 1000 * 4
    assert L.mp_ragged_config(4, 256, 1) == MP_ERR_ARG
    assert L.mp_ragged_config(0, 384, 1) == MP_ERR_ARG
    assert L.mp_ragged_config(3, 512, 1) == MP_ERR_ARG      # 8192 limbs need at least 1024 threads
    assert L.mp_ragged_config(0, 256, 0) == MP_ERR_ARG
    assert L.mp_ragged_config(0, 256, 9) == MP_ERR_ARG


def test_lds_plan_bounds(L):
    """The library's own LDS sizing (mp_lds_bytes, the figure every launch
    checks) fits gfx950's 160 KB per workgroup at every width up to 2^18 bits
    and grows with the width; wider launches are refused, not truncated."""
    from paper_2606_06386_amd.binding import MP_OP_DIVREM, MP_OP_MUL, MP_OP_SHINV
    lim = 160 * 1024
    prev = 0
    for nu in (64, 1024, 2048, 4096, 6000, 8192):
        b = L.mp_lds_bytes(MP_OP_DIVREM, nu, nu)
        assert prev < b <= lim, (nu, b)
        prev = b
        assert L.mp_lds_bytes(MP_OP_DIVREM, nu, 1) <= b
        assert 0 < L.mp_lds_bytes(MP_OP_SHINV, nu, nu) <= lim
    # the 2^16-bit workload keeps four workgroups per compute unit
    assert 4 * L.mp_lds_bytes(MP_OP_DIVREM, 2048, 1024) <= lim
    assert L.mp_lds_bytes(MP_OP_MUL, 8192, 6145) < L.mp_lds_bytes(MP_OP_MUL, 8192, 8192) <= lim
    for bad in ((MP_OP_DIVREM, 0, 4), (MP_OP_DIVREM, 8193, 4), (MP_OP_MUL, 4, 9000), (7, 4, 4)):
        assert L.mp_lds_bytes(*bad) == -1


def test_knobs(L):
    from paper_2606_06386_amd.binding import (MP_ERR_ARG, MP_KNOB_MFMA_MIN, MP_KNOB_SMALL_LIMIT, MP_OK,
                                              MP_SMALL_LIMIT_AUTO)
    m0, s0 = L.mp_get_knob(MP_KNOB_MFMA_MIN), L.mp_get_knob(MP_KNOB_SMALL_LIMIT)
    assert m0 >= 1 and (0 <= s0 <= 140 or s0 == MP_SMALL_LIMIT_AUTO)
    try:
        assert L.mp_set_knob(MP_KNOB_MFMA_MIN, 1 << 30) == MP_OK
        assert L.mp_get_knob(MP_KNOB_MFMA_MIN) == 1 << 30
        assert L.mp_set_knob(MP_KNOB_MFMA_MIN, 0) == MP_ERR_ARG
        assert L.mp_set_knob(MP_KNOB_SMALL_LIMIT, 141) == MP_ERR_ARG
        assert L.mp_set_knob(MP_KNOB_SMALL_LIMIT, -1) == MP_ERR_ARG
        assert L.mp_set_knob(MP_KNOB_SMALL_LIMIT, 140) == MP_OK
        assert L.mp_set_knob(MP_KNOB_SMALL_LIMIT, MP_SMALL_LIMIT_AUTO) == MP_OK
        assert L.mp_get_knob(MP_KNOB_SMALL_LIMIT) == MP_SMALL_LIMIT_AUTO
        assert L.mp_set_knob(9, 1) == MP_ERR_ARG and L.mp_get_knob(9) == -1
    finally:
        L.mp_set_knob(MP_KNOB_MFMA_MIN, m0)
        L.mp_set_knob(MP_KNOB_SMALL_LIMIT, s0)


def test_cost_model_values():
    from paper_2606_06386_amd import costmodel as cm
    # u*shinv and v*q are at least h*d + (k+1)*d; Refine adds less than both
    for h, k in [(1024, 511), (2048, 1023), (8192, 2047)]:
        d = h - k
        base = h * d + (k + 1) * d
        w = cm.division_cost(h, k)
        assert base < w < 2 * base
    assert cm.division_cost(2048, 1023) == 4391342
    assert cm.low_product_cost(3, 5, 7) == 15 and cm.low_product_cost(3, 5, 2) == 3
    assert cm.division_cost(10, 10) == 0 and cm.division_cost(10, 0) == 0


def test_cost_model_clipped():
    """Clipped products: column counts by enumeration on small shapes, and the
    quotient/remainder products roughly halved at 2^16 bits."""
    from paper_2606_06386_amd import costmodel as cm
    for a, b in [(3, 5), (7, 7), (9, 4), (1, 6)]:
        for c in range(a + b + 1):
            pairs = [(i, j) for i in range(a) for j in range(b)]
            assert cm.low_product_cost(a, b, c) == sum(1 for i, j in pairs if i + j < c)
            assert cm.high_product_cost(a, b, c) == sum(1 for i, j in pairs if i + j >= c)
    h, k = 2048, 1023
    d = h - k
    assert cm.division_cost_clipped(h, k) == 1777660
    assert cm.division_cost_clipped(h, k) - cm.refine_cost(h, k, True) < 0.6 * (h * d + (k + 1) * d)
    assert cm.refine_cost(h, k, True) < 0.6 * cm.refine_cost(h, k)
    assert cm.division_cost_clipped(10, 10) == 0
