"""Parity of the HIP path (through the C ABI) with the oracle, bit-exact.

Every comparison is element by element on the same seeded inputs: products,
shifted inverses, quotients, remainders and per-instance status codes.
Sizes span several 256-column strips with ragged tails; the named workloads
run at their full batch in the launch configuration the benchmark times.
"""
import random

import numpy as np
import pytest

import oracle
from paper_2606_06386_amd import inputs as I

pytestmark = pytest.mark.gpu
B = 1 << 32


@pytest.fixture(scope="module")
def mp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2606_06386_amd import binding
    binding.lib()
    return binding


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.uint32).view(np.int32)).cuda()


def _host(t):
    return t.cpu().numpy().view(np.uint32)


def _divrem(mp, u, v, nq):
    import torch
    q, r, st = mp.divrem(_dev(u), _dev(v), nq=nq)
    torch.cuda.synchronize()
    return _host(q), _host(r), st.cpu().numpy()


def _expect_divrem(mp, u, v, nq, label):
    q, r, st = _divrem(mp, u, v, nq)
    qo, ro, so = oracle.divrem(u, v, nq=nq, nr=v.shape[1])
    bad = [j for j in range(len(u)) if st[j] != so[j] or (q[j] != qo[j]).any() or (r[j] != ro[j]).any()]
    assert not bad, f"{label}: {len(bad)} mismatching instances, first {bad[:8]}, status {st[bad[:8]]}"
    return q, r, st


def _rnd(rng, n):
    return rng.getrandbits(32 * n) | (1 << (32 * n - 1)) if n else 0


def _stack(vals, n):
    return np.stack([I.from_int(x, n) for x in vals])


# ------------------------------------------------------------------ mul

# Shapes chosen to reach every way the matrix-core product deals its strips
# to waves: strips W apart (fewer than two pairs per wave), adjacent pairs
# (at least two), an odd strip left alone, pairs whose diagonal ranges do not
# overlap (short operand of 64 limbs), at 256, 512 and 1024 threads.
@pytest.mark.parametrize("na,nb", [(1, 1), (2, 3), (5, 300), (300, 5), (257, 256), (256, 257), (700, 1300),
                                   (1024, 1024), (64, 2048), (2048, 1025), (4093, 3), (4096, 4096),
                                   (8192, 6145), (8192, 8192),
                                   (2048, 2048), (2047, 2049), (2048, 1999), (2048, 1700), (1500, 2048), (64, 4096),
                                   (3000, 4096), (4096, 2000), (5000, 8192), (64, 8192)])
def test_mul_matches_oracle(mp, na, nb):
    import torch
    rng = np.random.default_rng(na * 7919 + nb)
    batch = 3
    a = rng.integers(0, 2 ** 32, (batch, na), dtype=np.uint64).astype(np.uint32)
    b = rng.integers(0, 2 ** 32, (batch, nb), dtype=np.uint64).astype(np.uint32)
    a[1] = 0xFFFFFFFF                      # longest carry chains
    b[1] = 0xFFFFFFFF
    a[2, na // 2:] = 0                     # leading zero limbs
    c = mp.mul(_dev(a), _dev(b))
    torch.cuda.synchronize()
    assert (_host(c) == oracle.mul(a, b)).all()


# --------------------------------------------------------------- divrem

def test_divrem_random_sizes(mp):
    rng = random.Random(3)
    for nu in [2, 3, 4, 5, 7, 8, 9, 12, 17, 33, 64, 100, 255, 256, 257, 300, 513, 1000]:
        nvs = sorted({2, 3, nu // 2, nu - 1, nu} - {0, 1})
        for nv in nvs:
            us = [_rnd(rng, nu) for _ in range(8)]
            vs = [_rnd(rng, nv) for _ in range(8)]
            _expect_divrem(mp, _stack(us, nu), _stack(vs, nv), nu, f"random {nu}/{nv}")


def _structured_cases():
    rng = random.Random(11)
    cases = []
    for k in [1, 2, 3, 5, 7, 11, 19]:
        for h in range(k + 1, min(3 * k + 6, 40)):
            vs = [B ** k + 1, B ** k + 2, B ** k + B ** (k - 1), 2 * B ** k + 1, B ** (k + 1) - 1, B ** k,
                  3 * B ** k, B ** k + _rnd(rng, k), B ** (k + 1) // 2, B ** (k + 1) // 2 + 1,
                  B ** k * 0x80000000 + 1]
            for v in vs:
                if v.bit_length() > 32 * h:
                    continue
                for u in [B ** h - 1, _rnd(rng, h), v * _rnd(rng, max(1, h - k - 1)) + v - 1, v, v - 1, v + 1]:
                    if u.bit_length() <= 32 * h:
                        cases.append((u, v))
    return cases


def test_divrem_structured_divisors(mp):
    """Divisor families where the computed inverse is floor - 1 or floor + 1
    (B^k + 1, 2B^k + 1, ...), powers of B, B^(k+1) - 1, top limb 1 (a 65-bit
    initial approximation), 2v > B^h, with u = B^h - 1, v*w + v - 1, v, v+-1."""
    cases = _structured_cases()
    assert len(cases) > 5000
    u = _stack([c[0] for c in cases], 40)
    v = _stack([c[1] for c in cases], 40)
    _expect_divrem(mp, u, v, 40, "structured")


def test_divrem_edges_and_status(mp):
    rng = random.Random(5)
    cases = [(_rnd(rng, 30), 7), (_rnd(rng, 30), 0xFFFFFFFF), (_rnd(rng, 30), 1), (0, 5), (12345, 0),
             (_rnd(rng, 10), _rnd(rng, 20)), (_rnd(rng, 20), _rnd(rng, 20)), (B ** 25, B ** 25), (_rnd(rng, 5), 3),
             (_rnd(rng, 1), _rnd(rng, 1)), (0, 0), (B ** 39, 1), (B ** 40 - 1, B ** 40 - 1), (B ** 40 - 1, 2)]
    u = _stack([c[0] for c in cases], 40)
    v = _stack([c[1] for c in cases], 40)
    q, r, st = _expect_divrem(mp, u, v, 40, "edges")
    assert st[4] == oracle.REF_DIVZERO and st[10] == oracle.REF_DIVZERO
    # quotient width: nq too small for some instances
    cases = [(_rnd(rng, 30), _rnd(rng, 2)), (_rnd(rng, 30), _rnd(rng, 28)), (_rnd(rng, 30), 5), (_rnd(rng, 4), 9)]
    u = _stack([c[0] for c in cases], 30)
    v = _stack([c[1] for c in cases], 30)
    q, r, st = _expect_divrem(mp, u, v, 3, "qwidth")
    assert list(st) == [2, 0, 2, 2]       # quotients of 29, 3, 30 and 4 limbs


def test_divrem_small_values_in_wide_buffers(mp):
    """Tiny effective precisions inside 2^16 and 2^18-bit buffers: the same
    instances give the same results whatever the buffer (and workgroup) size."""
    rng = random.Random(8)
    us = [_rnd(rng, rng.randint(1, 60)) for _ in range(24)]
    vs = [_rnd(rng, rng.randint(1, 40)) for _ in range(24)]
    res = []
    for width in (64, 2048, 8192):
        q, r, st = _expect_divrem(mp, _stack(us, width), _stack(vs, width), width, f"width {width}")
        res.append((q[:, :64], r[:, :64]))
    for q, r in res[1:]:
        assert (q == res[0][0]).all() and (r == res[0][1]).all()


def test_divrem_2p15_full_batch(mp):
    c = I.config_c1()
    _expect_divrem(mp, c["u"], c["v"], c["nq"], c["name"])


def test_divrem_2p16_full_batch(mp):
    """The benchmark's workload, at its full batch, twice (a race shows as a
    difference between the runs)."""
    c = I.config_c2()
    q1, r1, _ = _expect_divrem(mp, c["u"], c["v"], c["nq"], c["name"])
    q2, r2, _ = _divrem(mp, c["u"], c["v"], c["nq"])
    assert (q1 == q2).all() and (r1 == r2).all()
    # the u = v*w + v - 1 family has the known answer (w, v - 1)
    for j in range(3 + 4 * 3, 200, 20):
        assert I.c2_family(j) == 3
        V = I.to_int(c["v"][j])
        assert (I.to_int(q1[j]) + 1) * V - 1 == I.to_int(c["u"][j]) and I.to_int(r1[j]) == V - 1


def test_divrem_2p18_full_batch(mp):
    c = I.config_c3()
    _expect_divrem(mp, c["u"], c["v"], c["nq"], c["name"])


def test_divrem_2p17_direct(mp):
    """Dividends of 4096 limbs (the 512-thread workgroup) against the oracle
    directly: random divisors of 1024..4096 limbs and the B^k + 1, 2B^k + 1
    families."""
    rng = random.Random(4096)
    n = 4096
    us, vs = [], []
    for i in range(48):
        k = rng.randint(1024, 4096)
        us.append(_rnd(rng, n))
        vs.append(_rnd(rng, k))
    for k in (1023, 1500, 2047, 3000, 4094):
        for v in (B ** k + 1, 2 * B ** k + 1):
            us.append(B ** n - 1)
            vs.append(v)
    for k in (1100, 2048, 3500):
        v = _rnd(rng, k)
        us.append(v * _rnd(rng, n - k) + v - 1)
        vs.append(v)
    _expect_divrem(mp, _stack(us, n), _stack(vs, n), n, "2^17 direct")


def test_divrem_2p18_structured(mp):
    """Full-depth Newton schedules at 2^18 bits with structured divisors."""
    n = 8192
    vals = []
    for k in (1, 2, 3, 100, 2047, 4095, 8190):
        for v in (B ** k + 1, 2 * B ** k + 1, B ** (k + 1) - 1, B ** k + B ** (k - 1)):
            vals.append((B ** n - 1, v))
    u = _stack([x for x, _ in vals], n)
    v = _stack([y for _, y in vals], n)
    _expect_divrem(mp, u, v, n, "2^18 structured")


# ---------------------------------------------------------------- shinv

def _expect_shinv(mp, v, h, nw, label):
    import torch
    w, st = mp.shinv(_dev(v), h, nw=nw)
    torch.cuda.synchronize()
    w, st = _host(w), st.cpu().numpy()
    wo, so = oracle.shinv(v, h, nw=nw)
    bad = [j for j in range(len(v)) if st[j] != so[j] or (w[j] != wo[j]).any()]
    assert not bad, f"{label}: mismatching instances {bad[:8]} status {st[bad[:8]]}"


def test_shinv_random(mp):
    rng = random.Random(21)
    for h in (1, 2, 3, 4, 7, 10, 33, 100, 513, 1024, 2048):
        for nv in sorted({1, 2, max(1, h // 2), h, h + 1}):
            vs = [_rnd(rng, nv) for _ in range(6)]
            _expect_shinv(mp, _stack(vs, nv + 1), h, h + 1, f"shinv h={h} nv={nv}")


def test_shinv_structured(mp):
    h = 40
    vals = []
    for k in range(0, 41):
        vals += [B ** k, B ** k + 1, 2 * B ** k + 1, B ** (k + 1) - 1, B ** k + B ** max(k - 1, 0)]
    vals += [B ** h // 2, B ** h // 2 + 1, B ** h, B ** h + 1, 0]
    v = _stack(vals, 42)
    _expect_shinv(mp, v, h, h + 1, "shinv structured")
    _expect_shinv(mp, v, h, 3, "shinv narrow output")


def test_shinv_2p16_and_2p18(mp):
    c = I.config_c2(batch=64)
    _expect_shinv(mp, c["v"], 2048, 1026, "shinv 2^16")
    c = I.config_c3(batch=16)
    _expect_shinv(mp, c["v"], 8192, 6146, "shinv 2^18")
