"""The error bounds behind clipped products, checked with exact integers.

A clipped product forms only the columns from c0 up.  With 32-bit limbs
(the vector-ALU product) the dropped part is non-negative and below
min(na, nb) B^(c0+1); with balanced radix-256 digits (the matrix-core
product, byte columns from 4 c0 up) it has either sign and stays below
2^17 c0 B^c0 in size.  Either way a shift by sh >= c0 + 2 limbs moves by at
most one, which is what lets the quotient estimate q0 = floor(u s / B^h),
with s within two of floor(B^h / v) and the columns of u s from (h-2) & ~7
up, land in [q - 4, q + 3] (so r0 = u - v q0 in [-3v, 5v)).  No part of
the library or the oracle is used: these are the inequalities themselves,
on random and structured operands (all-ones limbs, powers of B, B^k + 1)."""
import random

B = 1 << 32


def limbs(x, n):
    return [(x >> (32 * i)) & (B - 1) for i in range(n)]


def balanced_digits(x, n):
    """digits d_i in [-128, 127] with x = sum d_i 256^i (4n + 1 digits)"""
    d, c = [], 0
    for i in range(4 * n):
        b = ((x >> (8 * i)) & 255) + c
        if b >= 128:
            d.append(b - 256)
            c = 1
        else:
            d.append(b)
            c = 0
    d.append(c)
    return d


def clipped_limb_sum(a, na, b, nb, c0):
    al, bl = limbs(a, na), limbs(b, nb)
    return sum(x * y << (32 * (i + j)) for i, x in enumerate(al) for j, y in enumerate(bl) if i + j >= c0)


def clipped_digit_sum(a, na, b, nb, c0):
    ad, bd = balanced_digits(a, na), balanced_digits(b, nb)
    t = 0
    for i, x in enumerate(ad):
        if x:
            for j, y in enumerate(bd):
                if i + j >= 4 * c0:
                    t += (x * y) << (8 * (i + j))
    return t


def operands(rng, n):
    yield rng.getrandbits(32 * n) | 1 << (32 * n - 1)
    yield B ** n - 1
    yield B ** (n - 1)
    yield B ** (n - 1) + 1
    yield rng.getrandbits(32 * n) | 1 << (32 * n - 1)


def test_balanced_digits_represent_the_number():
    rng = random.Random(1)
    for n in (1, 2, 5, 9):
        for x in operands(rng, n):
            d = balanced_digits(x, n)
            assert all(-128 <= v <= 127 for v in d[:-1]) and d[-1] in (0, 1)
            assert sum(v << (8 * i) for i, v in enumerate(d)) == x


def test_dropped_columns_bounds():
    rng = random.Random(2)
    for na, nb in [(3, 5), (8, 8), (12, 5), (16, 20)]:
        for a in operands(rng, na):
            for b in operands(rng, nb):
                t = a * b
                for c0 in range(0, na + nb, 2):
                    dv = t - clipped_limb_sum(a, na, b, nb, c0)
                    assert 0 <= dv < min(na, nb) * B ** (c0 + 1)
                    dm = t - clipped_digit_sum(a, na, b, nb, c0)
                    assert abs(dm) < 2 ** 17 * max(c0, 1) * B ** c0
                    sh = c0 + 2
                    for tf in (t - dv, t - dm):
                        assert abs((tf >> (32 * sh)) - (t >> (32 * sh))) <= 1


def test_quotient_estimate_range():
    """s = floor(B^h / v) + lam, lam in -2..2, u s clipped from (h-2) & ~7:
    q0 = floor(formed / B^h) is within [q - 4, q + 3] on either engine."""
    rng = random.Random(3)
    for h, k in [(6, 3), (10, 5), (17, 8), (24, 11)]:
        vs = [B ** k + 1, 2 * B ** k + 1, B ** (k + 1) - 1, rng.getrandbits(32 * (k + 1)) | B ** k]
        for v in vs:
            for u in (B ** h - 1, rng.getrandbits(32 * h) | 1 << (32 * h - 1), v * (B ** (h - k - 1)) + v - 1):
                if u >= B ** h:
                    continue          # u must have h limbs
                q = u // v
                s0 = B ** h // v
                c0 = max(h - 2, 0) & ~7
                for lam in (-2, -1, 0, 1, 2):
                    s = s0 + lam
                    ns = (s.bit_length() + 31) // 32
                    for formed in (clipped_limb_sum(u, h, s, ns, c0), clipped_digit_sum(u, h, s, ns, c0)):
                        q0 = formed >> (32 * h)
                        assert q - 4 <= q0 <= q + 3
                        r0 = u - v * q0
                        assert -3 * v <= r0 < 5 * v and abs(r0) < B ** (k + 2) // 2
