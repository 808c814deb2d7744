"""Algorithmic work of the shifted-inverse division, in 32x32->64-bit limb products.

W(h, k) counts the limb products the method needs for one division with
h = prec(u) and k = prec(v) - 1 limbs: the products of every Refine iteration
of Alg. 1 (PowDiff's full or low product, Step's w*x) and the two products of
Alg. 3 (u * shinv, v * q), each at the operand sizes the iteration schedule
implies, with the full product where the paper says Mult and only the needed
low columns where it says MultMod.  Padding, guard rows and the quotient
corrections are not counted.

W_clipped(h, k) counts what the implementation computes: the Refine loop
with each Step product w*x formed only from column sh-2 (sh = H-2m, rounded
down to a multiple of 8) up, then only the columns of u * shinv from
c0 = h-2 (rounded likewise; the lower columns change floor(u s / B^h) by at
most one), and only the low k+2 columns of v * q (the remainder is within a
few v of u).

Schedule (Alg. 1, Refine; B = 2^32, g = 2 guard limbs): l starts at 2;
iteration i has m = min(h-k+1-l, l), s = max(0, k-2l+1-g), divisor prefix
v' = v >> s limbs (k+1-s limbs), iterate w with l+g limbs, PowDiff precision
h' = k+l-s+g and L = prec(v') + prec(w) - (l-g) + 1; the correction x has
about prec(v') limbs; after iteration i >= 2, l grows to l+m-1.
"""
import math


def low_product_cost(a: int, b: int, cols: int) -> int:
    """Limb products in the low `cols` columns of an a x b limb product."""
    n = 0
    for c in range(min(cols, a + b - 1)):
        n += min(c + 1, a, b, a + b - 1 - c)
    return n


def high_product_cost(a: int, b: int, c0: int) -> int:
    """Limb products in the columns >= c0 of an a x b limb product."""
    return a * b - low_product_cost(a, b, c0)


def iterations(h: int, k: int) -> int:
    d = h - k - 1
    return 2 + (math.ceil(math.log2(d)) if d > 1 else 0)


def refine_cost(h: int, k: int, clipped: bool = False) -> int:
    """Limb products of the Refine loop for B^k <= v < B^(k+1)."""
    g, l, w = 2, 2, 0
    total = 0
    for i in range(iterations(h, k)):
        m = min(h - k + 1 - l, l)
        s = max(0, k - 2 * l + 1 - g)
        nvp = k + 1 - s
        nw = l + g
        hp = k + l - s + g
        L = nvp + nw - (l - g) + 1
        total += nvp * nw if L >= hp else low_product_cost(nvp, nw, L)
        sh = k + l + m - s + g - 2 * m         # Step: w * x, x ~ prec(v') limbs
        cs = (max(sh - 2, 0) & ~7) if clipped and nw + nvp >= sh + 1 else 0
        total += high_product_cost(nw, nvp, cs)
        if i >= 2:
            l = l + m - 1
    return total


def division_cost(h: int, k: int) -> int:
    """W(h, k): limb products of one division (0 when u < v or v < B^1)."""
    if k <= 0 or h <= k:
        return 0
    d = h - k
    return refine_cost(h, k) + h * d + (k + 1) * d


def division_cost_clipped(h: int, k: int) -> int:
    """W_clipped(h, k): limb products of one division as implemented."""
    if k <= 0 or h <= k:
        return 0
    d = h - k
    c0 = max(h - 2, 0) & ~7
    return refine_cost(h, k, True) + high_product_cost(h, d, c0) + low_product_cost(k + 1, d, k + 2)


def shinv_cost(h: int, k: int) -> int:
    """Limb products of Alg. 1 alone (the Refine loop)."""
    if k <= 0 or h <= k:
        return 0
    return refine_cost(h, k)


def mul_cost(na: int, nb: int) -> int:
    return na * nb
