"""Pins of the oracle (CPU only).

The oracle (``oracle/``) computes plain definitions: schoolbook products,
Knuth Algorithm D, and floor(B^h / v).  These tests tie it to things other
than itself:
  * native 128-bit division of the compiler runtime, exhaustively over an
    edge-value limb set and on random operands (``pin_int128.c``);
  * the worked examples printed in the paper (``golden/paper_examples.txt``);
  * CPython's big-integer ``divmod`` / ``*`` / ``//`` at every size up to
    8192 limbs (an independent library routine);
  * closed forms and the defining invariants;
  * planted mistakes: mutated copies of the oracle must fail the pins.
"""
import os
import random
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
from paper_2606_06386_amd import inputs as I

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
B = 1 << 32


def _build_pin(src_c, outdir):
    exe = os.path.join(outdir, "pin_int128")
    subprocess.run(["gcc", "-O2", "-I", os.path.join(ROOT, "oracle"), "-o", exe,
                    os.path.join(HERE, "pin_int128.c"), src_c], check=True)
    return exe


def test_pin_native_int128():
    with tempfile.TemporaryDirectory() as d:
        exe = _build_pin(os.path.join(ROOT, "oracle", "mpref.c"), d)
        out = subprocess.run([exe], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "failures 0" in out.stdout


# Plausible mistakes; each must be caught by the 128-bit pin.
MUTANTS = [
    ("drop the add-back step", "if (d >> 32) {", "if (0) {"),
    ("drop the second-limb qhat test",
     "while (qhat >= B || qhat * vn[n - 2] > ((rhat << 32) | un[j + n - 2])) {",
     "while (qhat >= B) {"),
    ("wrong limb in the qhat test", "| un[j + n - 2])) {", "| un[j + n - 1])) {"),
    ("wrong unnormalize shift", "(un[i + 1] << (32 - s))", "(un[i + 1] << s)"),
    ("short division keeps quotient as remainder", "rem = t % d;", "rem = t / d;"),
    ("u == v treated as u < v", "ref_cmp(u, v, n) < 0)", "ref_cmp(u, v, n) <= 0)"),
    ("B^h off by one limb", "bh[h] = 1;", "bh[h > 0 ? h - 1 : 0] = 1;"),
    ("product drops the final carry", "c[i + nb] = (uint32_t)carry;", "c[i + nb] = 0;"),
    ("borrow ignored in multiply-subtract",
     "uint64_t d = (uint64_t)un[i + j] - (p & 0xffffffffu) - borrow;",
     "uint64_t d = (uint64_t)un[i + j] - (p & 0xffffffffu);"),
]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistakes(name, old, new):
    src = open(os.path.join(ROOT, "oracle", "mpref.c")).read()
    assert src.count(old) == 1, name
    with tempfile.TemporaryDirectory() as d:
        shutil.copy(os.path.join(ROOT, "oracle", "mpref.h"), d)
        mut = os.path.join(d, "mpref.c")
        open(mut, "w").write(src.replace(old, new))
        exe = _build_pin(mut, d)
        out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode != 0, f"mutant '{name}' survived the pins"


def _golden():
    rows = []
    for line in open(os.path.join(HERE, "golden", "paper_examples.txt")):
        line = line.split("#")[0].split()
        if line:
            assert line[0] == "divrem"
            rows.append(tuple(int(x) for x in line[1:]))
    return rows


def test_paper_worked_examples():
    rows = _golden()
    assert len(rows) == 4
    for u, v, q, r in rows:
        q_, r_, st = oracle.divrem(I.from_int(u, 2)[None], I.from_int(v, 2)[None], nq=2, nr=2)
        assert st[0] == 0
        assert I.to_int(q_[0]) == q and I.to_int(r_[0]) == r


def _rand(rng, n):
    return rng.getrandbits(32 * n) | (1 << (32 * n - 1)) if n else 0


SIZES = [(1, 1), (2, 1), (2, 2), (3, 2), (5, 3), (17, 9), (64, 33), (255, 128),
         (1024, 512), (2048, 1024), (2048, 2), (4096, 4095), (8192, 2048), (8192, 7000)]


@pytest.mark.parametrize("nu,nv", SIZES)
def test_divrem_matches_python(nu, nv):
    rng = random.Random(nu * 10007 + nv)
    batch = 3 if nu >= 4096 else 6
    us = [_rand(rng, nu) for _ in range(batch)]
    vs = [_rand(rng, nv) for _ in range(batch)]
    u = np.stack([I.from_int(x, nu) for x in us])
    v = np.stack([I.from_int(x, nv) for x in vs])
    q, r, st = oracle.divrem(u, v, nq=nu, nr=nv)
    assert (st == 0).all()
    for j in range(batch):
        qq, rr = divmod(us[j], vs[j])
        assert I.to_int(q[j]) == qq and I.to_int(r[j]) == rr


@pytest.mark.parametrize("na,nb", [(1, 1), (3, 7), (100, 37), (1025, 2048), (8192, 6145)])
def test_mul_matches_python(na, nb):
    rng = random.Random(na * 31 + nb)
    xa, xb = rng.getrandbits(32 * na), rng.getrandbits(32 * nb)
    c = oracle.mul(I.from_int(xa, na), I.from_int(xb, nb))
    assert I.to_int(c[0]) == xa * xb


def test_mul_closed_forms():
    for n in (1, 2, 5, 64, 1000):
        ones = np.full((1, n), 0xFFFFFFFF, dtype=np.uint32)
        c = I.to_int(oracle.mul(ones, ones)[0])
        assert c == (1 << (64 * n)) - 2 * (1 << (32 * n)) + 1      # (B^n - 1)^2
        rng = random.Random(n)
        a = I.from_int(rng.getrandbits(32 * n), n)[None]
        one = I.from_int(1, 1)[None]
        assert I.to_int(oracle.mul(a, one)[0]) == I.to_int(a[0])
        b = I.from_int(rng.getrandbits(32 * n), n)[None]
        assert (oracle.mul(a, b) == oracle.mul(b, a)).all()


@pytest.mark.parametrize("h,nv", [(1, 1), (3, 2), (10, 6), (100, 40), (2048, 1024), (8192, 2048)])
def test_shinv_matches_python(h, nv):
    rng = random.Random(h + 7 * nv)
    vs = [_rand(rng, nv) for _ in range(4)]
    v = np.stack([I.from_int(x, nv) for x in vs])
    w, st = oracle.shinv(v, h)
    assert (st == 0).all()
    for j in range(4):
        assert I.to_int(w[j]) == (1 << (32 * h)) // vs[j]
        # defining invariant of floor(B^h / v): 0 <= B^h - v*w < v
        d = (1 << (32 * h)) - vs[j] * I.to_int(w[j])
        assert 0 <= d < vs[j]


def test_shinv_closed_forms():
    h = 12
    cases = []
    for k in range(0, 13):                         # v = B^k  ->  B^(h-k)  (Alg. 1 special case)
        cases.append(((1 << (32 * k)), 1 << (32 * (h - k))))
    cases.append((1, 1 << (32 * h)))               # shinv_h(1) = B^h
    cases.append((2, 1 << (32 * h - 1)))           # shinv_h(2) = 2^(32h-1)
    for k in range(1, 8):                          # v = B^k - 1  ->  sum_{j=1}^{h div k} B^(h-jk)
        cases.append(((1 << (32 * k)) - 1, sum(1 << (32 * (h - j * k)) for j in range(1, h // k + 1))))
    cases.append(((1 << (32 * h)) + 1, 0))         # v > B^h -> 0
    cases.append(((1 << (32 * h)) // 2 + 1, 1))    # B^h/2 < v <= B^h -> 1
    cases.append(((1 << (32 * h)), 1))
    nv = h + 1
    v = np.stack([I.from_int(c[0], nv) for c in cases])
    w, st = oracle.shinv(v, h)
    assert (st == 0).all()
    for j, (_, want) in enumerate(cases):
        assert I.to_int(w[j]) == want, j


def test_divrem_closed_forms_and_edges():
    rng = random.Random(5)
    n = 40
    cases = []
    vv = _rand(rng, 20)
    ww = _rand(rng, 19)
    cases.append((vv * ww + vv - 1, vv, ww, vv - 1))                 # u = v*w + v - 1
    cases.append((vv - 5, vv, 0, vv - 5))                            # u < v
    k = 19
    cases.append(((1 << (64 * k)) - 1, (1 << (32 * k)) + 1, (1 << (32 * k)) - 1, 0))  # B^2k-1 = (B^k+1)(B^k-1)
    x = _rand(rng, 33)
    cases.append((x, 1, x, 0))                                       # divide by 1
    cases.append((x, x, 1, 0))                                       # divide by itself
    cases.append((0, vv, 0, 0))                                      # zero dividend
    cases.append((x, 1 << (32 * 7), x >> (32 * 7), x & ((1 << (32 * 7)) - 1)))  # v = B^7
    u = np.stack([I.from_int(c[0], n) for c in cases])
    v = np.stack([I.from_int(c[1], n) for c in cases])
    q, r, st = oracle.divrem(u, v)
    for j, (_, _, qq, rr) in enumerate(cases):
        assert st[j] == 0 and I.to_int(q[j]) == qq and I.to_int(r[j]) == rr, j


def test_divrem_status_codes():
    u = I.from_int(12345, 4)[None]
    q, r, st = oracle.divrem(u, np.zeros((1, 4), dtype=np.uint32))
    assert st[0] == oracle.REF_DIVZERO and not q.any() and not r.any()
    big = I.from_int((1 << 100) + 3, 4)[None]
    q, r, st = oracle.divrem(big, I.from_int(3, 4)[None], nq=2)      # quotient needs 3+ limbs
    assert st[0] == oracle.REF_QWIDTH and not q.any() and not r.any()


def test_invariants_on_workload_samples():
    """q*v + r = u and 0 <= r < v (which determine (q, r) uniquely), checked
    with CPython arithmetic on samples of the 2^15, 2^16 and 2^18-bit workloads."""
    c1 = I.config_c1()
    c2 = I.config_c2(index=np.arange(0, 4096, 97))
    c3 = I.config_c3(index=np.array([0, 1, 100, 255]))
    for c in (c1, c2, c3):
        sel = np.arange(min(len(c["u"]), 12))
        u, v = c["u"][sel], c["v"][sel]
        q, r, st = oracle.divrem(u, v, nq=c["nq"])
        assert (st == 0).all()
        for j in range(len(sel)):
            U, V, Q, R = (I.to_int(x[j]) for x in (u, v, q, r))
            assert Q * V + R == U and 0 <= R < V
