"""Every launch configuration gives the oracle's bits.

The run-time knobs choose where the work runs (the head launch for the
early Refine iterations, or the per-instance workgroups for all of them;
products on the matrix cores or on the vector ALU), never what is computed:
each setting is compared element by element with the oracle on structured
divisors and on samples of the named workloads, through the C ABI."""
import random

import numpy as np
import pytest

import oracle
from paper_2606_06386_amd import inputs as I

pytestmark = pytest.mark.gpu
B = 1 << 32

# (small_limit, mfma_min): default, no head, short and long head iterations,
# products on the vector ALU only, matrix cores from 16-limb operands
SETTINGS = [(64, 64), (0, 64), (16, 64), (128, 64), (140, 64), (64, 1 << 20), (136, 16)]


@pytest.fixture(scope="module")
def mp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2606_06386_amd import binding
    binding.lib()
    return binding


@pytest.fixture
def knobs(mp):
    old = (mp.get_knob(mp.MP_KNOB_SMALL_LIMIT), mp.get_knob(mp.MP_KNOB_MFMA_MIN))

    def set_(small, mfma):
        mp.set_knob(mp.MP_KNOB_SMALL_LIMIT, small)
        mp.set_knob(mp.MP_KNOB_MFMA_MIN, mfma)
    yield set_
    set_(*old)


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.uint32).view(np.int32)).cuda()


def _check(mp, u, v, nq, label):
    import torch
    q, r, st = mp.divrem(_dev(u), _dev(v), nq=nq)
    torch.cuda.synchronize()
    q, r, st = q.cpu().numpy().view(np.uint32), r.cpu().numpy().view(np.uint32), st.cpu().numpy()
    qo, ro, so = oracle.divrem(u, v, nq=nq, nr=v.shape[1])
    bad = [j for j in range(len(u)) if st[j] != so[j] or (q[j] != qo[j]).any() or (r[j] != ro[j]).any()]
    info = [(j, int(st[j]), int(so[j]), int(np.argmax(q[j] != qo[j])) if (q[j] != qo[j]).any() else -1)
            for j in bad[:6]]
    assert not bad, f"{label}: {len(bad)} mismatching instances (index, status, expected, first bad q limb) {info}"


def _structured(width):
    rng = random.Random(17)
    rnd = lambda n: rng.getrandbits(32 * n) | (1 << (32 * n - 1))
    vals = []
    for k in (1, 2, 5, 11, 19, 40, 70, 130, 300):
        if k + 2 > width:
            continue
        h = min(width, 2 * k + 30 + k // 2)
        for v in (B ** k + 1, 2 * B ** k + 1, B ** (k + 1) - 1, B ** k + B ** (k - 1), B ** k * 0x80000000 + 1,
                  B ** k + rnd(k)):
            for u in (B ** h - 1, v * rnd(max(1, h - k - 1)) + v - 1, rnd(h)):
                if u.bit_length() <= 32 * width:
                    vals.append((u, v))
    return (np.stack([I.from_int(a, width) for a, _ in vals]), np.stack([I.from_int(b, width) for _, b in vals]))


@pytest.mark.parametrize("small,mfma", SETTINGS)
def test_structured_every_setting(mp, knobs, small, mfma):
    knobs(small, mfma)
    u, v = _structured(512)
    _check(mp, u, v, 512, f"structured small={small} mfma={mfma}")
    # a quotient row too short for a head record: the per-instance workgroups do every step
    _check(mp, u[:, :40], np.where(np.arange(512)[None, :] < 40, v, 0)[:, :40], 12, "narrow q")


@pytest.mark.parametrize("small,mfma", SETTINGS)
def test_workload_samples_every_setting(mp, knobs, small, mfma):
    knobs(small, mfma)
    i = np.arange(256)
    c = I.config_c2(index=16 * i + i % 4)              # 256 instances: random and all five adversarial families
    _check(mp, c["u"], c["v"], c["nq"], f"2^16 sample small={small} mfma={mfma}")
    c = I.config_c3(index=np.arange(0, 256, 32))        # 8 instances at 2^18 bits
    _check(mp, c["u"], c["v"], c["nq"], f"2^18 sample small={small} mfma={mfma}")


@pytest.mark.parametrize("small", [0, 64, 128])
def test_shinv_every_head_setting(mp, knobs, small):
    import torch
    knobs(small, 64)
    vals = []
    for k in (1, 3, 10, 33, 64, 100, 200):
        vals += [B ** k + 1, 2 * B ** k + 1, B ** (k + 1) - 1, B ** k + B ** (k - 1), B ** k + 12345]
    v = np.stack([I.from_int(x, 202) for x in vals])
    for h in (40, 150, 400):
        w, st = mp.shinv(_dev(v), h, nw=h + 1)
        torch.cuda.synchronize()
        wo, so = oracle.shinv(v, h, nw=h + 1)
        assert (st.cpu().numpy() == so).all()
        assert (w.cpu().numpy().view(np.uint32) == wo).all(), f"shinv h={h} small={small}"


def test_auto_head_limit_both_sides_of_one_round(mp, knobs):
    """The automatic head limit picks 96 limbs for a batch whose bodies fit in
    one round of workgroups and 136 for a larger one; batches just below and
    just above that size give the oracle's bits, as do both fixed limits."""
    import torch
    slots = 4 * torch.cuda.get_device_properties(0).multi_processor_count   # body workgroups per round at 2^16 bits
    for count in (slots, slots + 1):
        i = np.arange(count)
        c = I.config_c2(index=i)
        for small in (mp.MP_SMALL_LIMIT_AUTO, 96, 136):
            knobs(small, 64)
            _check(mp, c["u"], c["v"], c["nq"], f"2^16 batch {count} small={small}")


@pytest.mark.parametrize("small", ["auto", 140, 64, 24])
def test_head_register_iterations_every_boundary(mp, knobs, small):
    """The head runs a Refine iteration in registers (one limb per lane) while
    v', the iterate, PowDiff's product and residual, the Step product and the
    new iterate all fit 64 limbs, and passes through LDS after that; divisor
    lengths 2..71 limbs and quotient lengths 2..130 limbs put the switch at
    every iteration, with random and structured divisors."""
    knobs(mp.MP_SMALL_LIMIT_AUTO if small == "auto" else small, 64)
    rng = random.Random(23)
    width = 208
    us, vs = [], []
    for k in range(1, 71, 3):
        for d in (2, 3, 5, 9, 17, 33, 65, 130):
            if k + 1 + d > width:
                continue
            for v in (rng.getrandbits(32 * (k + 1)) | (1 << (32 * (k + 1) - 1)), B ** k + 1, B ** (k + 1) - 1):
                u = rng.getrandbits(32 * (k + d)) | (1 << (32 * (k + d) - 1))
                us.append(u)
                vs.append(v)
    u = np.stack([I.from_int(a, width) for a in us])
    v = np.stack([I.from_int(b, width) for b in vs])
    _check(mp, u, v, width, f"head boundary sweep small={small}")
