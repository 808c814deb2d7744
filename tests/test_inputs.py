"""The seeded input generator (shared by the oracle's tests and the GPU path's
tests/benchmark): published splitmix64 values, determinism, per-instance
regeneration, and the structure of the named workloads."""
import numpy as np

from paper_2606_06386_amd import inputs as I


def test_splitmix64_reference_sequence():
    # first outputs of splitmix64 started at state 0 (Vigna's reference code)
    want = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    got = [int(x) for x in I.draws(np.array([0], dtype=np.uint64), 0, 3)[0]]
    assert got == want


def test_instance_regenerates_alone():
    full = I.config_c2(batch=64)
    for j in (0, 3, 7, 11, 15, 19, 63):
        one = I.config_c2(index=[j])
        assert (one["u"][0] == full["u"][j]).all() and (one["v"][0] == full["v"][j]).all()
    c3 = I.config_c3(batch=8)
    one = I.config_c3(index=[5])
    assert (one["u"][0] == c3["u"][5]).all() and one["nv_eff"][0] == c3["nv_eff"][5]


def test_workload_shapes():
    c1 = I.config_c1()
    assert c1["u"].shape == (1024, 1024) and c1["v"].shape == (1024, 512)
    assert (c1["u"][:, -1] != 0).all() and (c1["v"][:, -1] != 0).all()
    c3 = I.config_c3(batch=32)
    nv = c3["nv_eff"]
    assert ((nv >= 2048) & (nv <= 8192)).all()
    for j in range(32):
        assert c3["v"][j, nv[j] - 1] != 0 and not c3["v"][j, nv[j]:].any()


def test_c2_adversarial_families():
    c = I.config_c2(batch=80)
    u, v = c["u"], c["v"]
    seen = set()
    for j in range(80):
        f = I.c2_family(j)
        seen.add(f)
        U, V = I.to_int(u[j]), I.to_int(v[j])
        if f == -1:
            assert u[j, -1] and v[j, -1]
        elif f == 0:
            assert V == (1 << (32 * 1024)) - 1
        elif f == 1:
            assert V == (1 << (32 * 1023)) + 1
        elif f == 2:
            assert v[j, -1] == 1
        elif f == 3:
            q, r = divmod(U, V)
            assert r == V - 1 and q.bit_length() <= 32 * 1023
        elif f == 4:
            assert U < V
    assert seen == {-1, 0, 1, 2, 3, 4}


def test_limb_conversions_roundtrip():
    x = (1 << 200) + 12345678901234567890
    assert I.to_int(I.from_int(x, 8)) == x


def test_config_c4_mixed_widths():
    """Mixed-precision workload: widths from the four classes, divisor lengths
    in [ceil(n/4), n], top limbs nonzero, any instance regenerable alone."""
    c = I.config_c4(count=256)
    assert set(int(n) for n in c["n"]) == set(I.C4_WIDTHS)
    for u, v, n, nv in zip(c["u"], c["v"], c["n"], c["nv"]):
        assert len(u) == n and len(v) == nv and (n + 3) // 4 <= nv <= n
        assert u[-1] != 0 and v[-1] != 0
    one = I.config_c4(index=[77])
    assert (one["u"][0] == c["u"][77]).all() and (one["v"][0] == c["v"][77]).all()


def test_ragged_pack_roundtrip():
    from paper_2606_06386_amd import ragged as R
    c = I.config_c4(count=40)
    p = R.pack(c["u"], c["v"])
    d = p["desc"]
    for f in ("u_off", "v_off", "q_off", "r_off"):
        assert (d[f] % 4 == 0).all()
    # ranges are disjoint and inside their pools
    for off, n, size in ((d["u_off"], d["nu"], len(p["u_pool"])), (d["q_off"], d["nq"], p["q_limbs"]),
                         (d["r_off"], d["nv"], p["r_limbs"])):
        order = np.argsort(off)
        ends = off[order] + n[order]
        assert (ends[:-1] <= off[order][1:]).all() and ends[-1] <= size
    us = R.unpack(p["u_pool"], np.rec.fromarrays([d["u_off"], d["nu"]], names="q_off,nq"), "q")
    assert all((a == b).all() for a, b in zip(us, c["u"]))
