"""Ragged (mixed-precision) batches through mp_divrem_ragged, bit-exact.

Each instance is checked against the oracle and against the uniform-batch
entry point on the same operands; descriptors that leave their pools are
rejected per instance without writing; the launch sequence replays from a
captured graph with the same results.
"""
import numpy as np
import pytest

import oracle
from paper_2606_06386_amd import inputs as I
from paper_2606_06386_amd import ragged as R

pytestmark = pytest.mark.gpu
CANARY = 0xA5A5A5A5
CANARY_I32 = CANARY - (1 << 32)     # the same bits as an int32 fill value


@pytest.fixture(scope="module")
def mp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2606_06386_amd import binding
    binding.lib()
    return binding


def _run(mp, us, vs, nqs=None, fill=CANARY):
    import torch
    packed = R.pack(us, vs, nqs)
    rb = mp.Ragged(packed)
    rb.q.fill_(fill - (1 << 32) if fill >= (1 << 31) else fill)
    rb.r.fill_(fill - (1 << 32) if fill >= (1 << 31) else fill)
    rb.status.fill_(-1)
    rb.run()
    torch.cuda.synchronize()
    q = rb.q.cpu().numpy().view(np.uint32)
    r = rb.r.cpu().numpy().view(np.uint32)
    return packed, rb, R.unpack(q, packed["desc"], "q"), R.unpack(r, packed["desc"], "r"), rb.status.cpu().numpy()


def _oracle_one(u, v, nq):
    qo, ro, so = oracle.divrem(u[None, :], v[None, :], nq=nq, nr=len(v))
    return qo[0], ro[0], int(so[0])


def _check(us, vs, nqs, q, r, st, label):
    bad = []
    for j, (u, v) in enumerate(zip(us, vs)):
        qo, ro, so = _oracle_one(u, v, nqs[j])
        if st[j] != so or (q[j] != qo).any() or (r[j] != ro).any():
            bad.append(j)
    assert not bad, f"{label}: {len(bad)} mismatching instances, first {bad[:8]}, status {st[bad[:8]]}"


def test_ragged_c4_sample_vs_oracle(mp):
    """A sample of the mixed-precision workload (all four width classes)."""
    c = I.config_c4(index=np.arange(0, 8192, 128))
    nqs = [len(u) for u in c["u"]]
    _, _, q, r, st = _run(mp, c["u"], c["v"])
    assert sorted(set(len(u) for u in c["u"])) == [1024, 2048, 4096, 8192]
    _check(c["u"], c["v"], nqs, q, r, st, "C4 sample")
    assert (st == 0).all()


def test_ragged_equals_uniform_batches(mp):
    """Per class, the ragged result equals the uniform-batch entry point's."""
    import torch
    c = I.config_c4(index=np.arange(40))
    _, _, q, r, st = _run(mp, c["u"], c["v"])
    for n in I.C4_WIDTHS:
        js = [j for j, u in enumerate(c["u"]) if len(u) == n]
        if not js:
            continue
        nv = max(len(c["v"][j]) for j in js)
        u = np.stack([c["u"][j] for j in js])
        v = np.zeros((len(js), nv), dtype=np.uint32)
        for i, j in enumerate(js):
            v[i, :len(c["v"][j])] = c["v"][j]
        t = lambda a: torch.from_numpy(a.view(np.int32)).cuda()
        qb, rb, sb = mp.divrem(t(u), t(v), nq=n)
        torch.cuda.synchronize()
        qb, rb = qb.cpu().numpy().view(np.uint32), rb.cpu().numpy().view(np.uint32)
        for i, j in enumerate(js):
            assert (q[j] == qb[i]).all(), (n, j)
            assert (r[j] == rb[i, :len(c["v"][j])]).all() and not rb[i, len(c["v"][j]):].any(), (n, j)
            assert st[j] == sb[i].item()


def test_ragged_edge_instances(mp):
    """Degenerate instances mixed with ordinary ones: v = 0, u < v, u = 0,
    divisor wider than dividend, single-limb and power-of-B divisors, widths
    that are not multiples of 4, a quotient buffer too narrow."""
    rng = np.random.default_rng(7)
    top = lambda n: np.concatenate([rng.integers(0, 2**32, n - 1, dtype=np.uint64).astype(np.uint32),
                                    np.array([rng.integers(1, 2**32)], dtype=np.uint32)])
    us, vs, nqs = [], [], []
    def add(u, v, nq=None):
        us.append(np.asarray(u, dtype=np.uint32))
        vs.append(np.asarray(v, dtype=np.uint32))
        nqs.append(len(u) if nq is None else nq)
    add(top(1500), np.zeros(700, dtype=np.uint32))                   # v = 0
    add(top(301), top(302))                                          # u < v, divisor wider
    add(np.zeros(9, dtype=np.uint32), top(3))                        # u = 0
    add(top(2049), top(1))                                           # single limb divisor
    p = np.zeros(600, dtype=np.uint32); p[599] = 1
    add(top(3001), p)                                                # v = B^599
    add(top(8192), top(8191))                                        # widest class, q of 2 limbs
    add(top(1025), top(5), nq=4)                                     # quotient needs more than 4 limbs
    add(top(7), top(3))                                              # tiny
    add(top(4097), top(2049))                                        # class boundary + 1
    add(top(1024), top(1024))
    _, _, q, r, st = _run(mp, us, vs, nqs)
    _check(us, vs, nqs, q, r, st, "edges")
    assert list(st[:1]) == [1] and st[6] == 2


def test_ragged_bad_descriptors(mp):
    """Descriptors whose ranges leave their pools, or whose widths are out of
    range, get MP_INST_BADDESC and leave their outputs unwritten; the other
    instances of the batch are computed."""
    import torch
    c = I.config_c4(index=np.arange(6))
    packed = R.pack(c["u"], c["v"])
    d = packed["desc"]
    d["u_off"][1] = len(packed["u_pool"]) - d["nu"][1] + 1        # u leaves its pool
    d["nv"][2] = 0                                                 # zero-width divisor
    d["q_off"][3] = packed["q_limbs"] - 2                          # q leaves its pool
    d["r_off"][4] = -4                                             # negative offset
    rb = mp.Ragged(packed)
    rb.q.fill_(CANARY_I32)
    rb.r.fill_(CANARY_I32)
    rb.status.fill_(-1)
    rb.run()
    torch.cuda.synchronize()
    st = rb.status.cpu().numpy()
    assert list(st[1:5]) == [4, 4, 4, 4]
    assert st[0] == 0 and st[5] == 0
    q = R.unpack(rb.q.cpu().numpy().view(np.uint32), packed["desc"], "q")
    r = R.unpack(rb.r.cpu().numpy().view(np.uint32), packed["desc"], "r")
    for j in (0, 5):
        qo, ro, _ = _oracle_one(c["u"][j], c["v"][j], len(c["u"][j]))
        assert (q[j] == qo).all() and (r[j] == ro).all()
    for j in (1, 2):          # their output ranges are still inside the pools
        assert (q[j] == CANARY).all()


def test_ragged_single_class_and_empty(mp):
    """A batch with one class only, and an empty batch."""
    import torch
    rng = np.random.default_rng(11)
    us = [np.append(rng.integers(0, 2**32, 2047, dtype=np.uint64).astype(np.uint32), np.uint32(5)) for _ in range(9)]
    vs = [np.append(rng.integers(0, 2**32, 999, dtype=np.uint64).astype(np.uint32), np.uint32(3)) for _ in range(9)]
    _, _, q, r, st = _run(mp, us, vs)
    _check(us, vs, [2048] * 9, q, r, st, "one class")
    p = torch.zeros(4, dtype=torch.int32, device="cuda")
    assert mp.lib().mp_divrem_ragged(p.data_ptr(), 4, p.data_ptr(), 4, p.data_ptr(), p.data_ptr(), 4, p.data_ptr(),
                                     4, p.data_ptr(), 0, p.data_ptr(), None) == 0


def test_ragged_graph_replay(mp):
    """The whole launch sequence (bucketing + class kernels on forked streams)
    captured once and replayed three times, with eager work and
    synchronisation between replays; each replay matches the eager result."""
    import torch
    c = I.config_c4(index=np.arange(100, 164))
    packed = R.pack(c["u"], c["v"])
    rb = mp.Ragged(packed)
    rb.run()
    torch.cuda.synchronize()
    q0, r0, s0 = rb.q.clone(), rb.r.clone(), rb.status.clone()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        rb.run()                         # the stream's fork set exists before capture
        with torch.cuda.graph(g, stream=s):
            rb.run()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for rep in range(3):
        rb.q.zero_()
        rb.r.zero_()
        rb.status.fill_(-1)
        x = torch.arange(1 << 20, device="cuda").sum()           # unrelated eager work
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert x.item() == (1 << 20) * ((1 << 20) - 1) // 2
        assert torch.equal(rb.q, q0) and torch.equal(rb.r, r0) and torch.equal(rb.status, s0), rep


def test_tuner_configs_give_identical_results(mp, tmp_path):
    """The autotuner picks a valid configuration per class and caches it; the
    results of a mixed batch do not depend on the launch configuration."""
    import torch
    from paper_2606_06386_amd import tune
    c = I.config_c4(index=np.arange(200, 248))
    packed = R.pack(c["u"], c["v"])
    outs = []
    for cfg in ([(256, 1), (256, 1), (512, 1), (1024, 1)], [(1024, 8), (512, 2), (1024, 3), (1024, 2)]):
        for cls, (t, g) in enumerate(cfg):
            mp.ragged_config(cls, t, g)
        rb = mp.Ragged(packed)
        rb.run()
        torch.cuda.synchronize()
        outs.append((rb.q.cpu().numpy().copy(), rb.r.cpu().numpy().copy(), rb.status.cpu().numpy().copy()))
    assert all((a == b).all() for a, b in zip(outs[0], outs[1]))
    with pytest.raises(mp.MPError):
        mp.ragged_config(3, 512, 1)                 # 8192 limbs need 1024 threads
    best = tune.tune(counts=(32, 16, 8, 4), reps=1)
    assert set(best) == {0, 1, 2, 3}
    for cls, (t, g, ms) in best.items():
        assert (t, g) in tune.candidates(cls) and ms > 0
    cache = tmp_path / "tuned.json"
    entry, fresh = tune.ensure(cache=str(cache))
    assert fresh and cache.exists()
    kn = entry["knobs"]
    assert kn["small_limit"] in tune.SMALL_LIMITS and kn["mfma_min"] in tune.MFMA_MINS
    assert mp.get_knob(mp.MP_KNOB_SMALL_LIMIT) == kn["small_limit"]
    entry2, fresh2 = tune.ensure(cache=str(cache))
    assert not fresh2 and entry2 == entry


def test_ragged_graph_of_a_fresh_stream(mp):
    """Captured on a stream the library has not seen: the class kernels run in
    order inside the graph, with the same results."""
    import torch
    c = I.config_c4(index=np.arange(300, 340))
    rb = mp.Ragged(R.pack(c["u"], c["v"]))
    rb.run()
    torch.cuda.synchronize()
    q0, r0, s0 = rb.q.clone(), rb.r.clone(), rb.status.clone()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            rb.run()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for rep in range(2):
        rb.q.zero_()
        rb.r.zero_()
        rb.status.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(rb.q, q0) and torch.equal(rb.r, r0) and torch.equal(rb.status, s0), rep
