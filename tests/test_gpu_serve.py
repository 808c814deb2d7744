"""The serving loop on the GPU: every request answered, bit-exact against the
oracle on a sample, and bit-identical to the same division served alone."""
import numpy as np
import pytest

import oracle
from paper_2606_06386_amd import inputs as I
from paper_2606_06386_amd import ragged as R

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2606_06386_amd import binding
    binding.lib()
    return binding


def test_serving_mix_equals_alone(mp):
    import torch
    from paper_2606_06386_amd import serve
    c = I.config_c5(1e5, count=300)
    res = serve.serve(c["u"], c["v"], c["arrival"], max_batch=64, depth=2)
    q, r, st = res["requests"].results()
    assert (st == 0).all()
    assert np.isfinite(res["latency"]).all() and (res["latency"] > 0).all()
    assert sum(res["batches"]) == 300 and len(res["batches"]) > 1
    # a sample against the oracle
    for j in range(0, 300, 23):
        qo, ro, so = oracle.divrem(c["u"][j][None, :], c["v"][j][None, :], nq=len(c["u"][j]), nr=len(c["v"][j]))
        assert so[0] == 0 and (q[j] == qo[0]).all() and (r[j] == ro[0]).all(), j
    # alone: a one-instance ragged batch and a one-instance uniform batch
    for j in range(0, 300, 37):
        rb = mp.Ragged(R.pack([c["u"][j]], [c["v"][j]]))
        rb.run()
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a[None, :]).view(np.int32)).cuda()
        qb, rbt, sb = mp.divrem(t(c["u"][j]), t(c["v"][j]))
        torch.cuda.synchronize()
        assert (rb.q.cpu().numpy().view(np.uint32)[:len(q[j])] == q[j]).all(), j
        assert (rb.r.cpu().numpy().view(np.uint32)[:len(r[j])] == r[j]).all(), j
        assert (qb.cpu().numpy().view(np.uint32)[0] == q[j]).all(), j
        assert (rbt.cpu().numpy().view(np.uint32)[0] == r[j]).all(), j
        assert sb.item() == 0


def test_plain_path_serves_the_same_answers(mp):
    """The plain per-width backend on the same trace: every request answered
    and equal to the ragged serving run's bits (and a sample to the oracle)."""
    from paper_2606_06386_amd import serve
    c = I.config_c5(1e5, count=200)
    a = serve.serve(c["u"], c["v"], c["arrival"], path="ragged", max_batch=48, depth=3)
    b = serve.serve(c["u"], c["v"], c["arrival"], path="plain", max_batch=48, depth=3)
    qa, ra, sa = a["requests"].results()
    qb, rb, sb = b["requests"].results()
    assert (sa == 0).all() and (sb == 0).all()
    assert all((x == y).all() for x, y in zip(qa, qb)) and all((x == y).all() for x, y in zip(ra, rb))
    for j in range(0, 200, 41):
        qo, ro, so = oracle.divrem(c["u"][j][None, :], c["v"][j][None, :], nq=len(c["u"][j]), nr=len(c["v"][j]))
        assert (qb[j] == qo[0]).all() and (rb[j] == ro[0]).all(), j
