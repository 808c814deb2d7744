"""mp_divrem_ragged_static (no workspace, no allocation) gives the same bits
as mp_divrem_ragged on the same batches, called twice in a row with the
second batch smaller than the first, both through the C ABI."""
import numpy as np
import pytest

import oracle
from paper_2606_06386_amd import inputs as I

pytestmark = pytest.mark.gpu


def _batch(mp, index):
    from paper_2606_06386_amd import ragged as R
    m = I.config_c4(index=index)
    return m, mp.Ragged(R.pack(m["u"], m["v"]))


def _results(rb):
    import torch
    torch.cuda.synchronize()
    return (rb.q.cpu().numpy().copy(), rb.r.cpu().numpy().copy(), rb.status.cpu().numpy().copy())


def test_static_equals_workspace_entry_point():
    import torch
    from paper_2606_06386_amd import binding as mp
    from paper_2606_06386_amd import ragged as R
    assert torch.cuda.is_available()
    for index in (np.arange(0, 1200), np.arange(5000, 5150)):    # second call: smaller batch
        m, rb = _batch(mp, index)
        rb.run()
        q1, r1, s1 = _results(rb)
        for t in (rb.q, rb.r, rb.status):
            t.fill_(-1)
        rb.run_static()
        q2, r2, s2 = _results(rb)
        assert (s1 == 0).all() and (s2 == s1).all()
        # every instance's rows (the pools' alignment gaps are nobody's output)
        desc = np.frombuffer(rb.desc.cpu().numpy().tobytes(), dtype=R.DESC_DTYPE)
        for a, b in ((q1, q2), (r1, r2)):
            which = "q" if a is q1 else "r"
            ra, rb_ = R.unpack(a.view(np.uint32), desc, which), R.unpack(b.view(np.uint32), desc, which)
            assert all((x == y).all() for x, y in zip(ra, rb_)), which
        # a few instances of each call against the oracle
        qs = R.unpack(q2.view(np.uint32), desc, "q")
        rs = R.unpack(r2.view(np.uint32), desc, "r")
        for j in range(0, len(index), max(1, len(index) // 6)):
            u, v = m["u"][j], m["v"][j]
            qo, ro, so = oracle.divrem(u[None, :], v[None, :], nq=len(u), nr=len(v))
            assert so[0] == 0 and (qs[j] == qo[0]).all() and (rs[j] == ro[0]).all(), j
