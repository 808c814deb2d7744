"""Host logic of the serving loop (no GPU): admission, ordering, depth,
nothing dropped, oversized requests admitted alone."""
import numpy as np

from paper_2606_06386_amd import inputs as I
from paper_2606_06386_amd.serve import Scheduler


class FakeClock:
    def __init__(self, dt=1e-5):
        self.t, self.dt = 0.0, dt

    def __call__(self):
        self.t += self.dt
        return self.t


class FakeBackend:
    """Batches take a fixed time per limb; records every launch."""

    def __init__(self, clock, nlimbs, per_limb=1e-8, depth=2):
        self.clock, self.nlimbs, self.per_limb = clock, nlimbs, per_limb
        self.launches, self.depth, self.busy_until = [], depth, 0.0
        self.inflight = 0
        self.max_inflight = 0

    def launch(self, slot, ids):
        start = max(self.clock.t, self.busy_until)       # batches run one after another
        end = start + self.per_limb * float(np.sum(self.nlimbs[ids]))
        self.busy_until = end
        self.launches.append((slot, list(ids), self.clock.t))
        self.inflight += 1
        self.max_inflight = max(self.max_inflight, self.inflight)
        return [end, False]

    def done(self, h):
        if not h[1] and self.clock.t >= h[0]:
            h[1] = True
            self.inflight -= 1
        return h[1]


def _serve(arrival, nlimbs, max_batch, max_limbs, depth):
    clock = FakeClock()
    be = FakeBackend(clock, np.asarray(nlimbs), depth=depth)
    sch = Scheduler(be, {"limbs": (nlimbs, max_limbs)}, max_batch=max_batch, depth=depth)
    done_at, sizes, launch_s = sch.run(arrival, clock=clock)
    assert launch_s >= 0
    return be, sch, done_at, sizes


def test_every_request_served_once_in_arrival_order():
    rng = np.random.default_rng(1)
    arrival = np.cumsum(rng.exponential(1e-4, 500))
    nlimbs = rng.integers(1024, 8193, 500)
    be, sch, done_at, sizes = _serve(arrival, nlimbs, max_batch=64, max_limbs=100000, depth=2)
    ids = [j for _, b, _ in be.launches for j in b]
    assert sorted(ids) == list(range(500))
    assert ids == sorted(ids, key=lambda j: arrival[j])         # FIFO by arrival
    assert not np.isnan(done_at).any() and (done_at >= arrival).all()
    assert be.max_inflight <= 2
    for _, b, t in be.launches:
        assert len(b) <= 64 and (sum(nlimbs[b]) <= 100000 or len(b) == 1)
        assert (arrival[b] <= t + 1e-12).all()                  # launched only after arriving
    assert sum(sizes) == 500


def test_oversized_request_waits_then_is_admitted_alone():
    arrival = np.array([0.0, 0.0, 0.0, 0.0, 0.0])
    nlimbs = np.array([1000, 1000, 50000, 1000, 1000])
    be, sch, done_at, sizes = _serve(arrival, nlimbs, max_batch=8, max_limbs=4000, depth=1)
    batches = [b for _, b, _ in be.launches]
    assert batches == [[0, 1], [2], [3, 4]]
    assert not np.isnan(done_at).any()


def test_admit_respects_every_budget():
    class Nop:
        pass
    sch = Scheduler(Nop(), {"limbs": ([10] * 100, 1000)}, max_batch=7)
    assert sch.admit(list(range(20))) == list(range(7))
    sch = Scheduler(Nop(), {"limbs": ([300] * 100, 1000)}, max_batch=50)
    assert sch.admit(list(range(20))) == [0, 1, 2]
    # two budgets: the first one to run out ends the batch
    sch = Scheduler(Nop(), {"hbm": ([100] * 100, 1000), "lds": ([0.3] * 100, 1.0)}, max_batch=50)
    assert sch.admit(list(range(20))) == [0, 1, 2]
    sch = Scheduler(Nop(), {"hbm": ([400] * 100, 1000), "lds": ([0.1] * 100, 1.0)}, max_batch=50)
    assert sch.admit(list(range(20))) == [0, 1]


def test_c5_workload_shapes():
    c = I.config_c5(1e4, count=300)
    assert c["n"].min() >= 1024 and c["n"].max() <= 8192
    for u, v, n, nv in zip(c["u"], c["v"], c["n"], c["nv"]):
        assert len(u) == n and len(v) == nv and (n + 7) // 8 <= nv <= n and u[-1] and v[-1]
    gaps = np.diff(np.concatenate([[0.0], c["arrival"]]))
    assert (gaps > 0).all() and abs(gaps.mean() * 1e4 - 1) < 0.2      # Poisson rate 1e4/s
    # operands do not depend on the rate; a subset regenerates the same requests
    d = I.config_c5(1e3, index=[5, 17])
    assert (d["u"][1] == c["u"][17]).all() and (d["v"][0] == c["v"][5]).all()
    assert abs(d["arrival"][1] * 1e3 / 18 - 1) < 1.0
