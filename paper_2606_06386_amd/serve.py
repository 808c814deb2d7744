"""Serving loop: continuous batching of division requests on one GPU.

Requests (u, v) are resident in device memory (packed pools, as after their
upload); each becomes visible to the scheduler at its arrival time.  The loop
repeatedly
  * retires finished batches (an event per batch; the completion time of
    every request in it is the moment the host sees the event complete),
  * forms the next batch from the waiting requests in arrival order under an
    admission budget (at most `max_batch` requests and `max_limbs` dividend
    limbs per batch; a single request above the limb budget is admitted on
    its own once it reaches the head of the queue, so nothing is dropped),
  * launches it with mp_divrem_ragged (descriptors and request ids go up
    through pinned host buffers on the same stream), keeping up to `depth`
    batches in flight so that the host prepares the next while the device
    runs the current one.
Every request's result is written to its own place in the output pools, so
a request gives the same bits alone or in any batch: each division is
computed by one workgroup from its own operands only.

The scheduling logic is independent of the device (``Scheduler`` with a
backend object); ``GpuBackend`` is the one that launches the kernels.
"""
import collections
import time

import numpy as np


class Scheduler:
    """Admission and batching over a backend with launch(slot, ids) -> handle
    and done(handle) -> bool."""

    def __init__(self, backend, nlimbs, max_batch=2048, max_limbs=1 << 22, depth=2):
        self.backend = backend
        self.nlimbs = np.asarray(nlimbs, dtype=np.int64)
        self.max_batch = int(max_batch)
        self.max_limbs = int(max_limbs)
        self.depth = int(depth)

    def admit(self, queue):
        """Requests of the next batch: a prefix of the queue within the budget
        (the head request alone when it exceeds the limb budget)."""
        take, limbs = [], 0
        for j in queue:
            n = int(self.nlimbs[j])
            if take and (len(take) >= self.max_batch or limbs + n > self.max_limbs):
                break
            take.append(j)
            limbs += n
            if len(take) >= self.max_batch:
                break
        return take

    def run(self, arrival, clock=time.perf_counter, idle=None):
        """Serve requests with the given arrival times (seconds from start).
        Returns (completion times, batch sizes) in seconds from start."""
        arrival = np.asarray(arrival, dtype=np.float64)
        order = np.argsort(arrival, kind="stable")
        n = len(arrival)
        done_at = np.full(n, np.nan)
        queue = collections.deque()
        inflight = collections.deque()
        sizes = []
        nxt, finished, slot = 0, 0, 0
        t0 = clock()
        while finished < n:
            now = clock() - t0
            while nxt < n and arrival[order[nxt]] <= now:
                queue.append(int(order[nxt]))
                nxt += 1
            while inflight and self.backend.done(inflight[0][0]):
                h, ids = inflight.popleft()
                t = clock() - t0
                done_at[ids] = t
                finished += len(ids)
            if queue and len(inflight) < self.depth:
                take = self.admit(queue)
                for _ in take:
                    queue.popleft()
                ids = np.asarray(take, dtype=np.int64)
                inflight.append((self.backend.launch(slot, ids), ids))
                slot = (slot + 1) % self.depth
                sizes.append(len(take))
            elif idle is not None:
                idle()
        return done_at, sizes


class GpuBackend:
    """Device side of the serving loop: request pools, per-slot pinned
    descriptor buffers, workspaces and status buffers."""

    def __init__(self, us, vs, max_batch, depth=2, device="cuda"):
        import torch
        from . import binding, ragged
        self.torch, self.binding = torch, binding
        packed = ragged.pack(us, vs)
        self.desc = packed["desc"]
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).to(device)
        self.u, self.v = t(packed["u_pool"]), t(packed["v_pool"])
        self.q = torch.zeros(packed["q_limbs"], dtype=torch.int32, device=device)
        self.r = torch.zeros(packed["r_limbs"], dtype=torch.int32, device=device)
        self.status = torch.full((len(us),), -1, dtype=torch.int32, device=device)
        self.max_batch = max_batch
        nb = int(binding.lib().mp_ragged_workspace_bytes(max_batch))
        self.slots = []
        for _ in range(depth):
            self.slots.append({
                "desc_h": torch.empty(max_batch * 48, dtype=torch.uint8, pin_memory=True),
                "ids_h": torch.empty(max_batch, dtype=torch.int64, pin_memory=True),
                "desc_d": torch.empty(max_batch * 48, dtype=torch.uint8, device=device),
                "ids_d": torch.empty(max_batch, dtype=torch.int64, device=device),
                "st_d": torch.empty(max_batch, dtype=torch.int32, device=device),
                "ws": torch.empty((nb + 3) // 4, dtype=torch.int32, device=device),
            })
        self.stream = torch.cuda.current_stream()

    def launch(self, slot, ids):
        torch, s = self.torch, self.slots[slot]
        c = len(ids)
        assert 0 < c <= self.max_batch
        s["desc_h"][:c * 48].numpy()[:] = self.desc[ids].view(np.uint8)
        s["ids_h"][:c].numpy()[:] = ids
        s["desc_d"][:c * 48].copy_(s["desc_h"][:c * 48], non_blocking=True)
        s["ids_d"][:c].copy_(s["ids_h"][:c], non_blocking=True)
        rc = self.binding.lib().mp_divrem_ragged(
            self.u.data_ptr(), self.u.numel(), self.v.data_ptr(), self.v.numel(), s["desc_d"].data_ptr(),
            self.q.data_ptr(), self.q.numel(), self.r.data_ptr(), self.r.numel(), s["st_d"].data_ptr(), c,
            s["ws"].data_ptr(), self.binding._stream(self.stream))
        if rc != 0:
            raise self.binding.MPError("mp_divrem_ragged: %s" % self.binding.lib().mp_status_str(rc).decode())
        self.status.index_copy_(0, s["ids_d"][:c], s["st_d"][:c])
        ev = torch.cuda.Event()
        ev.record(self.stream)
        return ev

    def done(self, ev):
        return ev.query()

    def results(self):
        """(q rows, r rows, status) of every request, on the host."""
        from . import ragged
        self.torch.cuda.synchronize()
        q = self.q.cpu().numpy().view(np.uint32)
        r = self.r.cpu().numpy().view(np.uint32)
        return ragged.unpack(q, self.desc, "q"), ragged.unpack(r, self.desc, "r"), self.status.cpu().numpy()


def serve(us, vs, arrival, max_batch=2048, max_limbs=1 << 22, depth=2):
    """Run the serving loop on the GPU; returns dict with latencies (s), batch
    sizes, throughput and the backend (for the results)."""
    be = GpuBackend(us, vs, max_batch, depth)
    sch = Scheduler(be, [len(u) for u in us], max_batch, max_limbs, depth)
    done_at, sizes = sch.run(arrival)
    lat = done_at - np.asarray(arrival)
    span = float(np.nanmax(done_at)) if len(done_at) else 0.0
    return {"latency": lat, "batches": sizes, "div_per_s": len(us) / span if span > 0 else 0.0,
            "backend": be}
