"""Serving loop: continuous batching of division requests on one GPU.

Requests (u, v) wait in host memory until they are admitted.  The loop
repeatedly
  * retires finished batches: each batch records an event after its results
    have reached host memory, and a request is complete when the host sees
    its batch's event (so latency includes the operand upload, the
    divisions and the result download);
  * admits the waiting requests in arrival order into the next batch under
    the budgets of one in-flight slot: device bytes (operands, results,
    descriptors and status of the batch, within the slot's share of the HBM
    that was free when serving started) and LDS residency (the batch's
    instances may fill the device's workgroup LDS at most `lds_waves` times
    over), and at most `max_batch` requests; a single request above a budget
    is admitted alone once it reaches the head of the queue, so nothing is
    dropped;
  * uploads the batch and launches it on the slot's own stream, keeping up to
    `depth` batches in flight, so the host prepares the next batch while the
    device works and batches overlap on the device.
Each request is computed by one workgroup from its own operands, so it gives
the same bits alone or in any batch.

Two device backends serve the same trace: RaggedBackend (one
mp_divrem_ragged per batch, all widths together) and PlainBackend (the
batch's requests grouped by dividend width class, zero-padded into one
uniform mp_divrem_batch launch per class: the plain one-precision-per-launch
path).  The scheduling logic (Scheduler) is independent of the device and is
tested on the host with a fake backend.
"""
import collections
import time

import numpy as np

CLASS_WIDTHS = (1024, 2048, 4096, 8192)


def width_class(n):
    """index of the dividend width class of n limbs"""
    return int(np.searchsorted(CLASS_WIDTHS, n))


class Scheduler:
    """Admission and batching over a backend with launch(slot, ids) -> handle
    and done(handle) -> bool.  costs: name -> (per-request cost array,
    per-batch budget)."""

    def __init__(self, backend, costs, max_batch=4096, depth=2):
        self.backend = backend
        self.costs = {k: (np.asarray(c, dtype=np.float64), float(b)) for k, (c, b) in costs.items()}
        self.max_batch = int(max_batch)
        self.depth = int(depth)

    def admit(self, queue):
        """Requests of the next batch: a prefix of the queue within every
        budget (the head request alone when it exceeds one)."""
        take = []
        used = {k: 0.0 for k in self.costs}
        for j in queue:
            if take and len(take) >= self.max_batch:
                break
            if take and any(used[k] + c[j] > b for k, (c, b) in self.costs.items()):
                break
            take.append(j)
            for k, (c, _) in self.costs.items():
                used[k] += c[j]
        return take

    def run(self, arrival, clock=time.perf_counter, idle=None):
        """Serve requests with the given arrival times (seconds from start).
        Returns (completion times, batch sizes, host seconds spent launching)."""
        arrival = np.asarray(arrival, dtype=np.float64)
        order = np.argsort(arrival, kind="stable")
        n = len(arrival)
        done_at = np.full(n, np.nan)
        queue = collections.deque()
        inflight = collections.deque()
        sizes = []
        launch_s = 0.0
        nxt, finished, slot = 0, 0, 0
        t0 = clock()
        while finished < n:
            now = clock() - t0
            while nxt < n and arrival[order[nxt]] <= now:
                queue.append(int(order[nxt]))
                nxt += 1
            while inflight and self.backend.done(inflight[0][0]):
                _, ids = inflight.popleft()
                done_at[ids] = clock() - t0
                finished += len(ids)
            if queue and len(inflight) < self.depth:
                take = self.admit(queue)
                for _ in take:
                    queue.popleft()
                ids = np.asarray(take, dtype=np.int64)
                tl = clock()
                inflight.append((self.backend.launch(slot, ids), ids))
                launch_s += clock() - tl
                slot = (slot + 1) % self.depth
                sizes.append(len(take))
            elif idle is not None:
                idle()
        return done_at, sizes, launch_s


class _Requests:
    """All requests' operands and results in pinned host memory, each at a
    4-limb-aligned offset (the place a request arrives into and its results
    return to)."""

    def __init__(self, us, vs):
        import torch
        self.n = len(us)
        self.nu = np.array([len(u) for u in us], dtype=np.int64)
        self.nv = np.array([len(v) for v in vs], dtype=np.int64)
        w = lambda x: (x + 3) & ~3
        self.uo = np.concatenate([[0], np.cumsum(w(self.nu))])
        self.vo = np.concatenate([[0], np.cumsum(w(self.nv))])
        pin = lambda n: torch.zeros(max(int(n), 4), dtype=torch.int32).pin_memory()
        self.u, self.v = pin(self.uo[-1]), pin(self.vo[-1])
        self.q, self.r = pin(self.uo[-1]), pin(self.vo[-1])         # q has nu limbs, r has nv
        self.status = torch.full((self.n,), -1, dtype=torch.int32).pin_memory()
        uh, vh = self.u.numpy().view(np.uint32), self.v.numpy().view(np.uint32)
        for j in range(self.n):
            uh[self.uo[j]:self.uo[j] + self.nu[j]] = us[j]
            vh[self.vo[j]:self.vo[j] + self.nv[j]] = vs[j]

    def contiguous(self, ids):
        return len(ids) > 0 and ids[-1] - ids[0] + 1 == len(ids) and bool((np.diff(ids) == 1).all())

    def results(self):
        """(q rows, r rows, status) of every request"""
        qh, rh = self.q.numpy().view(np.uint32), self.r.numpy().view(np.uint32)
        qs = [qh[self.uo[j]:self.uo[j] + self.nu[j]] for j in range(self.n)]
        rs = [rh[self.vo[j]:self.vo[j] + self.nv[j]] for j in range(self.n)]
        return qs, rs, self.status.numpy()


def device_budgets(req, depth, lds_waves=2.0, hbm_share=0.5):
    """Per-batch budgets from what the device has: device bytes (a share of the
    HBM free now, split over the in-flight slots) and LDS residency (each
    request costs its workgroup's LDS as a fraction of the whole device's LDS;
    a batch may fill it lds_waves times over)."""
    import torch
    from . import binding
    free, _ = torch.cuda.mem_get_info()
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    dev_lds = props.multi_processor_count * 160 * 1024
    cls_lds = {w: binding.lds_bytes(binding.MP_OP_DIVREM, w, w) for w in CLASS_WIDTHS}
    lds = np.array([cls_lds[CLASS_WIDTHS[width_class(n)]] / dev_lds for n in req.nu])
    nbytes = 4 * (2 * req.nu + 2 * req.nv) + 48 + 4 + 16 + 64 * 4
    return {"hbm": (nbytes, free * hbm_share / depth), "lds": (lds, lds_waves)}


_slot_streams = {}


def slot_stream(device, path, slot):
    """The stream of in-flight slot `slot` of a serving path on `device`,
    shared by every backend of that path in the process: mp_divrem_ragged makes its fork streams once per
    caller stream, on first use, so reusing the slot streams keeps that set-up
    out of the serving loop of every run after the first."""
    import torch
    key = (str(device), path, int(slot))
    if key not in _slot_streams:
        _slot_streams[key] = torch.cuda.Stream(device=device)
    return _slot_streams[key]


class RaggedBackend:
    """Each batch is one mp_divrem_ragged call on the slot's own stream:
    operands up from pinned host memory, results back to it."""

    def __init__(self, req, depth, slot_bytes, max_batch, device="cuda"):
        import torch
        from . import binding, ragged
        self.torch, self.binding, self.req = torch, binding, req
        # descriptors of every request with its offsets relative to its own batch start filled at launch
        self.desc = np.zeros(req.n, dtype=ragged.DESC_DTYPE)
        self.desc["nu"], self.desc["nv"], self.desc["nq"] = req.nu, req.nv, req.nu
        cap_u = int(min(slot_bytes // 4, req.uo[-1])) + 4
        cap_v = int(min(slot_bytes // 4, req.vo[-1])) + 4
        nb = int(binding.lib().mp_ragged_workspace_bytes(max_batch))
        self.slots = []
        for i in range(depth):
            self.slots.append({
                "stream": slot_stream(device, "ragged", i),
                "u": torch.empty(cap_u, dtype=torch.int32, device=device),
                "v": torch.empty(cap_v, dtype=torch.int32, device=device),
                "q": torch.empty(cap_u, dtype=torch.int32, device=device),
                "r": torch.empty(cap_v, dtype=torch.int32, device=device),
                "st": torch.empty(max_batch, dtype=torch.int32, device=device),
                "desc_h": torch.empty(max_batch * 48, dtype=torch.uint8).pin_memory(),
                "desc_d": torch.empty(max_batch * 48, dtype=torch.uint8, device=device),
                "ws": torch.empty((nb + 3) // 4, dtype=torch.int32, device=device),
            })

    def launch(self, slot, ids):
        torch, req, s = self.torch, self.req, self.slots[slot]
        assert req.contiguous(ids), "batches are contiguous runs of requests in arrival order"
        j0, j1 = int(ids[0]), int(ids[-1]) + 1
        c = j1 - j0
        u0, u1, v0, v1 = req.uo[j0], req.uo[j1], req.vo[j0], req.vo[j1]
        if u1 - u0 > s["u"].numel() or v1 - v0 > s["v"].numel() or c > s["st"].numel():
            raise ValueError("batch exceeds the slot's device pools")
        d = self.desc[j0:j1].copy()
        d["u_off"], d["q_off"] = req.uo[j0:j1] - u0, req.uo[j0:j1] - u0
        d["v_off"], d["r_off"] = req.vo[j0:j1] - v0, req.vo[j0:j1] - v0
        s["desc_h"][:c * 48].numpy()[:] = d.view(np.uint8)
        st = s["stream"]
        with torch.cuda.stream(st):
            s["u"][:u1 - u0].copy_(req.u[u0:u1], non_blocking=True)
            s["v"][:v1 - v0].copy_(req.v[v0:v1], non_blocking=True)
            s["desc_d"][:c * 48].copy_(s["desc_h"][:c * 48], non_blocking=True)
            rc = self.binding.lib().mp_divrem_ragged(
                s["u"].data_ptr(), u1 - u0, s["v"].data_ptr(), v1 - v0, s["desc_d"].data_ptr(),
                s["q"].data_ptr(), u1 - u0, s["r"].data_ptr(), v1 - v0, s["st"].data_ptr(), c,
                s["ws"].data_ptr(), self.binding._stream(st))
            if rc != 0:
                raise self.binding.MPError("mp_divrem_ragged: %s" % self.binding.lib().mp_status_str(rc).decode())
            req.q[u0:u1].copy_(s["q"][:u1 - u0], non_blocking=True)
            req.r[v0:v1].copy_(s["r"][:v1 - v0], non_blocking=True)
            req.status[j0:j1].copy_(s["st"][:c], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(st)
        return ev

    def done(self, ev):
        return ev.query()


class PlainBackend:
    """Each batch as the plain path runs it: the requests grouped by dividend
    width class and zero-padded into one uniform mp_divrem_batch launch per
    class (dividend width = the class width, divisor width = the widest
    divisor of the group), on the slot's stream, operands up from and results
    back to pinned host memory."""

    def __init__(self, req, depth, slot_bytes, max_batch, device="cuda"):
        import torch
        from . import binding
        self.torch, self.binding, self.req = torch, binding, req
        self.cls = np.array([width_class(n) for n in req.nu])
        cap = int(min(slot_bytes // 4, 2 * CLASS_WIDTHS[-1] * max_batch)) + 8
        self.slots = []
        for i in range(depth):
            self.slots.append({
                "stream": slot_stream(device, "plain", i),
                "in_h": torch.empty(cap, dtype=torch.int32).pin_memory(),
                "out_h": torch.empty(cap, dtype=torch.int32).pin_memory(),
                "in_d": torch.empty(cap, dtype=torch.int32, device=device),
                "out_d": torch.empty(cap, dtype=torch.int32, device=device),
                "st": torch.empty(max_batch, dtype=torch.int32, device=device),
            })
        self.pending = {}

    def _pack(self, ids, W, nvm, buf):
        """u rows (W limbs) then v rows (nvm limbs) of the requests, zero-padded"""
        req = self.req
        n = len(ids)
        a = buf[:n * (W + nvm)].numpy().view(np.uint32)
        a[:] = 0
        uh, vh = req.u.numpy().view(np.uint32), req.v.numpy().view(np.uint32)
        U = a[:n * W].reshape(n, W)
        V = a[n * W:].reshape(n, nvm)
        for i, j in enumerate(ids):
            U[i, :req.nu[j]] = uh[req.uo[j]:req.uo[j] + req.nu[j]]
            V[i, :req.nv[j]] = vh[req.vo[j]:req.vo[j] + req.nv[j]]
        return n * (W + nvm)

    def launch(self, slot, ids):
        torch, s, req = self.torch, self.slots[slot], self.req
        st = s["stream"]
        ids = np.asarray(ids)
        groups = []
        off_in, off_out, off_st = 0, 0, 0
        for c in range(len(CLASS_WIDTHS)):
            g = ids[self.cls[ids] == c]
            if len(g) == 0:
                continue
            W, nvm = CLASS_WIDTHS[c], int(req.nv[g].max())
            nin = self._pack(g, W, nvm, s["in_h"][off_in:])
            groups.append((g, W, nvm, off_in, off_out, off_st))
            off_in += nin
            off_out += len(g) * (W + nvm)
            off_st += len(g)
        if off_in > s["in_h"].numel() or off_st > s["st"].numel():
            raise ValueError("batch exceeds the slot's pools")
        with torch.cuda.stream(st):
            s["in_d"][:off_in].copy_(s["in_h"][:off_in], non_blocking=True)
            for g, W, nvm, oi, oo, os_ in groups:
                n = len(g)
                u = s["in_d"][oi:oi + n * W].view(n, W)
                v = s["in_d"][oi + n * W:oi + n * (W + nvm)].view(n, nvm)
                q = s["out_d"][oo:oo + n * W].view(n, W)
                r = s["out_d"][oo + n * W:oo + n * (W + nvm)].view(n, nvm)
                self.binding.divrem(u, v, out=(q, r, s["st"][os_:os_ + n]), stream=st)
            s["out_h"][:off_out].copy_(s["out_d"][:off_out], non_blocking=True)
            stat = torch.empty(off_st, dtype=torch.int32).pin_memory()
            stat.copy_(s["st"][:off_st], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(st)
        self.pending[id(ev)] = (groups, stat, slot)
        return ev

    def done(self, ev):
        if not ev.query():
            return False
        groups, stat, slot = self.pending.pop(id(ev))
        # results back into the requests' places (host side of the plain path)
        req, out = self.req, self.slots[slot]["out_h"].numpy().view(np.uint32)
        qh, rh = req.q.numpy().view(np.uint32), req.r.numpy().view(np.uint32)
        sts = stat.numpy()
        for g, W, nvm, oi, oo, os_ in groups:
            n = len(g)
            Q = out[oo:oo + n * W].reshape(n, W)
            R = out[oo + n * W:oo + n * (W + nvm)].reshape(n, nvm)
            for i, j in enumerate(g):
                qh[req.uo[j]:req.uo[j] + req.nu[j]] = Q[i, :req.nu[j]]
                rh[req.vo[j]:req.vo[j] + req.nv[j]] = R[i, :req.nv[j]]
            req.status.numpy()[g] = sts[os_:os_ + n]
        return True


def serve(us, vs, arrival, path="ragged", depth=3, max_batch=4096, lds_waves=2.0, hbm_share=0.5):
    """Serve the requests with the given arrival times (s); path 'ragged' or
    'plain'.  Returns latencies (s), batch sizes, throughput, the host time
    spent preparing and launching batches, and the requests (for results)."""
    import torch
    req = _Requests(us, vs)
    budgets = device_budgets(req, depth, lds_waves, hbm_share)
    slot_bytes = budgets["hbm"][1]
    Backend = RaggedBackend if path == "ragged" else PlainBackend
    be = Backend(req, depth, slot_bytes, max_batch)
    sch = Scheduler(be, budgets, max_batch=max_batch, depth=depth)
    torch.cuda.synchronize()
    done_at, sizes, launch_s = sch.run(arrival)
    lat = done_at - np.asarray(arrival)
    span = float(np.nanmax(done_at)) if len(done_at) else 0.0
    return {"latency": lat, "batches": sizes, "div_per_s": len(us) / span if span > 0 else 0.0,
            "span_s": span, "host_launch_s": launch_s, "requests": req, "path": path}


def all_at_once(us, vs, path="ragged", reps=5):
    """Throughput of the requests as one device-resident batch: one
    mp_divrem_ragged call, or four uniform mp_divrem_batch launches (one per
    width class, zero-padded); mean ms of a run and divisions per second."""
    import torch
    from . import binding, ragged
    stream = torch.cuda.current_stream()
    if path == "ragged":
        rb = binding.Ragged(ragged.pack(us, vs))
        run = lambda: rb.run(stream)
    else:
        groups = []
        cls = np.array([width_class(len(u)) for u in us])
        for c, W in enumerate(CLASS_WIDTHS):
            js = np.nonzero(cls == c)[0]
            if len(js) == 0:
                continue
            nvm = max(len(vs[j]) for j in js)
            U = np.zeros((len(js), W), dtype=np.uint32)
            V = np.zeros((len(js), nvm), dtype=np.uint32)
            for i, j in enumerate(js):
                U[i, :len(us[j])] = us[j]
                V[i, :len(vs[j])] = vs[j]
            t = lambda a: torch.from_numpy(a.view(np.int32)).cuda()
            groups.append((t(U), t(V), (torch.empty((len(js), W), dtype=torch.int32, device="cuda"),
                                        torch.empty((len(js), nvm), dtype=torch.int32, device="cuda"),
                                        torch.empty(len(js), dtype=torch.int32, device="cuda"))))

        def run():
            for U, V, out in groups:
                binding.divrem(U, V, out=out, stream=stream)
    run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        run()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return {"ms": ms, "div_per_s": len(us) / (ms * 1e-3)}
