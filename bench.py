"""Benchmark: batched exact division at 2^16 bits on one MI355X.

One step = one mp_divrem_batch launch over the whole workload (every
instance goes through shifted inverse, quotient product, remainder product
and corrections).  Inputs are device-resident before the timed region.
Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--config c2|c1|c3|c4] [--no-cpu-baseline]

--config c5 runs the serving loop instead: 10^4 requests of 2^15..2^18 bits
with Poisson arrivals at 10^3 .. 10^6 per second, continuous batching over
mp_divrem_ragged; it reports throughput and p50/p99 latency per rate.

--config c4 times the mixed-precision batch instead: 8192 divisions with
dividends of 2^15..2^18 bits in one mp_divrem_ragged call (launch
configuration from the autotuner), beside the same divisions as four
uniform-width mp_divrem_batch launches.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "divisions/sec at 2^16-bit u (bit-exact) + % int-mul roofline; serving p99 latency"

# The products run on the int8 matrix cores: one 32x32-bit limb product is 16
# digit products (4 x 4 bytes), i.e. 32 int8 operations.  MI355X's published
# dense int8 matrix peak is 5.0e15 operations/s.
OPS_PER_LIMB_PRODUCT = 32
PEAK_INT8_OPS = 5.0e15
# For comparison, the vector-ALU multiply rate: 256 CUs x 4 SIMDs at 2.4 GHz,
# each SIMD issuing one wave64 v_mad_u64_u32 (64 limb products) every 4 cycles.
PEAK_LIMB_PRODUCTS = 256 * 4 * 16 * 2.4e9


def threads_for(width):
    """Workgroup size the library launches for dividends of `width` limbs."""
    return 256 if width <= 2048 else 512 if width <= 4096 else 1024


def prec_rows(x):
    """number of significant limbs of each row"""
    nz = x != 0
    return np.where(nz.any(axis=1), x.shape[1] - np.argmax(nz[:, ::-1], axis=1), 0)


def workload(name):
    from paper_2606_06386_amd import inputs as I
    return {"c1": I.config_c1, "c2": I.config_c2, "c3": I.config_c3}[name]()


def limb_products(u, v, clipped=True):
    """Algorithmic limb products of one launch over the batch: the cost model's
    W_clipped (what the kernels compute), or the method's W with full
    quotient and remainder products (clipped=False)."""
    from paper_2606_06386_amd import costmodel as cm
    cost = cm.division_cost_clipped if clipped else cm.division_cost
    hs, nvs = prec_rows(u), prec_rows(v)
    total = 0
    cache = {}
    for h, nvv in zip(hs.tolist(), nvs.tolist()):
        key = (h, nvv - 1)
        if key not in cache:
            cache[key] = cost(h, nvv - 1) if nvv >= 2 and h >= nvv else 0
        total += cache[key]
    return total


def ragged_limb_products(us, vs, clipped=True):
    from paper_2606_06386_amd import costmodel as cm
    cost = cm.division_cost_clipped if clipped else cm.division_cost
    cache, total = {}, 0
    for u, v in zip(us, vs):
        key = (len(u), len(v) - 1)          # top limbs are nonzero in the mixed workload
        if key not in cache:
            cache[key] = cost(*key) if key[1] >= 1 and key[0] > key[1] else 0
        total += cache[key]
    return total


def measured_traffic(workload_name):
    """HBM bytes per launch of k_divrem from committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE counts (each scaled by what the counter reads for a 256 MiB
    device copy), or None when those counts were taken on other kernel sources
    or another workload."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"k_divrem_{workload_name.split('_', 1)[1]}_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256(b"".join(open(os.path.join(ROOT, s_), "rb").read() for s_ in rec["sources"])).hexdigest()
    return rec["traffic_bytes_per_dispatch"] if h == rec["source_sha256"] else None


TRAFFIC_SOURCES = ["paper_2606_06386_amd/csrc/mp_prims_hip.hpp", "paper_2606_06386_amd/csrc/mp_core.hpp",
                   "paper_2606_06386_amd/csrc/mp_div.hpp", "paper_2606_06386_amd/csrc/launch.hpp",
                   "paper_2606_06386_amd/csrc/kernels.hip", "paper_2606_06386_amd/csrc/mpdiv.hip"]


def write_traffic(fetch_csv, write_csv, workload_name, kernels=("k_head_divrem", "k_divrem<")):
    """profiles/k_divrem_<workload>_traffic.json from two rocprofv3 --pmc
    counter files (FETCH_SIZE, WRITE_SIZE) of `bench.py --copy-calibration`:
    the mean KiB per dispatch of each kernel of one launch (the head and the
    per-instance kernel of mp_divrem_batch), summed, each counter scaled by
    what it reads for the 256 MiB device copy."""
    import csv
    import hashlib

    def read(path, counter):
        kern, copy = {k: [] for k in kernels}, []
        with open(path) as fh:
            for row in csv.DictReader(fh):
                if row["Counter_Name"] != counter:
                    continue
                v = float(row["Counter_Value"])
                hit = [k for k in kernels if k in row["Kernel_Name"]]
                if hit:
                    kern[hit[0]].append(v)
                elif "copyBuffer" in row["Kernel_Name"]:
                    copy.append(v)
        assert all(kern.values()) and copy, (path, counter, {k: len(x) for k, x in kern.items()}, len(copy))
        return sum(sum(x) / len(x) for x in kern.values()), max(copy)   # the 256 MiB copy is the largest

    f_k, f_c = read(fetch_csv, "FETCH_SIZE")
    w_k, w_c = read(write_csv, "WRITE_SIZE")
    nbytes = 256 << 20
    ff, wf = nbytes / 1024 / f_c, nbytes / 1024 / w_c
    h = hashlib.sha256(b"".join(open(os.path.join(ROOT, s_), "rb").read() for s_ in TRAFFIC_SOURCES)).hexdigest()
    rec = {"kernels": list(kernels), "workload": workload_name, "fetch_size_kib_per_dispatch": f_k,
           "write_size_kib_per_dispatch": w_k,
           "copy_calibration": {"bytes": nbytes, "fetch_size_kib": f_c, "write_size_kib": w_c},
           "fetch_factor": ff, "write_factor": wf, "traffic_bytes_per_dispatch": 1024 * (f_k * ff + w_k * wf),
           "source_sha256": h, "sources": TRAFFIC_SOURCES}
    path = os.path.join(ROOT, "profiles", f"k_divrem_{workload_name.split('_', 1)[1]}_traffic.json")
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec))


def cpu_baseline(c, q_gpu, r_gpu, budget_s=10.0):
    """The oracle (plain C, OpenMP over instances) on a bounded sample of the
    same workload, on all host cores and on one; also checks the GPU results of
    the sample bit-exactly."""
    import oracle
    u, v, nq = c["u"], c["v"], c["nq"]
    n = 32
    t0 = time.perf_counter()
    oracle.divrem_threads(u[:n], v[:n], nq, v.shape[1])
    t = time.perf_counter() - t0
    n = int(min(len(u), max(n, n * budget_s / max(t, 1e-3))))
    t0 = time.perf_counter()
    qo, ro, so, used = oracle.divrem_threads(u[:n], v[:n], nq, v.shape[1])
    t = time.perf_counter() - t0
    exact = int(((qo == q_gpu[:n]).all(axis=1) & (ro == r_gpu[:n]).all(axis=1)).sum())
    n1 = max(8, min(n, int(n / max(used, 1))))       # about the same CPU time on one core
    t0 = time.perf_counter()
    oracle.divrem_threads(u[:n1], v[:n1], nq, v.shape[1], nthreads=1)
    t1 = time.perf_counter() - t0
    info = host_info()
    return {"value": n / t, "unit": "div/s", "cores": int(used), "kind": "oracle",
            "sample": f"first {n} of {len(u)} instances of {c['name']} (Knuth D, gcc -O2, OpenMP)",
            "one_core": {"value": n1 / t1, "unit": "div/s", "sample": f"first {n1} instances"},
            **info}, exact, n


PROBES = ["v_mad_u64_u32", "v_mad_u64_u32+v_addc_co_u32", "v_mul_lo_u32+v_mul_hi_u32", "v_add_u32",
          "v_mul_u32_u24", "v_addc_co_u32_e64", "v_addc_co_u32_e32", "v_add3_u32", "v_lshl_add_u64",
          "v_cndmask_b32_e64", "v_mad_u64_u32+v_add_u32", "v_dot4_u32_u8", "v_mfma_i32_32x32x32_i8"]


def probe_rates():
    """Measured issue rates of the candidate limb-product instructions (one
    JSON line): lane-operations/s over all CUs and the implied cycles per wave64
    instruction sequence per SIMD at the 2.4 GHz peak clock."""
    import ctypes
    import torch
    from paper_2606_06386_amd import build as hb
    L = ctypes.CDLL(hb.PROBE_LIB)
    L.mp_probe_rate.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_double)]
    blocks, iters = 8192, 4000
    scratch = torch.empty(blocks * 256, dtype=torch.int32, device="cuda:0")
    out = {"probe": "integer issue rates", "blocks": blocks, "threads": 256, "iters": iters, "rates": {}}
    for v, name in enumerate(PROBES):
        ms, ops = ctypes.c_float(), ctypes.c_double()
        for _ in range(3):
            rc = L.mp_probe_rate(v, iters, blocks, ctypes.c_void_p(scratch.data_ptr()), ctypes.byref(ms),
                                 ctypes.byref(ops))
            assert rc == 0, rc
        rate = ops.value / (ms.value * 1e-3)
        cyc = 256 * 4 * 2.4e9 / (rate / 64)
        rec = {"lane_ops_per_s": rate, "ms": ms.value, "cycles_per_wave_op_at_2p4GHz": cyc}
        if name.startswith("v_mfma"):   # 8 wave-level MFMAs per iteration, 32*32*32 int8 MACs each
            rec = {"macs_per_s": rate / 64 * 32768, "ms": ms.value, "cycles_per_mfma_per_simd_at_2p4GHz": cyc}
        out["rates"][name] = rec
    print(json.dumps(out), flush=True)


def _timed(fn, steps, stream):
    """Runs fn `steps` times back to back on `stream`; returns the wall time
    of the whole run (synchronised on both sides) and the sorted durations of
    the steps from HIP events.  One event marks each boundary between steps
    (the end of one is the start of the next), so the instrumentation adds one
    event record per step to the timed region, not two."""
    import torch
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    marks[0].record(stream)
    for i in range(steps):
        fn()
        marks[i + 1].record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms = sorted(a.elapsed_time(b) for a, b in zip(marks[:-1], marks[1:]))
    return elapsed, ms


SETTLE_MS = 60.0   # untimed load before the warm-up steps (the shader clock's ramp lasts ~20-30 ms)


def settle(fn, stream, min_ms=SETTLE_MS):
    """Runs fn untimed until at least min_ms of wall time has passed, so that
    the timed steps see the clock the chip holds under this load rather than
    its ramp up from idle (step times fall by half over the first ~25 ms of
    load).  Returns the number of steps run."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n = 0
    while (time.perf_counter() - t0) * 1e3 < min_ms:
        for _ in range(4):
            fn()
        n += 4
        stream.synchronize()
    return n


def roofline(W, W_clipped, ms, kernel, traffic, algo_bytes):
    """Roofline object of a launch of ms milliseconds.  W is the method's
    algorithmic work (limb products of Alg. 1-3 at exact operand sizes, full
    quotient and remainder products); W_clipped is what the kernels form.
    The products run on the int8 matrix cores (32 int8 operations per limb
    product), so achieved and peak are int8 operations per second; the
    fraction of the vector-ALU multiply peak is given beside them."""
    rate = W / (ms * 1e-3)
    ops = OPS_PER_LIMB_PRODUCT * rate
    return {"bound": "mfma", "achieved": ops / 1e12, "peak": PEAK_INT8_OPS / 1e12, "unit": "int8 TOP/s",
            "frac": ops / PEAK_INT8_OPS, "traffic": traffic, "traffic_unit": "bytes/launch",
            "algorithmic_bytes": algo_bytes, "kernel": kernel,
            "work": "limb products of Alg. 1-3 at exact sizes (full u*shinv, v*q), 32 int8 ops each",
            "limb_products_per_launch": W, "limb_products_per_s": rate,
            "frac_clipped": OPS_PER_LIMB_PRODUCT * W_clipped / (ms * 1e-3) / PEAK_INT8_OPS,
            "limb_products_per_launch_clipped": W_clipped,
            "frac_valu_peak": rate / PEAK_LIMB_PRODUCTS, "valu_mad_peak_limb_products_per_s": PEAK_LIMB_PRODUCTS}


def host_info():
    """CPU model and core counts of this host."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": usable, "cpu_count": os.cpu_count()}


def time_divrem(binding, c, steps, warmup, stream):
    """Device-resident batch of c, timed per launch with HIP events on the
    launch stream; returns (elapsed s, sorted launch ms, q, r, status)."""
    import torch
    dev = torch.device("cuda:0")
    u_h, v_h, nq = c["u"], c["v"], c["nq"]
    batch = len(u_h)
    u = torch.from_numpy(u_h.view(np.int32)).to(dev)
    v = torch.from_numpy(v_h.view(np.int32)).to(dev)
    q = torch.empty((batch, nq), dtype=torch.int32, device=dev)
    r = torch.empty((batch, v_h.shape[1]), dtype=torch.int32, device=dev)
    st = torch.empty(batch, dtype=torch.int32, device=dev)
    step = lambda: binding.divrem(u, v, out=(q, r, st), stream=stream)
    nset = settle(step, stream)
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    elapsed, ms = _timed(step, steps, stream)
    return (elapsed, ms, q.cpu().numpy().view(np.uint32), r.cpu().numpy().view(np.uint32), st.cpu().numpy(),
            (u, v, q, r, st), nset)


def time_end_to_end(binding, c, steps, stream):
    """The same launches with the operands uploaded from pinned host memory
    before and the results downloaded after each one (PCIe included)."""
    import torch
    u_h, v_h, nq = c["u"], c["v"], c["nq"]
    batch = len(u_h)
    pin = lambda a: torch.from_numpy(a.view(np.int32)).pin_memory()
    uh, vh = pin(u_h), pin(v_h)
    qh = torch.empty((batch, nq), dtype=torch.int32).pin_memory()
    rh = torch.empty((batch, v_h.shape[1]), dtype=torch.int32).pin_memory()
    sh = torch.empty(batch, dtype=torch.int32).pin_memory()
    dev = torch.device("cuda:0")
    u, v = torch.empty_like(uh, device=dev), torch.empty_like(vh, device=dev)
    q, r, st = torch.empty_like(qh, device=dev), torch.empty_like(rh, device=dev), torch.empty_like(sh, device=dev)

    def step():
        u.copy_(uh, non_blocking=True)
        v.copy_(vh, non_blocking=True)
        binding.divrem(u, v, out=(q, r, st), stream=stream)
        qh.copy_(q, non_blocking=True)
        rh.copy_(r, non_blocking=True)
        sh.copy_(st, non_blocking=True)
    step()
    torch.cuda.synchronize()
    _, ms = _timed(step, steps, stream)
    mean = sum(ms) / len(ms)
    return {"ms": mean, "div_per_s": batch / (mean * 1e-3),
            "bytes_per_launch": 4 * (u_h.size + v_h.size + qh.numel() + rh.numel() + batch),
            "what": "H2D of u, v from pinned host memory + mp_divrem_batch + D2H of q, r, status per launch"}


def time_mul(binding, na, nb, batch, steps, warmup, stream):
    """mp_mul_batch of batch random na x nb-limb products: mean launch ms."""
    import torch
    g = torch.Generator(device="cuda:0").manual_seed(na * 131 + nb)
    a = torch.randint(-2 ** 31, 2 ** 31, (batch, na), dtype=torch.int32, device="cuda:0", generator=g)
    b = torch.randint(-2 ** 31, 2 ** 31, (batch, nb), dtype=torch.int32, device="cuda:0", generator=g)
    step = lambda: binding.mul(a, b, stream=stream)
    settle(step, stream)
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    _, ms = _timed(step, steps, stream)
    mean = sum(ms) / len(ms)
    ops = OPS_PER_LIMB_PRODUCT * na * nb * batch / (mean * 1e-3)
    return {"ms": mean, "batch": batch, "limb_products_per_s": na * nb * batch / (mean * 1e-3),
            "achieved": ops / 1e12, "unit": "int8 TOP/s", "frac": ops / PEAK_INT8_OPS}


def plain_result(c, elapsed, ms, q_h, r_h, status, steps):
    """Per-configuration figures of a timed plain batch."""
    u_h, v_h = c["u"], c["v"]
    batch = len(u_h)
    kmean = sum(ms) / len(ms)
    W = limb_products(u_h, v_h, clipped=False)
    Wc = limb_products(u_h, v_h)
    algo_bytes = 4 * (u_h.size + v_h.size + q_h.size + r_h.size) + 4 * batch   # u, v in; q, r, status out
    n = int(u_h.shape[1])
    return {"workload": c["name"], "batch": batch, "kernel_ms": {"mean": kmean, "median": ms[len(ms) // 2],
                                                                 "min": ms[0]},
            "div_per_s": batch * steps / elapsed, "div_per_s_kernel": batch / (kmean * 1e-3),
            "roofline": roofline(W, Wc, kmean, "k_head_divrem + k_divrem<%d>" % threads_for(n),
                                 measured_traffic(c["name"]), algo_bytes),
            "full_mult_equivalents_per_s": batch / (kmean * 1e-3) * (W / batch) / (n * n / 2),
            "status_ok": int((status == 0).sum())}


PHASES = [("load_prec", 0, 1), ("setup", 1, 2), ("initial_approx", 2, 3), ("one_wave_iters", 3, 4)]


RT_HZ = 100e6   # rate of the real-time counter (s_memrealtime)
kHEAD_WAVES = 4  # head instances (waves) per workgroup


def clock_stats(c0, c1, r0, r1, event_ms=None):
    """Shader clock and residency of a traced launch from per-workgroup cycle
    stamps (c0, c1) and real-time stamps (r0, r1) at its start and end: the
    mean shader clock (cycles over real time), the mean workgroup lifetime,
    the span from the first start to the last end, and the mean number of
    workgroups resident over that span.  With the launch's event time, the
    real-time counter's rate is checked against the span."""
    ok = (r1 > r0) & (c1 > c0)
    c0, c1, r0, r1 = c0[ok], c1[ok], r0[ok], r1[ok]
    span = float(r1.max() - r0.min())
    out = {"workgroups": int(ok.sum()),
           "shader_clock_ghz": float(np.mean((c1 - c0) / (r1 - r0))) * RT_HZ / 1e9,
           "workgroup_lifetime_us": float(np.mean(r1 - r0)) / RT_HZ * 1e6,
           "launch_span_us": span / RT_HZ * 1e6,
           "resident_workgroups": float(np.sum(r1 - r0)) / span if span > 0 else 0.0}
    if event_ms:
        out["event_ms"] = event_ms
    return out


def phase_trace(args):
    """Per-phase cycle breakdown of one k_divrem launch over the workload,
    from the phase stamps of libmpdiv_trace.so (build.py --trace): shader
    clock of workgroup thread 0 at each phase boundary, averaged over the
    instances that pass every phase.  Prints one JSON line."""
    import ctypes
    import torch
    from paper_2606_06386_amd import build as hb
    hb.LIB = hb.TRACE_LIB                    # before the binding loads the library
    from paper_2606_06386_amd import binding
    set_knobs(args)
    c = workload(args.config)
    u_h, v_h, nq = c["u"], c["v"], c["nq"]
    batch = len(u_h)
    assert batch <= 8192 and threads_for(u_h.shape[1]) == 256, "the trace buffer covers k_divrem<256>, 8192 blocks"
    dev = torch.device("cuda:0")
    u = torch.from_numpy(u_h.view(np.int32)).to(dev)
    v = torch.from_numpy(v_h.view(np.int32)).to(dev)
    out = (torch.empty((batch, nq), dtype=torch.int32, device=dev),
           torch.empty((batch, v_h.shape[1]), dtype=torch.int32, device=dev),
           torch.empty(batch, dtype=torch.int32, device=dev))
    settle(lambda: binding.divrem(u, v, out=out), torch.cuda.current_stream())
    for _ in range(max(1, args.warmup)):
        binding.divrem(u, v, out=out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    binding.divrem(u, v, out=out)
    e1.record()
    torch.cuda.synchronize()
    L = binding.lib()
    L.mp_trace_read_divrem.argtypes = [ctypes.c_void_p, ctypes.c_int]
    L.mp_trace_read_divrem.restype = ctypes.c_int
    st = np.zeros((batch, 32), dtype=np.uint64)
    assert L.mp_trace_read_divrem(st.ctypes.data, batch) == 0
    st = st.astype(np.float64)
    full = (st[:, :9] > 0).all(axis=1) & (np.diff(st[:, :9], axis=1) >= 0).all(axis=1)
    rows = st[full]
    res = {}
    for name, a, b in PHASES:
        res[name] = float(np.mean(rows[:, b] - rows[:, a]))
    prev = rows[:, 4].copy()
    last = prev.copy()
    for i in range(16):
        col = rows[:, 16 + i]
        if not (col > 0).any():
            continue
        res["iter_%d" % i] = float(np.mean(col - prev))
        prev = np.where(col > 0, col, prev)
        last = prev
    res["u_times_s"] = float(np.mean(rows[:, 5] - last))
    # sub-steps of the last Refine iteration (stamps 11-13 hold its values)
    it_end = [16 + i for i in range(16) if (rows[:, 16 + i] > 0).any()]
    if len(it_end) >= 2 and (rows[:, [11, 12, 13]] > 0).all():
        prev_end, end = rows[:, it_end[-2]], rows[:, it_end[-1]]
        res["last_iter_powdiff_product"] = float(np.mean(rows[:, 11] - prev_end))
        res["last_iter_residual"] = float(np.mean(rows[:, 12] - rows[:, 11]))
        res["last_iter_step_product"] = float(np.mean(rows[:, 13] - rows[:, 12]))
        res["last_iter_step_add"] = float(np.mean(end - rows[:, 13]))
    # the head launch (one wave per instance): its own stamps
    L.mp_trace_read_head.argtypes = [ctypes.c_void_p, ctypes.c_int]
    L.mp_trace_read_head.restype = ctypes.c_int
    hs = np.zeros((batch, 32), dtype=np.uint64)
    assert L.mp_trace_read_head(hs.ctypes.data, batch) == 0
    hs = hs.astype(np.float64)
    hfull = (hs[:, [0, 1, 2, 3, 4]] > 0).all(axis=1)
    hr = hs[hfull]
    head = {"instances": int(hfull.sum())}
    if len(hr):
        head["precisions"] = float(np.mean(hr[:, 1] - hr[:, 0]))
        head["stage_v"] = float(np.mean(hr[:, 2] - hr[:, 1]))
        head["initial_approx"] = float(np.mean(hr[:, 3] - hr[:, 2]))
        prev_h = hr[:, 3].copy()
        for i in range(16):
            col = hr[:, 16 + i]
            if not (col > 0).any():
                continue
            head["iter_%d" % i] = float(np.mean(np.where(col > 0, col - prev_h, 0)))
            prev_h = np.where(col > 0, col, prev_h)
        # sub-steps of iterations 3 and 6 (PowDiff product, residual, Step product, Step add)
        for i, sl in ((3, 5), (6, 8)):
            if "iter_%d" % i not in head or "iter_%d" % (i - 1) not in head:
                continue
            ok = (hr[:, [15 + i, sl, sl + 1, sl + 2, 16 + i]] > 0).all(axis=1)
            if ok.any():
                r = hr[ok]
                t = [r[:, 15 + i], r[:, sl], r[:, sl + 1], r[:, sl + 2], r[:, 16 + i]]
                head["iter_%d_steps" % i] = [float(np.mean(t[j + 1] - t[j])) for j in range(4)]
        # real-time stamps (100 MHz) at each head's start and end: the spread
        # of starts (dispatch) and of durations behind the kernel's length
        rt = hs[hfull][:, [14, 15]]
        if (rt > 0).all():
            st_us, en_us = (rt[:, 0] - rt[:, 0].min()) / RT_HZ * 1e6, (rt[:, 1] - rt[:, 0].min()) / RT_HZ * 1e6
            dur = en_us - st_us
            head["realtime_us"] = {"start_p50": float(np.percentile(st_us, 50)), "start_max": float(st_us.max()),
                                   "duration_p50": float(np.percentile(dur, 50)),
                                   "duration_p90": float(np.percentile(dur, 90)), "duration_max": float(dur.max()),
                                   "end_max": float(en_us.max())}
            # medians per quarter of the head workgroups, in launch order
            wgq = (np.nonzero(hfull)[0] // kHEAD_WAVES) * 4 // max(1, -(-len(hs) // kHEAD_WAVES))
            head["realtime_us"]["duration_p50_by_wg_quarter"] = [float(np.median(dur[wgq == r])) if (wgq == r).any()
                                                                 else None for r in range(4)]
        head["record"] = float(np.mean(hr[:, 4] - prev_h))
        head["total"] = float(np.mean(hr[:, 4] - hr[:, 0]))
        head["span_all_waves"] = float(hr[:, 4].max() - hr[:, 0].min())
    res["v_times_q"] = float(np.mean(rows[:, 6] - rows[:, 5]))
    res["corrections"] = float(np.mean(rows[:, 7] - rows[:, 6]))
    res["store"] = float(np.mean(rows[:, 8] - rows[:, 7]))
    total = float(np.mean(rows[:, 8] - rows[:, 0]))
    # every product of the body: shape, conversion, strips of the first wave, carries
    L.mp_trace_read_products.argtypes = [ctypes.c_void_p, ctypes.c_int]
    L.mp_trace_read_products.restype = ctypes.c_int
    pt = np.zeros((batch, 48, 6), dtype=np.uint64)
    assert L.mp_trace_read_products(pt.ctypes.data, batch) == 0
    prods = []
    ptf = pt[full]
    ref = ptf[0]
    for j in range(48):
        # the instances whose j-th product has the reference instance's shape
        same = (ptf[:, j, 0] == ref[j, 0]) & (ptf[:, j, 1] == ref[j, 1]) & (ptf[:, j, 5] >= ptf[:, j, 2]) & \
            (ptf[:, j, 2] > 0)
        if ref[j, 2] == 0 or not same.any():
            break
        r = ptf[same][:, j, :].astype(np.float64)
        sh0, sh1 = int(ref[j, 0]), int(ref[j, 1])
        prods.append({"short": sh0 & 0xFFFFFFFF, "long": sh0 >> 32, "ncols": sh1 & 0xFFFFFFFF, "c0": sh1 >> 32,
                      "instances": int(same.sum()),
                      "operands": float(np.mean(r[:, 3] - r[:, 2])), "strips": float(np.mean(r[:, 4] - r[:, 3])),
                      "carries": float(np.mean(r[:, 5] - r[:, 4])), "total": float(np.mean(r[:, 5] - r[:, 2]))})
    print(json.dumps({"phase_trace": c["name"], "kernel": "k_divrem<256>", "head": head, "products": prods,
                      "instances": int(full.sum()),
                      "knobs": knobs_now(), "clock": "shader cycles (s_memtime) of workgroup thread 0",
                      "body_clock": clock_stats(st[:, 0], st[:, 8], st[:, 14], st[:, 15], e0.elapsed_time(e1)),
                      "total_cycles": total, "cycles": res,
                      "share": {k: v / total for k, v in res.items()}}), flush=True)


def phase_trace_mul(args, na=2048, nb=2048, batch=4096):
    """Per-phase cycle breakdown of one mp_mul_batch launch (the trace build):
    clearing, digit conversion, the first wave's matrix-core strips, strip
    carries, the copy out.  Prints one JSON line."""
    import ctypes
    import torch
    from paper_2606_06386_amd import build as hb
    hb.LIB = hb.TRACE_LIB
    from paper_2606_06386_amd import binding
    g = torch.Generator(device="cuda:0").manual_seed(7)
    a = torch.randint(-2 ** 31, 2 ** 31, (batch, na), dtype=torch.int32, device="cuda:0", generator=g)
    b = torch.randint(-2 ** 31, 2 ** 31, (batch, nb), dtype=torch.int32, device="cuda:0", generator=g)
    settle(lambda: binding.mul(a, b), torch.cuda.current_stream())
    for _ in range(3):
        binding.mul(a, b)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    binding.mul(a, b)
    e1.record()
    torch.cuda.synchronize()
    L = binding.lib()
    L.mp_trace_read_mul.argtypes = [ctypes.c_void_p, ctypes.c_int]
    L.mp_trace_read_mul.restype = ctypes.c_int
    st = np.zeros((batch, 32), dtype=np.uint64)
    assert L.mp_trace_read_mul(st.ctypes.data, batch) == 0
    st = st.astype(np.float64)
    rows = st[(st[:, [0, 1, 2, 3, 4, 5, 10]] > 0).all(axis=1)]
    ph = {"clear": (0, 1), "digit_conversion": (1, 2), "strips_first_wave": (2, 10), "strips_wait_and_carries": (10, 3),
          "sync": (3, 4), "copy_out": (4, 5)}
    res = {k: float(np.mean(rows[:, b_] - rows[:, a_])) for k, (a_, b_) in ph.items()}
    total = float(np.mean(rows[:, 5] - rows[:, 0]))
    clk = clock_stats(st[:, 0], st[:, 5], st[:, 6], st[:, 7], e0.elapsed_time(e1))
    print(json.dumps({"phase_trace": "mul %dx%d batch %d" % (na, nb, batch), "kernel": "k_mul<256>",
                      "workgroups": len(rows), "total_cycles": total, "cycles": res,
                      "share": {k: v / total for k, v in res.items()}, "clock": clk}), flush=True)


def set_knobs(args):
    from paper_2606_06386_amd import binding
    if args.mfma_min is not None:
        binding.set_knob(binding.MP_KNOB_MFMA_MIN, args.mfma_min)
    if args.small_limit is not None:
        binding.set_knob(binding.MP_KNOB_SMALL_LIMIT, args.small_limit)


def knobs_now():
    from paper_2606_06386_amd import binding
    sl = binding.get_knob(binding.MP_KNOB_SMALL_LIMIT)
    return {"mfma_min": binding.get_knob(binding.MP_KNOB_MFMA_MIN),
            "small_limit": "auto (136 with several rounds of workgroups, else 96)"
            if sl == binding.MP_SMALL_LIMIT_AUTO else sl}


def run_mixed(args):
    """The mixed-precision batch: one mp_divrem_ragged call per step."""
    import torch
    import oracle
    from paper_2606_06386_amd import binding, inputs as I, ragged as R, tune
    c = I.config_c4()
    us, vs = c["u"], c["v"]
    count = len(us)
    tuned, fresh = tune.ensure(log=lambda m: print(m, file=sys.stderr, flush=True))
    rb = binding.Ragged(R.pack(us, vs))
    stream = torch.cuda.current_stream()
    nset = settle(lambda: rb.run(stream), stream)
    for _ in range(args.warmup):
        rb.run(stream)
    elapsed, ms = _timed(lambda: rb.run(stream), args.steps, stream)
    kmean = sum(ms) / len(ms)

    # the same launch sequence captured once in a graph and replayed
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        rb.run()                                  # the side stream's fork set, outside capture
        with torch.cuda.graph(g, stream=side):
            rb.run()
    stream.wait_stream(side)
    torch.cuda.synchronize()
    for _ in range(max(1, args.warmup // 4)):
        g.replay()
    _, gms = _timed(g.replay, args.steps, stream)
    gmean = sum(gms) / len(gms)

    # the same divisions as four uniform launches (one per dividend width)
    groups = []
    for n in I.C4_WIDTHS:
        js = [j for j in range(count) if len(us[j]) == n]
        v = np.zeros((len(js), n), dtype=np.uint32)
        for i, j in enumerate(js):
            v[i, :len(vs[j])] = vs[j]
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).cuda()
        ud, vd = t(np.stack([us[j] for j in js])), t(v)
        out = (torch.empty((len(js), n), dtype=torch.int32, device="cuda"),
               torch.empty((len(js), n), dtype=torch.int32, device="cuda"),
               torch.empty(len(js), dtype=torch.int32, device="cuda"))
        groups.append((ud, vd, out))

    def plain():
        for ud, vd, out in groups:
            binding.divrem(ud, vd, out=out, stream=stream)
    for _ in range(max(1, args.warmup // 4)):
        plain()
    _, pms = _timed(plain, max(3, args.steps // 4), stream)
    pmean = sum(pms) / len(pms)

    status = rb.status.cpu().numpy()
    qp, rp = rb.q.cpu().numpy().view(np.uint32), rb.r.cpu().numpy().view(np.uint32)
    packed_desc = np.frombuffer(rb.desc.cpu().numpy().tobytes(), dtype=R.DESC_DTYPE)
    qs, rs = R.unpack(qp, packed_desc, "q"), R.unpack(rp, packed_desc, "r")
    W = ragged_limb_products(us, vs)
    algo_bytes = 4 * sum(2 * len(u) + 2 * len(v) for u, v in zip(us, vs)) + 4 * count + 48 * count
    line = {
        "metric": METRIC,
        "value": count * args.steps / elapsed,
        "unit": "div/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "settle": {"min_ms": SETTLE_MS, "steps": nset,
                   "what": "untimed steps before the warm-up, until the shader clock has left its ramp from idle"},
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": c["name"], "bits": "2^15..2^18 mixed", "batch": count,
                   "widths": list(I.C4_WIDTHS), "nv": "uniform in [ceil(n/4), n]"},
        "kernel_ms": {"mean": kmean, "median": ms[len(ms) // 2], "min": ms[0]},
        "graph_replay_ms": {"mean": gmean, "median": gms[len(gms) // 2], "min": gms[0]},
        "uniform_launches_ms": {"mean": pmean, "min": pms[0]},
        "ragged_over_uniform": pmean / kmean, "graph_over_uniform": pmean / gmean,
        "tuned": tuned, "tuned_now": fresh,
        "limb_products_per_launch": W,
        "limb_products_per_launch_full_products": ragged_limb_products(us, vs, clipped=False),
        "roofline": roofline(ragged_limb_products(us, vs, clipped=False), W, kmean,
                             "k_ragged_prep + k_head_ragged + k_ragged (4 width classes)", None, algo_bytes),
        "status_ok": int((status == 0).sum()),
    }
    if not args.no_cpu_baseline:
        # the oracle on the first instances (grouped by width), checked against the GPU
        m, t_cpu, exact, used = 0, 0.0, 0, 0
        while t_cpu < 10.0 and m < count:
            js = list(range(m, min(count, m + 64)))
            for n in I.C4_WIDTHS:
                g = [j for j in js if len(us[j]) == n]
                if not g:
                    continue
                v = np.zeros((len(g), n), dtype=np.uint32)
                for i, j in enumerate(g):
                    v[i, :len(vs[j])] = vs[j]
                t0 = time.perf_counter()
                qo, ro, so, used = oracle.divrem_threads(np.stack([us[j] for j in g]), v, n, n)
                t_cpu += time.perf_counter() - t0
                exact += sum(int((qo[i] == qs[j]).all() and (ro[i, :len(vs[j])] == rs[j]).all()
                                 and not ro[i, len(vs[j]):].any()) for i, j in enumerate(g))
            m = js[-1] + 1
        line["cpu_baseline"] = {"value": m / t_cpu, "unit": "div/s", "cores": int(used), "kind": "oracle",
                                "sample": f"first {m} of {count} instances of {c['name']} "
                                          "(Knuth D, gcc -O2, OpenMP, per width)"}
        line["parity_sample"] = f"{exact}/{m} bit-exact vs oracle"
    print(json.dumps(line), flush=True)


def serving_run(rate, count, ops=None, path="ragged", depth=3):
    """One serving run of the 2^15..2^18-bit request trace at `rate` arrivals/s
    through the ragged (continuous batching) or the plain per-width path;
    returns its summary (latencies in ms, upload and download included)."""
    from paper_2606_06386_amd import inputs as I, serve
    c = ops if ops is not None else I.config_c5(rate, count=count)
    arrival = I.c5_arrivals(rate, count)
    res = serve.serve(c["u"][:count], c["v"][:count], arrival, path=path, depth=depth)
    lat = res["latency"] * 1e3
    st = res["requests"].status.numpy()
    return {"path": path, "rate_per_s": rate, "requests": count, "div_per_s": res["div_per_s"],
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_batch": float(np.mean(res["batches"])), "batches": len(res["batches"]),
            "host_launch_share": res["host_launch_s"] / max(res["span_s"], 1e-9),
            "status_ok": int((st == 0).sum())}, res


def serving_parity(ops, res, count, every=250):
    """a sample of a serving run's results against the oracle"""
    import oracle
    q, r, st = res["requests"].results()
    js = list(range(0, count, every))
    exact = 0
    for j in js:
        qo, ro, so = oracle.divrem(ops["u"][j][None, :], ops["v"][j][None, :], nq=len(ops["u"][j]),
                                   nr=len(ops["v"][j]))
        exact += int(so[0] == st[j] and (qo[0] == q[j]).all() and (ro[0] == r[j]).all())
    return f"{exact}/{len(js)} bit-exact vs oracle"


def serving_compare(count=10000, rates=(1e6,), parity=True):
    """Serving and the plain path on the same arrival traces, and both as one
    device-resident batch (throughput only)."""
    from paper_2606_06386_amd import inputs as I, serve, tune
    tune.ensure(log=lambda m: print(m, file=sys.stderr, flush=True))
    ops = I.config_c5(1e3, count=count)
    # warm-up at full size: first launches, the slot streams and the pinned
    # request pools (a freshly pinned pool is slow on its first transfers)
    serving_run(max(rates), count, ops)
    serving_run(max(rates), count, ops, path="plain")
    out = {"workload": "serve_2p15_2p18_n%d" % count, "rates": []}
    for rate in rates:
        row_s, res = serving_run(rate, count, ops)
        row_p, res_p = serving_run(rate, count, ops, path="plain")
        row = {"rate_per_s": rate, "serving": row_s, "plain": row_p,
               "serving_over_plain": row_s["div_per_s"] / max(row_p["div_per_s"], 1e-9)}
        if parity:
            row["serving"]["parity_sample"] = serving_parity(ops, res, count)
            row["plain"]["parity_sample"] = serving_parity(ops, res_p, count)
        out["rates"].append(row)
        print(json.dumps(row), file=sys.stderr, flush=True)
    out["all_at_once"] = {"ragged": serve.all_at_once(ops["u"], ops["v"], "ragged"),
                          "plain_four_launches": serve.all_at_once(ops["u"], ops["v"], "plain")}
    return out


def run_serving(args):
    res = serving_compare(rates=(1e3, 1e4, 1e5, 1e6))
    top = res["rates"][-1]
    line = {
        "metric": METRIC, "value": top["serving"]["div_per_s"], "unit": "div/s", "n_gpus": 1,
        "steps": len(res["rates"]), "warmup": 0, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": res["workload"], "bits": "2^x, x ~ U[15, 18]", "nv": "uniform in [ceil(n/8), n]",
                   "arrivals": "Poisson", "admission": "HBM free share and LDS residency", "depth": 3},
        "serving": res,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", default="c2", choices=["c1", "c2", "c3", "c4", "c5", "mul"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--probe", action="store_true", help="measure integer instruction issue rates instead")
    ap.add_argument("--no-serving", action="store_true", help="skip the short serving run")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the product timings, the end-to-end run and the other precisions")
    ap.add_argument("--write-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the traffic record of --config's workload from two counter files and exit")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="end with one 256 MiB device copy (reference for HBM byte counters)")
    ap.add_argument("--mfma-min", type=int, default=None,
                    help="knob: shortest product operand (limbs) run on the matrix cores (huge = vector ALU only)")
    ap.add_argument("--small-limit", type=int, default=None,
                    help="knob: Refine iterations with a shorter iterate run on one wave")
    ap.add_argument("--phase-trace", action="store_true",
                    help="per-phase cycle breakdown from the trace build of the library instead")
    ap.add_argument("--phase-trace-mul", action="store_true",
                    help="per-phase cycle breakdown of the 2048 x 2048-limb product kernel instead")
    args = ap.parse_args()
    if args.write_traffic:
        write_traffic(*args.write_traffic, workload_name={"c1": "divrem_2p15_b1024", "c2": "divrem_2p16_b4096",
                                                          "c3": "divrem_2p18_b256"}[args.config])
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: division instances are independent, so a multi-GPU "
              "run would only split the batch; --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2606_06386_amd import binding

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.probe:
        probe_rates()
        return
    if args.phase_trace:
        phase_trace(args)
        return
    if args.phase_trace_mul:
        phase_trace_mul(args)
        return
    set_knobs(args)
    if args.config == "c4":
        run_mixed(args)
        return
    if args.config == "c5":
        run_serving(args)
        return
    if args.config == "mul":
        # the product the method is parameterised by, at 2^16 bits: full
        # 2048 x 2048-limb products and the 2048 x 1025 shape of u * shinv
        stream = torch.cuda.current_stream()
        res = {n: time_mul(binding, a, b, 4096, args.steps, args.warmup, stream)
               for n, (a, b) in {"2048x2048": (2048, 2048), "2048x1025": (2048, 1025)}.items()}
        print(json.dumps({"metric": "mp_mul_batch limb products/s", "value": res["2048x2048"]["limb_products_per_s"],
                          "unit": "limb products/s", "config": {"workload": "mul_2p16_b4096", "batch": 4096},
                          "mul": res}), flush=True)
        return
    stream = torch.cuda.current_stream()
    c = workload(args.config)
    elapsed, ms, q_h, r_h, status, dev_bufs, nset = time_divrem(binding, c, args.steps, args.warmup, stream)
    res = plain_result(c, elapsed, ms, q_h, r_h, status, args.steps)
    u_h, v_h = c["u"], c["v"]
    batch = len(u_h)
    line = {
        "metric": METRIC,
        "value": res["div_per_s"],
        "unit": "div/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "settle": {"min_ms": SETTLE_MS, "steps": nset,
                   "what": "untimed steps before the warm-up, until the shader clock has left its ramp from idle"},
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": c["name"], "bits": c["bits"], "batch": batch, "nu": int(u_h.shape[1]),
                   "nv": int(v_h.shape[1]), "nq": c["nq"]},
        "kernel_ms": res["kernel_ms"],
        "roofline": res["roofline"],
        "full_mult_equivalents_per_s": res["full_mult_equivalents_per_s"],
        "status_ok": res["status_ok"],
        "knobs": knobs_now(),
    }
    del dev_bufs
    if args.copy_calibration:
        x = torch.empty(64 << 20, dtype=torch.int32, device="cuda:0")
        y = torch.ones_like(x)
        x.copy_(y)
        torch.cuda.synchronize()
        del x, y
    if not args.no_extras:
        # the paper's Table 1 column: time of the batch of divisions over a batch
        # of multiplications of the same precision and count
        n = int(u_h.shape[1])
        mul_full = time_mul(binding, n, n, batch, max(5, args.steps // 2), 3, stream)
        mul_q = time_mul(binding, n, n // 2 + 1, batch, max(5, args.steps // 2), 3, stream)
        line["mul"] = {"%dx%d" % (n, n): mul_full, "%dx%d" % (n, n // 2 + 1): mul_q}
        line["t_div_over_t_mul"] = res["kernel_ms"]["mean"] / mul_full["ms"]
        line["end_to_end"] = time_end_to_end(binding, c, max(5, args.steps // 2), stream)
        if args.config == "c2":
            # the other plain precisions, each checked against the oracle in full
            import oracle
            subs = {}
            for name in ("c1", "c3"):
                cs = workload(name)
                el, ms2, q2, r2, st2, bufs, _ = time_divrem(binding, cs, max(5, args.steps // 2), 3, stream)
                sub = plain_result(cs, el, ms2, q2, r2, st2, max(5, args.steps // 2))
                del bufs
                if not args.no_cpu_baseline:
                    qo, ro, so = oracle.divrem(cs["u"], cs["v"], nq=cs["nq"], nr=cs["v"].shape[1])
                    ok = ((qo == q2).all(axis=1) & (ro == r2).all(axis=1) & (so == st2)).sum()
                    sub["parity_sample"] = f"{int(ok)}/{len(q2)} bit-exact vs oracle"
                subs[name] = sub
            line["configs"] = subs
    if not args.no_serving:
        # serving beside the throughput (outside the timed region): 10^4
        # requests of 2^15..2^18 bits arriving at 10^6 per second, served with
        # continuous batching and through the plain per-width path on the same
        # trace; latency from arrival to results in host memory
        line["serving"] = serving_compare(rates=(1e6,), parity=not args.no_cpu_baseline)
    if not args.no_cpu_baseline:
        cb, exact, n_cpu = cpu_baseline(c, q_h, r_h)
        line["cpu_baseline"] = cb
        line["parity_sample"] = f"{exact}/{n_cpu} bit-exact vs oracle"
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
