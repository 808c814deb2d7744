"""Benchmark: batched exact division at 2^16 bits on one MI355X.

One step = one mp_divrem_batch launch over the whole workload (every
instance goes through shifted inverse, quotient product, remainder product
and corrections).  Inputs are device-resident before the timed region.
Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--config c2|c1|c3] [--no-cpu-baseline]
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

# Integer-multiply roofline of MI355X: 256 CUs x 4 SIMDs at 2.4 GHz, each SIMD
# issuing one wave64 v_mad_u64_u32 (64 limb products of 32x32->64 bits) every
# 4 cycles, i.e. 64 limb products per clock per CU.  (Simple 32-bit ALU ops
# such as v_add_u32 issue twice as fast on gfx950; the probe mode measures both.)
PEAK_LIMB_PRODUCTS = 256 * 4 * 16 * 2.4e9


def prec_rows(x):
    """number of significant limbs of each row"""
    nz = x != 0
    return np.where(nz.any(axis=1), x.shape[1] - np.argmax(nz[:, ::-1], axis=1), 0)


def workload(name):
    from paper_2606_06386_amd import inputs as I
    return {"c1": I.config_c1, "c2": I.config_c2, "c3": I.config_c3}[name]()


def limb_products(u, v):
    """Algorithmic limb products of one launch over the batch (cost model W)."""
    from paper_2606_06386_amd import costmodel as cm
    hs, nvs = prec_rows(u), prec_rows(v)
    total = 0
    cache = {}
    for h, nvv in zip(hs.tolist(), nvs.tolist()):
        key = (h, nvv - 1)
        if key not in cache:
            cache[key] = cm.division_cost(h, nvv - 1) if nvv >= 2 and h >= nvv else 0
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
    h = hashlib.sha256(b"".join(open(os.path.join(ROOT, s), "rb").read() for s in rec["sources"])).hexdigest()
    return rec["traffic_bytes_per_dispatch"] if h == rec["source_sha256"] else None


def cpu_baseline(c, q_gpu, r_gpu, budget_s=10.0):
    """The oracle (plain C, OpenMP over instances) on a bounded sample of the
    same workload; also checks the GPU results of the sample bit-exactly."""
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
    return {"value": n / t, "unit": "div/s", "cores": int(used), "kind": "oracle",
            "sample": f"first {n} of {len(u)} instances of {c['name']} (Knuth D, gcc -O2, OpenMP)"}, exact, n


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", default="c2", choices=["c1", "c2", "c3"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--probe", action="store_true", help="measure integer instruction issue rates instead")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: every division instance is independent and this "
              "build runs on a single MI355X; --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2606_06386_amd import binding

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.probe:
        probe_rates()
        return
    dev = torch.device("cuda:0")
    c = workload(args.config)
    u_h, v_h, nq = c["u"], c["v"], c["nq"]
    batch = len(u_h)
    u = torch.from_numpy(u_h.view(np.int32)).to(dev)
    v = torch.from_numpy(v_h.view(np.int32)).to(dev)
    q = torch.empty((batch, nq), dtype=torch.int32, device=dev)
    r = torch.empty((batch, v_h.shape[1]), dtype=torch.int32, device=dev)
    st = torch.empty(batch, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        binding.divrem(u, v, out=(q, r, st), stream=stream)
    torch.cuda.synchronize()

    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        starts[i].record(stream)
        binding.divrem(u, v, out=(q, r, st), stream=stream)
        ends[i].record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kernel_ms = sorted(s.elapsed_time(e) for s, e in zip(starts, ends))
    kmean = sum(kernel_ms) / len(kernel_ms)

    status = st.cpu().numpy()
    q_h, r_h = q.cpu().numpy().view(np.uint32), r.cpu().numpy().view(np.uint32)
    W = limb_products(u_h, v_h)
    achieved = W / (kmean * 1e-3)
    algo_bytes = 4 * (u_h.size + v_h.size + q_h.size + r_h.size) + 4 * batch   # u, v in; q, r, status out
    line = {
        "metric": METRIC,
        "value": batch * args.steps / elapsed,
        "unit": "div/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": c["name"], "bits": c["bits"], "batch": batch, "nu": int(u_h.shape[1]),
                   "nv": int(v_h.shape[1]), "nq": nq},
        "kernel_ms": {"mean": kmean, "median": kernel_ms[len(kernel_ms) // 2], "min": kernel_ms[0]},
        "limb_products_per_launch": W,
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_LIMB_PRODUCTS / 1e12,
                     "unit": "T limb-products/s", "frac": achieved / PEAK_LIMB_PRODUCTS,
                     "traffic": measured_traffic(c["name"]), "traffic_unit": "bytes/launch",
                     "algorithmic_bytes": algo_bytes, "kernel": "k_divrem"},
        "status_ok": int((status == 0).sum()),
    }
    if not args.no_cpu_baseline:
        cb, exact, n = cpu_baseline(c, q_h, r_h)
        line["cpu_baseline"] = cb
        line["parity_sample"] = f"{exact}/{n} bit-exact vs oracle"
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
