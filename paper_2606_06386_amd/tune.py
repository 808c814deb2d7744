"""Autotuner for the launch configuration of mixed-precision batches.

For each dividend width class of mp_divrem_ragged (<= 1024, 2048, 4096, 8192
limbs) it times a one-class batch of seeded random divisions under every
valid (threads per workgroup, hence limbs per thread in the linear passes;
persistent workgroups per compute unit) and installs the fastest with
mp_ragged_config.  Then, on a seeded mixed batch, it times the two
process-wide knobs of the method's schedule and product engine: where the
Newton precision-doubling schedule hands over from the one-wave head to the
per-instance workgroups (MP_KNOB_SMALL_LIMIT) and from which operand length
products move from the vector ALU to the matrix cores (MP_KNOB_MFMA_MIN),
and installs the fastest pair.  Results are cached in a JSON file keyed by
the device (architecture name and compute-unit count) and by a hash of the
kernel sources, so a cache entry is never applied to a different chip or to
changed kernels.  Timing runs on the GPU; nothing here computes any part of
a division, and every setting gives the same bits.
"""
import hashlib
import json
import os

import numpy as np

from . import inputs as I

CLASS_WIDTHS = (1024, 2048, 4096, 8192)
THREADS = (256, 512, 1024)
WGS_PER_CU = (1, 2, 3, 4, 6, 8)
DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_ragged.json")
_CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")


def source_hash():
    h = hashlib.sha256()
    for f in sorted(os.listdir(_CSRC)):
        with open(os.path.join(_CSRC, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def device_key():
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return "%s/%dcu/%s" % (p.gcnArchName.split(":")[0], p.multi_processor_count, source_hash())


def candidates(cls):
    w = CLASS_WIDTHS[cls]
    return [(t, g) for t in THREADS if 8 * t >= w for g in WGS_PER_CU]


def class_batch(cls, count):
    """Seeded one-class divisions: width n of the class, divisor length
    uniform in [ceil(n/4), n] (the mixed workload's distribution)."""
    n = CLASS_WIDTHS[cls]
    st = I.instance_states(I.SEED_C4 ^ (0x7E0000 + cls), np.arange(count))
    nvs = I.uniform_int(I.substream(st, 2), (n + 3) // 4, n)
    s0, s1 = I.substream(st, 0), I.substream(st, 1)
    us = list(I.limbs_top_nonzero(s0, n))
    vs = [I.limbs_top_nonzero(s1[r:r + 1], int(nv))[0] for r, nv in enumerate(nvs)]
    return us, vs


def _time(rb, reps):
    import torch
    rb.run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        rb.run()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


AUTO = -2           # the library's per-launch head limit (MP_SMALL_LIMIT_AUTO)
SMALL_LIMITS = (AUTO, 32, 48, 64, 80, 96, 112, 128, 136)
MFMA_MINS = (32, 64, 96, 128)
AUTO_SLACK = 1.01    # the per-launch setting is kept unless a fixed one is >1% faster


def tune_knobs(count=1024, reps=3, log=None):
    """Time every (small_limit, mfma_min) pair on a seeded mixed batch (all four
    width classes); installs and returns the fastest as {knob: value, 'ms': ms}.
    The per-launch head limit (AUTO) adapts to each batch's size, so it is
    preferred over a fixed limit that is not clearly faster on this batch."""
    from . import binding, ragged
    m = I.config_c4(index=np.arange(0, 8 * count, 8))
    rb = binding.Ragged(ragged.pack(m["u"], m["v"]))
    times = []
    for sl in SMALL_LIMITS:
        for mm in MFMA_MINS:
            binding.set_knob(binding.MP_KNOB_SMALL_LIMIT, sl)
            binding.set_knob(binding.MP_KNOB_MFMA_MIN, mm)
            ms = _time(rb, reps)
            times.append((ms, sl, mm))
            if log:
                log("knobs small_limit %s, mfma_min %d: %.3f ms" % ("auto" if sl == AUTO else sl, mm, ms))
    ms, sl, mm = min(times)
    auto_ms, _, auto_mm = min(t for t in times if t[1] == AUTO)
    if auto_ms <= ms * AUTO_SLACK:
        ms, sl, mm = auto_ms, AUTO, auto_mm
    binding.set_knob(binding.MP_KNOB_SMALL_LIMIT, sl)
    binding.set_knob(binding.MP_KNOB_MFMA_MIN, mm)
    return {"small_limit": sl, "mfma_min": mm, "ms": ms}


def tune(counts=(2048, 1024, 512, 256), reps=3, log=None):
    """Time every candidate per class; returns {cls: (threads, wgs_per_cu, ms)}."""
    from . import binding, ragged
    best = {}
    for cls in range(len(CLASS_WIDTHS)):
        us, vs = class_batch(cls, counts[cls])
        rb = binding.Ragged(ragged.pack(us, vs))
        times = []
        for t, g in candidates(cls):
            binding.ragged_config(cls, t, g)
            ms = _time(rb, reps)
            times.append((ms, t, g))
            if log:
                log("class %d (<= %d limbs): threads %d, %d WG/CU: %.3f ms" % (cls, CLASS_WIDTHS[cls], t, g, ms))
        ms, t, g = min(times)
        binding.ragged_config(cls, t, g)
        best[cls] = (t, g, ms)
    return best


def apply(entry):
    """Install a cache entry: {'classes': {cls: (threads, wgs_per_cu, ms)},
    'knobs': {'small_limit': .., 'mfma_min': ..}}."""
    from . import binding
    for cls, (t, g, _) in entry["classes"].items():
        binding.ragged_config(int(cls), int(t), int(g))
    kn = entry.get("knobs")
    if kn:
        binding.set_knob(binding.MP_KNOB_SMALL_LIMIT, int(kn["small_limit"]))
        binding.set_knob(binding.MP_KNOB_MFMA_MIN, int(kn["mfma_min"]))


def ensure(cache=DEFAULT_CACHE, log=None):
    """Install the cached configuration for this device, tuning (and writing
    the cache, where writable) when there is none."""
    key = device_key()
    data = {}
    if os.path.exists(cache):
        with open(cache) as fh:
            data = json.load(fh)
    if key in data and "classes" in data[key]:
        apply(data[key])
        return data[key], False
    best = tune(log=log)
    knobs = tune_knobs(log=log)
    data[key] = {"classes": {str(k): list(v) for k, v in best.items()}, "knobs": knobs}
    try:
        with open(cache, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
    except OSError:
        pass
    return data[key], True
