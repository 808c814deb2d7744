"""Build step for libmpdiv.so, the HIP library behind include/mpdiv.h.

Compiles the sources in csrc/ for gfx950 with hipcc into libmpdiv.so next to
this file (in-tree, so the built library travels with the source tree).
kernels.hip is compiled once per kernel family and workgroup size (each
object holds one launcher and its kernel) and once for the head kernels, and all objects are compiled in
parallel, then linked with the host API (mpdiv.hip).
"""
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJDIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmpdiv.so")
# diagnostic variant: the same kernels with phase stamps (MP_PHASE_TRACE), built on request only
TRACE_LIB = os.path.join(HERE, "libmpdiv_trace.so")
# instruction issue-rate probe (calibrates the integer-multiply roofline)
PROBE_LIB = os.path.join(HERE, "libmpprobe.so")
PROBE_SOURCES = [os.path.join(CSRC, "probe_rates.hip")]
HEADERS = [os.path.join(CSRC, f) for f in ("mp_prims_hip.hpp", "mp_core.hpp", "mp_div.hpp", "launch.hpp")]

# (object name, source, defines): one object per kernel family x workgroup size
FAMILIES = {0: "mul", 1: "shinv", 2: "divrem", 3: "ragged"}
THREADS = (256, 512, 1024)
UNITS = [("api", "mpdiv.hip", []), ("k_head", "kernels.hip", ["-DMP_KFAMILY=4", "-DMP_KT=64"])] + [
    (f"k_{name}_{t}", "kernels.hip", [f"-DMP_KFAMILY={fam}", f"-DMP_KT={t}"])
    for fam, name in FAMILIES.items() for t in THREADS]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed-FP32 instruction selection anywhere in this library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-command-line-argument",
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def _compile(unit, verbose, extra=(), objdir=OBJDIR):
    name, src, defs = unit
    out = os.path.join(objdir, name + ".o")
    _run(["hipcc", *HIPCC_FLAGS, *extra, *defs, "-c", "-o", out, os.path.join(CSRC, src)], verbose)
    return out


def build_objects(verbose=False, extra=(), jobs=None, objdir=OBJDIR):
    """Compile every unit (in parallel); returns the object paths."""
    os.makedirs(objdir, exist_ok=True)
    jobs = jobs or min(len(UNITS), max(1, os.cpu_count() or 1), 16)
    with ThreadPoolExecutor(jobs) as ex:
        return list(ex.map(lambda u: _compile(u, verbose, extra, objdir), UNITS))


def link(objs, out, verbose=False):
    tmp = out + ".tmp"
    _run(["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs], verbose)
    os.replace(tmp, out)


def build(verbose: bool = False) -> str:
    link(build_objects(verbose), LIB, verbose)
    _run(["hipcc", *HIPCC_FLAGS, "-shared", "-o", PROBE_LIB + ".tmp", *PROBE_SOURCES], verbose)
    os.replace(PROBE_LIB + ".tmp", PROBE_LIB)
    return LIB


def build_trace(verbose: bool = False) -> str:
    """libmpdiv_trace.so: every kernel with its phase stamps (bench.py --phase-trace)."""
    link(build_objects(verbose, extra=("-DMP_PHASE_TRACE",), objdir=os.path.join(OBJDIR, "trace")), TRACE_LIB,
         verbose)
    return TRACE_LIB


if __name__ == "__main__":
    import sys
    print(build_trace(verbose=True) if "--trace" in sys.argv else build(verbose=True))
