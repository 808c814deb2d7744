"""Build step for libmpdiv.so, the HIP library behind include/mpdiv.h.

Compiles csrc/mpdiv.hip for gfx950 with hipcc into libmpdiv.so next to this
file (in-tree, so the built library travels with the source tree).
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libmpdiv.so")
SOURCES = [os.path.join(HERE, "csrc", "mpdiv.hip")]
# instruction issue-rate probe (calibrates the integer-multiply roofline)
PROBE_LIB = os.path.join(HERE, "libmpprobe.so")
PROBE_SOURCES = [os.path.join(HERE, "csrc", "probe_rates.hip")]
HEADERS = [os.path.join(HERE, "csrc", f) for f in ("mp_prims_hip.hpp", "mp_core.hpp", "mp_div.hpp")]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed-FP32 instruction selection anywhere in this library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-command-line-argument",
]


def _hipcc(out, sources, verbose):
    tmp = out + ".tmp"
    cmd = ["hipcc", *HIPCC_FLAGS, "-o", tmp, *sources]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)


def build(verbose: bool = False) -> str:
    _hipcc(LIB, SOURCES, verbose)
    _hipcc(PROBE_LIB, PROBE_SOURCES, verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
