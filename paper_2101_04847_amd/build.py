"""Build liblb.so (the gfx950 HIP library behind include/lb.h) in-tree.

    python -m paper_2101_04847_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "liblb.so")
PROBE = os.path.join(PKG, "bw_probe")
PROBE_LIB = os.path.join(PKG, "libbwprobe.so")
SOURCES = [os.path.join(CSRC, "lb.hip"), os.path.join(CSRC, "lb3.hip")]
HEADERS = [os.path.join(CSRC, "lb_kernels.hpp"), os.path.join(CSRC, "lb_internal.hpp"),
           os.path.join(CSRC, "lb_memory.hpp"),
           os.path.join(CSRC, "lb3_kernels.hpp"), os.path.join(ROOT, "include", "lb.h"),
           os.path.join(ROOT, "include", "lb3.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # FP64 results are defined by the order of the model's expressions:
    # no FMA contraction anywhere.
    "-ffp-contract=off",
    # no packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
]


def _report_warnings(text: str) -> None:
    """Echo compiler warnings; the host pass's note that it does not know the
    device-only packed-fp32 feature is expected and dropped."""
    lines = [ln for ln in text.splitlines() if ln.strip() and "packed-fp32-ops" not in ln]
    if lines:
        sys.stderr.write("\n".join(lines) + "\n")


def build(verbose: bool = False) -> str:
    """Compile every source into liblb.so (always recompiles)."""
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, *FLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-o", tmp, *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building liblb.so")
    _report_warnings(res.stderr)
    os.replace(tmp, LIB)
    # the bandwidth probe (measured roofline denominator): a shared library
    # for in-process use by the benchmark and a stand-alone program
    for out, extra in ((PROBE_LIB, ["-fPIC", "-shared"]), (PROBE, ["-DBW_PROBE_MAIN"])):
        tmp = out + ".tmp%d" % os.getpid()
        cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
               "-packed-fp32-ops", *extra, "-o", tmp, os.path.join(CSRC, "bw_probe.hip")]
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError("hipcc failed building " + os.path.basename(out))
        os.replace(tmp, out)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
