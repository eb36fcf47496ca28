"""Build step for libosc.so (the HIP kernels and the C ABI of include/osc.h).

Compiles the sources under ``csrc/`` for gfx950 with hipcc into
``paper_1311_7579_amd/libosc.so``.  Packed FP32 instructions are switched
off for the device code; the host pass warns that it does not know that
target feature, which is harmless.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libosc.so")
SOURCES = ["osc_host.hip", "osc_kernels.hip", "osc_batch.hip", "osc_serve.hip", "osc_template.hip"]
ARCH = os.environ.get("OSC_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    # FMA contraction only within one expression (and never where a
    # "#pragma clang fp contract(off)" says so): every kernel instantiation
    # then rounds the same arithmetic the same way
    "-ffp-contract=on", "-Wall",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # interleave independent events within a wave (occupancy is bounded by
    # the LDS histograms, not by registers)
    "-mllvm", "-amdgpu-sched-strategy=max-ilp",
    "-I", os.path.join(ROOT, "include"),
]


def hipcc() -> str:
    for cand in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), "hipcc"):
        if os.path.sep not in cand or os.path.exists(cand):
            return cand
    return "hipcc"


def build(verbose: bool = False, extra=()) -> str:
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *HIPCC_FLAGS, *extra, "-o", tmp] + [os.path.join(CSRC, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libosc.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
