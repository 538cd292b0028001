"""Builds libacopf.so (host C++ + gfx950 kernels) in-tree with hipcc.

    python -m paper_2203_10587_amd.build
"""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libacopf.so")
SOURCES = ["acopf_host.cpp", "acopf_batch.cpp", "acopf_kernels.hip", "acopf_rng.hip",
           "acopf_couple.hip", "acopf_reduce.hip"]
ARCH = "gfx950"

HIP_FLAGS = [
    "-x", "hip", "-std=c++17", "-O3", f"--offload-arch={ARCH}", "-fPIC",
    # bitwise-reproducible arithmetic: no compiler-chosen fused multiply-adds
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
]


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.isabs(c) and os.path.exists(c) or not os.path.isabs(c)):
            return c
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    """Compile every source into libacopf.so; returns its path."""
    srcs = [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    tmp = LIB + ".tmp"
    cmd = [_hipcc()] + HIP_FLAGS + ["-shared", "-o", tmp] + srcs
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libacopf.so")
    os.replace(tmp, LIB)
    # Optional check of the generated ISA (only present where it is built).
    chk = os.path.join(CSRC, "isa_check.py")
    if os.path.exists(chk):
        import importlib.util
        spec = importlib.util.spec_from_file_location("isa_check", chk)
        mod = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(mod)
        mod.check(_hipcc(), HIP_FLAGS, [s for s in srcs if s.endswith(".hip")])
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
