"""Build-time check of the generated gfx950 ISA: the kernels must not write
through the scalar data cache (scalar stores, scalar atomics, or the scalar
cache's write-back/invalidate-for-write instructions).  Run on the build
machine only; not shipped to GPU runs.
"""
import re
import subprocess

FORBIDDEN = re.compile(r"^\s*(s_store_|s_buffer_store|s_scratch_store|s_atomic|s_buffer_atomic|s_dcache_wb|s_dcache_discard)", re.M)


def check(hipcc, flags, hip_sources):
    for src in hip_sources:
        cmd = [hipcc] + flags + ["--cuda-device-only", "-S", "-o", "-", src]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("ISA dump failed: " + r.stderr[-2000:])
        bad = FORBIDDEN.findall(r.stdout)
        if bad:
            raise RuntimeError(f"{src}: forbidden scalar-cache write instructions: {sorted(set(bad))}")
