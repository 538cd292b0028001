"""Host tiler of the bus tiles (no GPU): the positions each work item and
each bus lane store, checked against the CSR pattern column by column, and
coverage (every Jacobian and Hessian entry outside the flow and generator
blocks stored exactly once), for every tile size, on grids with parallel
branches, phase shifters and generator-free buses."""
import ctypes as C
import os
import shutil
import subprocess

import pytest

from paper_2203_10587_amd import acopf as A
from paper_2203_10587_amd import synth as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("tiler") / "libtile_check.so")
    cmd = [HIPCC, "-x", "hip", "-std=c++17", "-O1", "--offload-arch=gfx950", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I" + os.path.join(ROOT, "include"),
           "-I" + os.path.join(ROOT, "paper_2203_10587_amd", "csrc"),
           "-o", out, os.path.join(ROOT, "tests", "native", "tile_check.cpp")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    lib = C.CDLL(out)
    lib.tile_check.argtypes = [C.POINTER(A.acopf_net_desc), C.c_int, C.c_uint]
    return lib


GRIDS = {
    "ring9": lambda: S.random_grid(9, 12, 3, seed=1, parallel=1),
    "parallel60": lambda: S.random_grid(60, 95, 20, seed=5, parallel=3),
    "parallel400": lambda: S.random_grid(400, 700, 80, seed=7, parallel=3),
    "rgg2000": lambda: S.rgg_grid(2000, 3000, seed=3),
}


@pytest.mark.parametrize("name", sorted(GRIDS))
@pytest.mark.parametrize("tile_be", [64, 128, 256, 512])
def test_positions_and_coverage(checker, name, tile_be):
    d = A._Desc(GRIDS[name]())
    assert checker.tile_check(C.byref(d.desc), tile_be, 0) == 0


@pytest.mark.parametrize("slacks", [1, 2, 3])
@pytest.mark.parametrize("tile_be", [64, 256, 512])
def test_positions_with_slacks(checker, slacks, tile_be):
    """Slack columns (imbalance 1, load loss 2, both 3) lengthen the balance
    rows: every position still holds its pattern column, and the gen tiles
    cover the generators and the slack variables once."""
    for name in ("parallel60", "rgg2000"):
        d = A._Desc(GRIDS[name]())
        assert checker.tile_check(C.byref(d.desc), tile_be, slacks) == 0, name
