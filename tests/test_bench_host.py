"""Host logic of the benchmark (no GPU): the one-GPU refusal, the
algorithmic byte models against sizes counted from the oracle's own
patterns, and the gating of the recorded HBM traffic by the kernel hash."""
import json
import os
import subprocess
import sys

import pytest

import oracle as O
from paper_2203_10587_amd import synth as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""


def _tiny():
    g = S.random_grid(9, 12, 3, seed=1, parallel=1)
    it = S.draw_iterate(g, __import__("numpy").random.default_rng(0))
    return g, {"name": "tiny", "grids": [g, g], "iterates": [it, it], "kind": "grids"}


def test_algorithmic_bytes_counts_from_the_oracle_pattern():
    """Two instances of one network: inputs and outputs twice, the network
    primitives once."""
    g, w = _tiny()
    mdl = O.prepare(g)
    n, m = mdl.n, mdl.m
    nnz_j, nnz_h = len(mdl.jac_col), len(mdl.hess_col)
    per = 8 * n + 8 * m + 8 + 8 * (1 + n + m + nnz_j + nnz_h)
    net = 56 * g.nbranch + 32 * g.nbus + 28 * g.ngen
    assert bench.algorithmic_bytes(w) == 2 * per + net
    pb = bench.product_bytes(w)
    assert pb == {"vjp": 2 * (16 * n + 8 * m + 8) + net, "hvp": 2 * (24 * n + 8 * m + 8) + net,
                  "jvp": 2 * (16 * n + 8 * m) + net}


def test_recorded_traffic_follows_the_kernel_hash(monkeypatch):
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
        doc = json.load(fh)
    ent = doc["n1_security_2000bus_x1000"]
    from paper_2203_10587_amd import profiling as P
    if ent["kernel_hash"] != P.kernel_hash():
        pytest.skip("the recorded counters predate the current kernel sources")
    got = bench.load_traffic("k_eval_all", "n1_security_2000bus_x1000")
    assert got == pytest.approx(ent["fetch_bytes"] + ent["write_bytes"], rel=0, abs=0)
    assert bench.load_traffic("k_eval_all", "no_such_workload") is None
    monkeypatch.setattr(P, "kernel_hash", lambda: "0" * 16)
    assert bench.load_traffic("k_eval_all", "n1_security_2000bus_x1000") is None


def test_traffic_keys():
    w = {"name": "n1_security_2000bus_x1000"}
    assert bench.traffic_key(w, "polar") == "n1_security_2000bus_x1000"
    assert bench.traffic_key(w, "slacks") == "n1_security_2000bus_x1000_slacks"
