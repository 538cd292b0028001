"""Helpers shared by the GPU parity tests: run the HIP path through the C-ABI
binding and compare with the oracle under the row-scaled relative rule
|gpu - oracle| <= tol * max(|oracle|, scale)."""
import sys

import numpy as np

import oracle as O

TOL = 1e-12


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def assert_close(name, gpu, orc, scale, tol=TOL):
    gpu = np.asarray(gpu, dtype=np.float64)
    orc = np.asarray(orc, dtype=np.float64)
    assert gpu.shape == orc.shape, (name, gpu.shape, orc.shape)
    bound = tol * np.maximum(np.abs(orc), np.asarray(scale, dtype=np.float64))
    err = np.abs(gpu - orc)
    bad = ~(err <= bound)
    if np.any(bad):
        k = int(np.flatnonzero(bad)[0])
        raise AssertionError(
            f"{name}: {int(bad.sum())} of {bad.size} entries out of tolerance; first at {k}: "
            f"gpu={gpu.flat[k]!r} oracle={orc.flat[k]!r} scale={np.asarray(scale).flat[k] if np.ndim(scale) else scale!r}")
    ratio = float(np.max(err / np.where(bound > 0, bound, 1.0))) if err.size else 0.0
    return ratio


def oracle_all(grid, it, w_f=None, w_c=None):
    mdl = O.prepare(grid)
    out = O.evaluate(mdl, it.x, it.sigma, it.lam)
    sc = O.scales(mdl, it.x, out, it.sigma, it.lam)
    res = {"mdl": mdl, "out": out, "scale": sc}
    if w_c is not None:
        res["u"] = O.vjp(mdl, it.x, w_f, w_c)
        res["u_scale"] = O.vjp_scale(mdl, it.x, w_f, w_c)
    return res


def compare_outputs(tag, gpu, ref, tol=TOL):
    out, sc = ref["out"], ref["scale"]
    r = {}
    if "f" in gpu:
        r["f"] = assert_close(tag + ".f", [gpu["f"]], [out["f"]], [sc["f"]], tol)
    for k in ("grad_f", "c", "jac_val", "hess_val"):
        if k in gpu:
            r[k] = assert_close(f"{tag}.{k}", gpu[k], out[k], sc[k], tol)
    if "u" in gpu:
        r["u"] = assert_close(tag + ".u", gpu["u"], ref["u"], ref["u_scale"], tol)
    for k in ("hd", "jd"):  # H d and J d along a direction
        if k in gpu:
            r[k] = assert_close(f"{tag}.{k}", gpu[k], ref[k], ref[k + "_scale"], tol)
    return r
