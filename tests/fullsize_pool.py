"""Host-side checking of full-size batches against the oracle, instance by
instance, in a pool of spawned processes (numpy, scipy and the oracle only:
the workers never touch the GPU).  The parent evaluates the batch on the GPU,
copies the outputs to the host and sends each instance's slices here; every
worker regenerates its instances from the same seeded generators and
compares under the row-scaled rule of tests/parity.py, CSR patterns with ==.

Workloads: "n1" (1,000 outages of the 2,000-bus grid) and "uneven" (512
scenario grids of 200..25,000 buses), in the models "polar", "cartesian"
and "slacks" (polar with both slack blocks).
"""
import multiprocessing as mp
import os

import numpy as np

SLACK_COSTS = dict(imb_cost=(0.4, 30.0), loss_cost=(1.5, 90.0))

_W = {}


def workers() -> int:
    """The host's share for one GPU: at most 16 processes."""
    return max(1, min(16, len(os.sched_getaffinity(0))))


def draw(model, k, g, it):
    """(x, lambda, sigma) of instance k in a model: the workload's polar
    iterate; cartesian: a draw seeded by [2203, k]; slacks: the polar
    iterate followed by six slack blocks U(0, 0.05) seeded by [2203, k]."""
    from paper_2203_10587_amd import synth as S
    if model == "polar":
        return it.x, it.lam, it.sigma
    rng = np.random.default_rng([2203, k])
    if model == "cartesian":
        c = S.draw_iterate_cartesian(g, rng, it.sigma)
        return c.x, c.lam, c.sigma
    return np.concatenate([it.x, rng.uniform(0.0, 0.05, 6 * g.nbus)]), it.lam, it.sigma


def direction(k, n):
    """The direction of the HVP and JVP of instance k (length n)."""
    return np.random.default_rng([2204, k]).standard_normal(n)


def _init(kind, model):
    from threadpoolctl import threadpool_limits
    from paper_2203_10587_amd import synth as S
    threadpool_limits(1)
    _W["kind"], _W["model"] = kind, model
    if kind == "n1":
        _W["os"] = S.n1_security_set(0)


def instance(kind, k, os_=None):
    from paper_2203_10587_amd import synth as S
    if kind == "n1":
        return S.n1_instance(os_, k)
    _, g, it = S.uneven_scenarios(0, only=[k])[0]
    return g, it


def reference(model, g, x, lam, sigma, w=None, d=None):
    """Oracle outputs, scales and patterns of one instance in a model; with
    a direction d (polar), also H d and J d from the oracle's matrices, with
    the scales of the product tests (J: the row scale times |d| summed over
    the row's columns; H: the row's largest |entry| times the sum of |d| over
    its columns)."""
    import oracle as O
    from oracle import cartesian as OC
    from oracle import slacks as OS
    mdl = O.prepare(g)
    if model == "polar":
        out = O.evaluate(mdl, x, sigma, lam)
        sc = O.scales(mdl, x, out, sigma, lam)
        pat = (mdl.jac_rowptr, mdl.jac_col, mdl.hess_rowptr, mdl.hess_col)
        vjp = (lambda wf, wc: (O.vjp(mdl, x, wf, wc), O.vjp_scale(mdl, x, wf, wc)))
    elif model == "cartesian":
        out = OC.evaluate(mdl, x, sigma, lam)
        sc = OC.scales(mdl, x, out, sigma, lam)
        pat = OC.pattern(mdl)
        vjp = (lambda wf, wc: (OC.vjp(mdl, x, wf, wc), OC.vjp_scale(mdl, x, wf, wc)))
    else:
        spec = OS.Spec(imbalance=True, loadloss=True, **SLACK_COSTS)
        out = OS.evaluate(mdl, spec, x, sigma, lam)
        sc = OS.scales(mdl, spec, x, out, sigma, lam)
        pat = OS.pattern(mdl, spec)
        vjp = (lambda wf, wc: (OS.vjp(mdl, spec, x, wf, wc), OS.vjp_scale(mdl, spec, x, wf, wc)))
    ref = {"out": out, "scale": sc}
    if w is not None:
        ref["u"], ref["u_scale"] = vjp(*w)
    if d is not None:
        assert model == "polar"
        J = O.jacobian_matrix(mdl, x)
        H = O.hessian_matrix(mdl, x, sigma, lam)
        sj = O.jacobian_row_scales(mdl, x, out["jac_val"])
        rows = np.repeat(np.arange(mdl.m), np.diff(mdl.jac_rowptr))
        ref["jd"] = J @ d
        ref["jd_scale"] = np.bincount(rows, weights=sj * np.abs(d[mdl.jac_col]), minlength=mdl.m)
        Habs = abs(H).tocsr()
        ref["hd"] = H @ d
        ref["hd_scale"] = Habs.max(axis=1).toarray().ravel() * ((Habs > 0).astype(float) @ np.abs(d))
    return ref, pat


def check(item):
    """item = (k, gpu outputs dict, library CSR patterns or None, (w_f, w_c)
    or None, whether the outputs hold H d and J d along direction(k, n)).
    Returns (k, nbus, worst error/bound per output) or (k, nbus, message) on
    a mismatch."""
    from tests.parity import compare_outputs
    k, got, pat, w, prod = item
    kind, model = _W["kind"], _W["model"]
    g, it = instance(kind, k, _W.get("os"))
    x, lam, sigma = draw(model, k, g, it)
    try:
        ref, opat = reference(model, g, x, lam, sigma, w, direction(k, len(x)) if prod else None)
        if pat is not None:
            for name, a, b in zip(("jac_rowptr", "jac_col", "hess_rowptr", "hess_col"), pat, opat):
                if not np.array_equal(np.asarray(a), np.asarray(b)):
                    raise AssertionError(f"{name} differs from the oracle's pattern")
        return k, g.nbus, compare_outputs(f"{kind}-{model}-{k}", got, ref)
    except AssertionError as e:
        return k, g.nbus, f"instance {k}: {e}"


def check_all(kind, model, items, nproc=None):
    """Check every item in a spawned pool; returns (results, failures)."""
    ctx = mp.get_context("spawn")
    res, bad = [], []
    with ctx.Pool(nproc or workers(), initializer=_init, initargs=(kind, model)) as pool:
        for r in pool.imap_unordered(check, items, chunksize=2):
            (bad if isinstance(r[2], str) else res).append(r)
    return res, bad
