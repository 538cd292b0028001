"""Every instance of the full-size workloads against the oracle.

  * 1,000 N-1 outages of the 2,000-bus grid (paper: SCOPFLOW section, the
    single-period security-constrained problem), evaluated in one launch of
    the schedule the benchmark times: f, grad f, c, J, H and the VJP of every
    instance, CSR patterns bit for bit, and (polar) the batched HVP and JVP
    of every instance along its own seeded direction; the same workload in
    the cartesian formulation and with both slack blocks;
  * the 512 uneven scenario grids of 200..25,000 buses (paper: SOPFLOW
    section, one period): every instance's outputs and VJP, and directional
    central differences through AcopfBatchEval over the whole batch;
  * one served request on each of the four resident grids of 1,000, 10,000,
    30,000 and 70,000 buses, against the oracle and against the same request
    served alone.
The oracle runs in a pool of host processes (tests/fullsize_pool.py)."""
import numpy as np
import pytest

from paper_2203_10587_amd import synth as S
from tests import fullsize_pool as FP
from tests.parity import compare_outputs, log

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]


def _torch():
    import torch
    return torch


def _evaluate(A, nets, points, w=None, products=False):
    """Pack points [(x, lam, sigma)], evaluate every output of every instance
    in one launch of the tuned schedule (and the batched VJP with weights
    w = (w_f, [w_c]) if given; with products, the batched HVP and JVP along
    each instance's seeded direction); host copies and the batch."""
    from paper_2203_10587_amd import tune
    torch = _torch()
    sched = tune.lookup_or_default(nets)
    b = A.acopf_batch_create(nets, **sched)
    K = b.count
    x, lam = np.empty(int(b.x_off[-1])), np.empty(int(b.c_off[-1]))
    for k, (xk, lk, _) in enumerate(points):
        x[b.x_off[k]:b.x_off[k + 1]] = xk
        lam[b.c_off[k]:b.c_off[k + 1]] = lk
    d = lambda a: torch.as_tensor(np.asarray(a, dtype=np.float64), device="cuda")
    nan = lambda n: torch.full((int(n),), np.nan, dtype=torch.float64, device="cuda")
    xt, lt, st = d(x), d(lam), d([p[2] for p in points])
    f, gf, c = nan(K), nan(b.x_off[-1]), nan(b.c_off[-1])
    jv, hv = nan(b.j_off[-1]), nan(b.h_off[-1])
    log(f"[full size] {K} instances, schedule {sched}")
    A.acopf_batch_eval(b, xt, st, lt, f, gf, c, jv, hv, A.ACOPF_ALL)
    host = {"f": f, "grad_f": gf, "c": c, "jac_val": jv, "hess_val": hv}
    if w is not None:
        wc = np.empty(int(b.c_off[-1]))
        for k in range(K):
            wc[b.c_off[k]:b.c_off[k + 1]] = w[1][k]
        u = nan(b.x_off[-1])
        A.acopf_batch_vjp(b, xt, d(w[0]), d(wc), u)
        host["u"] = u
    if products:
        dv = np.concatenate([FP.direction(k, int(b.x_off[k + 1] - b.x_off[k])) for k in range(K)])
        hd, jd = nan(b.x_off[-1]), nan(b.c_off[-1])
        A.acopf_batch_hvp(b, xt, st, lt, d(dv), hd)
        A.acopf_batch_jvp(b, xt, d(dv), jd)
        host["hd"], host["jd"] = hd, jd
    torch.cuda.synchronize()
    host = {k: v.cpu().numpy() for k, v in host.items()}
    for k, v in host.items():
        assert np.all(np.isfinite(v)), f"non-finite {k}"
    return host, b


def _items(b, host, nets, A, w=None, with_patterns=True):
    offs = {"grad_f": b.x_off, "c": b.c_off, "jac_val": b.j_off, "hess_val": b.h_off,
            "u": b.x_off, "hd": b.x_off, "jd": b.c_off}
    for k in range(b.count):
        got = {"f": float(host["f"][k])}
        for key, o in offs.items():
            if key in host:
                got[key] = host[key][int(o[k]):int(o[k + 1])]
        pat = A.acopf_pattern(nets[k]) if with_patterns else None
        yield k, got, pat, (None if w is None else (float(w[0][k]), w[1][k])), "hd" in host


def _report(tag, res, bad, count):
    for r in bad[:5]:
        log(f"[{tag}] {r[2]}")
    assert not bad, f"{tag}: {len(bad)} of {count} instances differ from the oracle"
    assert len(res) == count
    worst = {}
    for _, _, ratios in res:
        for key, v in ratios.items():
            worst[key] = max(worst.get(key, 0.0), v)
    log(f"[{tag}] all {count} instances within tolerance; worst error/bound " +
        ", ".join(f"{k} {v:.3g}" for k, v in sorted(worst.items())))


def _n1_nets(A, opts):
    os_ = S.n1_security_set(0)
    base = A.acopf_net_create_opts(os_.base, opts)
    return os_, base, [A.acopf_net_create_outage(base, int(l)) for l in os_.outages]


def test_n1_every_instance_polar(gpu_lib):
    from paper_2203_10587_amd import acopf as A
    os_, base, nets = _n1_nets(A, None)
    rng = np.random.default_rng(21)
    w = (rng.standard_normal(len(nets)), [rng.standard_normal(it.lam.shape) for it in os_.iterates])
    pts = [(it.x, it.lam, it.sigma) for it in os_.iterates]
    host, b = _evaluate(A, nets, pts, w, products=True)
    res, bad = FP.check_all("n1", "polar", _items(b, host, nets, A, w))
    _report("n1 polar", res, bad, len(nets))


@pytest.mark.parametrize("model", ["cartesian", "slacks"])
def test_n1_every_instance_other_models(gpu_lib, model):
    from paper_2203_10587_amd import acopf as A
    opts = (A.net_opts(A.ACOPF_CARTESIAN) if model == "cartesian" else
            A.net_opts(A.ACOPF_POLAR, A.ACOPF_SLACK_IMBALANCE | A.ACOPF_SLACK_LOADLOSS,
                       FP.SLACK_COSTS["imb_cost"], FP.SLACK_COSTS["loss_cost"]))
    os_, base, nets = _n1_nets(A, opts)
    pts = [FP.draw(model, k, *S.n1_instance(os_, k)) for k in range(len(nets))]
    host, b = _evaluate(A, nets, pts)
    res, bad = FP.check_all("n1", model, _items(b, host, nets, A))
    _report(f"n1 {model}", res, bad, len(nets))


def test_uneven_every_instance_and_directional_fd(gpu_lib):
    torch = _torch()
    from paper_2203_10587_amd import acopf as A
    from paper_2203_10587_amd.autograd import AcopfBatchEval
    inst = S.uneven_scenarios(0)
    nets = [A.acopf_net_create(g) for _, g, _ in inst]
    rng = np.random.default_rng(23)
    w = (rng.standard_normal(len(nets)), [rng.standard_normal(g.m) for _, g, _ in inst])
    pts = [(it.x, it.lam, it.sigma) for _, _, it in inst]
    host, b = _evaluate(A, nets, pts, w)
    res, bad = FP.check_all("uneven", "polar", _items(b, host, nets, A, w))
    _report("uneven", res, bad, len(nets))
    # directional central differences through the autograd function, every
    # instance of the batch at once
    K = b.count
    x = torch.as_tensor(np.concatenate([p[0] for p in pts]), device="cuda").requires_grad_(True)
    wc = torch.as_tensor(np.concatenate(w[1]), device="cuda")
    wf = torch.as_tensor(w[0], device="cuda")
    f, c = AcopfBatchEval.apply(x, b)
    ((f * wf).sum() + (c * wc).sum()).backward()
    u = x.grad.detach()
    v = torch.as_tensor(rng.standard_normal(x.numel()), device="cuda")
    h = 1e-6
    with torch.no_grad():
        fp, cp = AcopfBatchEval.apply(x + h * v, b)
        fm, cm = AcopfBatchEval.apply(x - h * v, b)
    ix = torch.repeat_interleave(torch.arange(K, device="cuda"),
                                 torch.as_tensor(np.diff(b.x_off), device="cuda"))
    ic = torch.repeat_interleave(torch.arange(K, device="cuda"),
                                 torch.as_tensor(np.diff(b.c_off), device="cuda"))
    seg = lambda t, idx: torch.zeros(K, dtype=torch.float64, device="cuda").index_add_(0, idx, t)
    fd = (seg(wc * (cp - cm), ic) + wf * (fp - fm)) / (2 * h)
    an = seg(u * v, ix)
    scale = seg((u * v).abs(), ix)
    err = ((fd - an).abs() / scale).cpu().numpy()
    log(f"[uneven fd] {K} instances, worst |fd - u'v| / sum|u v| = {err.max():.3g}")
    assert np.all(err <= 1e-6), int(np.argmax(err))


def test_served_grids_against_oracle(gpu_lib):
    """One seeded request per served grid (1k, 10k, 30k, 70k buses) through
    the GPU executor, all four in flight together: each result against the
    oracle at the host twin of its device-drawn iterate, and bit for bit
    against the same request served alone."""
    import oracle as O
    from oracle import rng as ORNG
    from paper_2203_10587_amd.serve import GpuExecutor, Server
    grids = S.served_grids(0)
    ex = GpuExecutor(grids, [2, 2, 2, 2])
    srv = Server(ex, budget_bytes=8 << 30, max_window=2)
    seeds = [7001, 7002, 7003, 7004]
    reqs = [srv.submit(g, s) for g, s in enumerate(seeds)]
    while not srv.idle():
        srv.step()
    assert all(r.status == "done" for r in reqs), [r.error for r in reqs]
    for r, g in zip(reqs, grids):
        got = ex.fetch(r.grid, r.slot)
        ex1 = GpuExecutor([g], [1])
        s1 = Server(ex1, budget_bytes=8 << 30)
        s1.submit(0, r.seed)
        while not s1.idle():
            s1.step()
        alone = ex1.fetch(0, 0)
        for key in got:
            np.testing.assert_array_equal(np.asarray(got[key]), np.asarray(alone[key]), err_msg=key)
        bounds = (float(g.gen_pmin[0]), float(g.gen_pmax[0]), float(g.gen_qmin[0]),
                  float(g.gen_qmax[0]))
        x, lam = ORNG.request_iterate(r.seed, g.nbus, g.ngen, g.m, bounds)
        np.testing.assert_array_equal(got["x"], x)
        np.testing.assert_allclose(got["lam"], lam, rtol=1e-14, atol=1e-14)
        log(f"[served grid] {g.nbus} buses: oracle")
        lam = got["lam"]  # the multipliers the kernel used (the host twin's to rounding)
        mdl = O.prepare(g)
        out = O.evaluate(mdl, x, 1.0, lam)
        ref = {"out": out, "scale": O.scales(mdl, x, out, 1.0, lam)}
        r_ = compare_outputs(f"served-{g.nbus}", {k: got[k] for k in
                                                   ("f", "grad_f", "c", "jac_val", "hess_val")}, ref)
        log(f"[served grid] {g.nbus} buses within tolerance: {r_}")
        del ex1, s1
