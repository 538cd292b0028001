"""Benchmark: ACOPF model evaluation (f, g, grad f, J, H in FP64) on one GPU.

Default workload: the batched N-1 security set -- a 2,000-bus / 3,000-branch
grid with 1,000 single-branch outages, each with its own iterate and
multipliers, evaluated in one kernel launch per step with the autotuned
schedule (one workgroup per tile, launched directly: the tuner found that
faster than a persistent grid replayed from a HIP graph, which is timed
beside it).  One step = one full evaluation of every instance.  Reported
beside it: the plain path (the same kernels, one instance per launch),
per-step latency percentiles, the roofline of the batched kernel, the
batched products, the other formulations, the 512 uneven scenario grids with
their VJP, 60 s of served Poisson requests, and the CPU oracle timed on a
bounded sample on this host.  Before each timed region the GPU runs untimed
steps until it has done WARM_MS of work, whatever --warmup says (short
warm-ups leave the clocks below their steady state).

    python bench.py [--gpus 1] [--steps 50] [--warmup 50]
                    [--workload n1|grid10k|uneven|served] [--model polar|cartesian|slacks]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "bus-evals/sec for f,g,∇f,J,H (batched vs plain, FP64); p50/p99 latency"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


WARM_MS = 200.0  # GPU time of untimed work before each timed region


def warm_to_steady(call, stream, min_ms=None, chunk=20, max_calls=20000):
    """Untimed calls until at least min_ms (default WARM_MS) of GPU time has
    run; returns the calls made and their GPU time."""
    import torch
    min_ms = WARM_MS if min_ms is None else min_ms
    done, gpu_ms = 0, 0.0
    while gpu_ms < min_ms and done < max_calls:
        s_, e_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s_.record(stream)
        for _ in range(chunk):
            call()
        e_.record(stream)
        torch.cuda.synchronize()
        gpu_ms += s_.elapsed_time(e_)
        done += chunk
    return {"calls": done, "gpu_ms": gpu_ms}


def time_calls(call, stream, n):
    """Mean ms per call over n calls back to back between two events on the
    launch stream."""
    import torch
    s_, e_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s_.record(stream)
    for _ in range(n):
        call()
    e_.record(stream)
    torch.cuda.synchronize()
    return s_.elapsed_time(e_) / n


# ---------------------------------------------------------------------------
# workloads


def workload_n1():
    from paper_2203_10587_amd import synth as S
    os_ = S.n1_security_set(0)
    return {"name": "n1_security_2000bus_x1000", "base": os_.base, "outages": os_.outages,
            "iterates": os_.iterates, "kind": "outage"}


def workload_grid10k():
    from paper_2203_10587_amd import synth as S
    g, it = S.grid_10k(0)
    return {"name": "single_10000bus", "grids": [g], "iterates": [it], "kind": "grids"}


def workload_uneven():
    from paper_2203_10587_amd import synth as S
    inst = S.uneven_scenarios(0)
    return {"name": "uneven_scenarios_x512", "grids": [g for _, g, _ in inst],
            "iterates": [it for _, _, it in inst], "kind": "grids"}


def instance_grid(w, k):
    from paper_2203_10587_amd import synth as S
    if w["kind"] == "outage":
        return S.remove_branch(w["base"], int(w["outages"][k]))
    return w["grids"][k]


def count(w):
    return len(w["iterates"])


# model variants: the polar representation (headline), the power-balance-
# cartesian one, and the polar one with both feasibility slack blocks
MODELS = ("polar", "cartesian", "slacks")
LABELS = {"polar": "power-balance-polar", "cartesian": "power-balance-cartesian",
          "slacks": "polar + load loss + power imbalance"}
IMB_COST, LOSS_COST = (0.0, 1000.0), (0.0, 10000.0)   # (c2, c1) per MW


def model_opts(A, model):
    if model == "cartesian":
        return A.net_opts(A.ACOPF_CARTESIAN)
    if model == "slacks":
        return A.net_opts(A.ACOPF_POLAR, A.ACOPF_SLACK_IMBALANCE | A.ACOPF_SLACK_LOADLOSS,
                          IMB_COST, LOSS_COST)
    return None


def model_iterate(w, k, model):
    """(x, lambda, sigma) of instance k for a model: the workload's polar
    iterate; for cartesian a seeded draw x = [e; f; Pg; Qg]; for slacks the
    polar iterate followed by six blocks of slacks U(0, 0.05)."""
    it = w["iterates"][k]
    if model == "polar":
        return it.x, it.lam, it.sigma
    from paper_2203_10587_amd import synth as S
    rng = np.random.default_rng([2203, k])
    g = instance_grid(w, k)
    if model == "cartesian":
        c = S.draw_iterate_cartesian(g, rng, it.sigma)
        return c.x, c.lam, it.sigma
    return np.concatenate([it.x, rng.uniform(0.0, 0.05, 6 * g.nbus)]), it.lam, it.sigma


def algorithmic_bytes(w, opts=None):
    """Bytes the method must move per full evaluation of the batch: inputs
    x (8n), lambda (8m), sigma (8); outputs 8 (1 + n + m + nnzJ + nnzH); the
    network primitives (56 B per branch, 32 B per bus, 28 B per generator)
    counted once per distinct network.  `opts` (net options) selects the
    model variant, whose sizes differ: the cartesian representation has nb
    more rows and 2 nb more Jacobian entries, each slack block nb more
    variables, Jacobian and Hessian entries."""
    from paper_2203_10587_amd import acopf as A
    tot = 0
    nets = set()
    for k in range(count(w)):
        g = w["base"] if w["kind"] == "outage" else w["grids"][k]
        d, *_ = A.acopf_pattern_host_opts(g, opts, int(w["outages"][k]) if w["kind"] == "outage" else -1)
        tot += 8 * d.n + 8 * d.m + 8 + 8 * (1 + d.n + d.m + d.nnz_jac + d.nnz_hess)
        key = id(g)
        if key not in nets:
            nets.add(key)
            tot += 56 * g.nbranch + 32 * g.nbus + 28 * g.ngen
    return tot


# ---------------------------------------------------------------------------
# CPU baseline: the oracle as it stands, single thread, bounded sample


def _oracle_runner(model):
    import oracle as O
    from oracle import cartesian as OC
    from oracle import slacks as OS
    spec = OS.Spec(imbalance=True, loadloss=True, imb_cost=IMB_COST, loss_cost=LOSS_COST)
    return {"polar": lambda mdl, x, s, l: O.evaluate(mdl, x, s, l),
            "cartesian": lambda mdl, x, s, l: OC.evaluate(mdl, x, s, l),
            "slacks": lambda mdl, x, s, l: OS.evaluate(mdl, spec, x, s, l)}[model]


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _pool_worker(args):
    """One pool process: prepare its instances (untimed), wait for the
    others, then evaluate them round-robin for budget_s seconds."""
    w, model, idxs, budget_s, barrier = args
    import oracle as O
    from threadpoolctl import threadpool_limits
    run = _oracle_runner(model)
    with threadpool_limits(1):
        work = []
        for idx in idxs:
            g = instance_grid(w, idx)
            x, lam, sigma = model_iterate(w, idx, model)
            work.append((O.prepare(g), x, lam, sigma, g.nbus))
        barrier.wait()
        t0 = time.perf_counter()
        buses, k = 0, 0
        while time.perf_counter() - t0 < budget_s or k == 0:
            mdl, x, lam, sigma, nb = work[k % len(work)]
            run(mdl, x, sigma, lam)
            buses += nb
            k += 1
        return buses, k, time.perf_counter() - t0


def cpu_pool_baseline(w, model="polar", budget_s=5.0, per_worker=12):
    """The oracle on a pool of host processes (one BLAS thread each), up to
    16 workers (this host's share for one GPU): aggregate bus-evals/s over
    budget_s seconds of concurrent evaluation."""
    import multiprocessing as mp
    P = max(1, min(16, len(os.sched_getaffinity(0))))
    order = np.random.default_rng(1).permutation(count(w))
    ctx = mp.get_context("fork")
    barrier = ctx.Manager().Barrier(P)
    n = len(order)  # instances dealt cyclically: every worker gets per_worker
    jobs = [(w, model, [int(order[(p * per_worker + j) % n]) for j in range(per_worker)],
             budget_s, barrier) for p in range(P)]
    with ctx.Pool(P) as pool:
        res = pool.map(_pool_worker, jobs)
    buses = sum(r[0] for r in res)
    evals = sum(r[1] for r in res)
    wall = max(r[2] for r in res)
    return {"value": buses / wall, "unit": "bus-evals/s", "cores": P, "kind": "oracle",
            "sample": f"{P} processes x {per_worker} instances of {w['name']} "
                      f"({LABELS[model]}), {evals} evaluations in {wall:.1f} s "
                      f"(one BLAS thread each; Y_bus and pattern build untimed)"}


def cpu_baseline(w, model="polar", budget_s=15.0):
    import oracle as O
    from threadpoolctl import threadpool_limits
    run = _oracle_runner(model)
    k = 0
    t_eval = 0.0
    buses = 0
    n_inst = count(w)
    order = np.random.default_rng(0).permutation(n_inst)
    with threadpool_limits(1):
        while k < n_inst and (t_eval < budget_s or k < 2):
            idx = int(order[k])
            g = instance_grid(w, idx)
            x, lam, sigma = model_iterate(w, idx, model)
            mdl = O.prepare(g)                      # Y_bus and patterns: not timed
            t0 = time.perf_counter()
            run(mdl, x, sigma, lam)
            t_eval += time.perf_counter() - t0
            buses += g.nbus
            k += 1
    return {"value": buses / t_eval, "unit": "bus-evals/s", "cores": 1, "kind": "oracle",
            "sample": f"{k} of {n_inst} instances of {w['name']} ({LABELS[model]}), "
                      f"full f, grad f, c, J, H "
                      f"(NumPy/SciPy FP64, one thread; Y_bus and pattern build untimed), "
                      f"{t_eval:.1f} s of evaluation",
            "cpu_model": _cpu_model()}


# ---------------------------------------------------------------------------


def traffic_key(w, model):
    """Entry of profiles/traffic.json for a workload in a model."""
    return w["name"] if model == "polar" else f"{w['name']}_{model}"


def load_traffic(kernel_name, workload):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it
    was taken on the current kernel sources."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        doc = json.load(open(p))
        ent = doc.get(workload)
        from paper_2203_10587_amd.profiling import kernel_hash
        if not ent or ent.get("kernel_hash") != kernel_hash():
            return None
        return float(ent["fetch_bytes"]) + float(ent["write_bytes"])
    except Exception:
        return None


def served(seconds: float, rate: float = 2000.0, budget_gb: float = 8.0, log_progress=True,
           gc_off: bool = False):
    """The served workload: four resident grids (1k/10k/30k/70k buses),
    open-loop Poisson arrivals, grid chosen uniformly per request, iterate
    drawn on the device from the request seed; continuous batching with
    admission by HBM budget."""
    import torch
    from paper_2203_10587_amd import synth as S
    from paper_2203_10587_amd.serve import GpuExecutor, Server, poisson_trace
    grids = S.served_grids(0)
    ex = GpuExecutor(grids, [512, 128, 48, 24])
    srv = Server(ex, budget_bytes=int(budget_gb * (1 << 30)), max_window=64, timeout_s=30.0)
    # warm the kernels and the allocator outside the timed trace
    warm = Server(ex, budget_bytes=int(budget_gb * (1 << 30)), max_window=64)
    for g in range(4):
        warm.submit(g, 12345 + g)
    while not warm.idle():
        warm.step()
    torch.cuda.synchronize()
    tr = poisson_trace(rate, seconds, 4, seed=1)
    prog = (lambda i, n: log(f"[serve] {i}/{n} arrivals")) if log_progress else None
    st = srv.run_trace(tr, progress=prog, time_limit_s=seconds * 3 + 30, gc_off=gc_off)
    st["grids_buses"] = [g.nbus for g in grids]
    st["offered_rate_rps"] = rate
    st["budget_bytes"] = int(budget_gb * (1 << 30))
    st["bus_evals_per_s"] = sum(grids[r.grid].nbus for r in srv.requests if r.status == "done") / st["wall_s"]
    return st


def product_bytes(w, opts=None):
    """Bytes each batched product must move per pass over the batch, with
    the network primitives counted once per distinct network as in
    algorithmic_bytes:
      VJP  u = w_f grad f + J' w_c   reads x, w_c, w_f; writes u  (16 n + 8 m + 8)
      HVP  H d                       reads x, lambda, sigma, d; writes H d  (24 n + 8 m + 8)
      JVP  J d                       reads x, d; writes J d  (16 n + 8 m)"""
    from paper_2203_10587_amd import acopf as A
    tot = {"vjp": 0, "hvp": 0, "jvp": 0}
    nets = set()
    for k in range(count(w)):
        g = w["base"] if w["kind"] == "outage" else w["grids"][k]
        d, *_ = A.acopf_pattern_host_opts(g, opts, int(w["outages"][k]) if w["kind"] == "outage" else -1)
        tot["vjp"] += 16 * d.n + 8 * d.m + 8
        tot["hvp"] += 24 * d.n + 8 * d.m + 8
        tot["jvp"] += 16 * d.n + 8 * d.m
        if id(g) not in nets:
            nets.add(id(g))
            for key in tot:
                tot[key] += 56 * g.nbranch + 32 * g.nbus + 28 * g.ngen
    return tot


def products_bench(A, w, model, batch, x, sigma, lam, nbus_total, steps, dev, stream):
    """The batched VJP, HVP and JVP over the step's batch and iterates
    (seeded directions and weights), each timed like the step: warm-up
    launches, then `steps` launches back to back between two events."""
    import torch
    K = batch.count
    nx, nc = int(batch.x_off[-1]), int(batch.c_off[-1])
    gen = torch.Generator(device=dev)
    gen.manual_seed(20220321)
    d = torch.randn(nx, dtype=torch.float64, device=dev, generator=gen)
    wc = torch.randn(nc, dtype=torch.float64, device=dev, generator=gen)
    wf = torch.ones(K, dtype=torch.float64, device=dev)
    u = torch.empty(nx, dtype=torch.float64, device=dev)
    hd = torch.empty(nx, dtype=torch.float64, device=dev)
    jd = torch.empty(nc, dtype=torch.float64, device=dev)
    calls = {"vjp": lambda: A.acopf_batch_vjp(batch, x, wf, wc, u, stream),
             "hvp": lambda: A.acopf_batch_hvp(batch, x, sigma, lam, d, hd, stream),
             "jvp": lambda: A.acopf_batch_jvp(batch, x, d, jd, stream)}
    nbytes = product_bytes(w, model_opts(A, model))
    out = {}
    for name, call in calls.items():
        warm_to_steady(call, stream)
        ms = time_calls(call, stream, steps)
        gbs = nbytes[name] / (ms / 1e3) / 1e9
        out[name] = {"ms_per_step": ms, "value": nbus_total / (ms / 1e3), "unit": "bus-evals/s",
                     "algorithmic_bytes": nbytes[name], "achieved_GBps": gbs,
                     "frac": gbs / HBM_PEAK_GBS}
        log(f"[bench] {name}: {ms:.4f} ms/step, {gbs:.0f} GB/s ({gbs / HBM_PEAK_GBS:.3f} of peak)")
    return out


LAT_SAMPLES = 200
PERSISTENT_SCHED = {"grid_mult": 4, "no_graph": 0}


def persistent_graph_bench(A, w, nets, sched, x, sigma, lam, nbus_total, steps, dev, stream):
    """The step with a persistent grid (4 workgroups per CU) replayed from
    one HIP graph, the tile class and XCD grouping of the tuned schedule."""
    import torch
    K = count(w)
    ps = dict(sched, **PERSISTENT_SCHED)
    pb = A.acopf_batch_create(nets, **ps)
    outs = [torch.empty(n, dtype=torch.float64, device=dev)
            for n in (K, int(pb.x_off[-1]), int(pb.c_off[-1]), int(pb.j_off[-1]),
                      int(pb.h_off[-1]))]

    def pstep():
        A.acopf_batch_eval(pb, x, sigma, lam, *outs, A.ACOPF_ALL, stream)

    warm_to_steady(pstep, stream)
    ms = time_calls(pstep, stream, steps)
    alg = algorithmic_bytes(w)
    res = {"schedule": ps, "ms_per_step": ms, "value": nbus_total / (ms / 1e3),
           "unit": "bus-evals/s", "frac": alg / (ms / 1e3) / 1e9 / HBM_PEAK_GBS}
    log(f"[bench] persistent graph-replayed schedule: {ms:.4f} ms/step, frac {res['frac']:.3f}")
    del outs
    pb.close()
    return res


def uneven_bench(A, steps, dev, stream):
    """The 512 uneven scenario grids (200..25,000 buses, loads scaled per
    scenario) in their tuned schedule: one full evaluation per step, then
    the batched VJP with seeded cotangents, each timed like the headline
    step, with algorithmic bytes, roofline fraction and counter traffic."""
    import torch
    from paper_2203_10587_amd import tune
    t0 = time.time()
    w = workload_uneven()
    K = count(w)
    _, nets = make_nets(A, w, "polar")
    sched = tune.lookup_or_default(nets)
    b = A.acopf_batch_create(nets, **sched)
    x, lam = packed_inputs(w, b, "polar")
    x, lam = x.to(dev), lam.to(dev)
    sigma = torch.tensor([it.sigma for it in w["iterates"]], dtype=torch.float64, device=dev)
    outs = [torch.empty(n, dtype=torch.float64, device=dev)
            for n in (K, int(b.x_off[-1]), int(b.c_off[-1]), int(b.j_off[-1]), int(b.h_off[-1]))]
    nbus = sum(int(n.dims.nbus) for n in nets)
    log(f"[bench] uneven: {K} grids, {nbus} buses, prepared in {time.time() - t0:.1f}s")

    def ustep():
        A.acopf_batch_eval(b, x, sigma, lam, *outs, A.ACOPF_ALL, stream)

    warm_to_steady(ustep, stream)
    ms = time_calls(ustep, stream, steps)
    alg = algorithmic_bytes(w)
    res = {"workload": w["name"], "instances": K, "buses_per_step": nbus, "schedule": sched,
           "ms_per_step": ms, "value": nbus / (ms / 1e3), "unit": "bus-evals/s",
           "algorithmic_bytes": alg, "achieved_GBps": alg / (ms / 1e3) / 1e9,
           "frac": alg / (ms / 1e3) / 1e9 / HBM_PEAK_GBS,
           "traffic": load_traffic("k_eval_all", traffic_key(w, "polar"))}
    log(f"[bench] uneven: {ms:.4f} ms/step, {res['value']:.4e} bus-evals/s, frac {res['frac']:.3f}")
    gen = torch.Generator(device=dev)
    gen.manual_seed(20220322)
    wc = torch.randn(int(b.c_off[-1]), dtype=torch.float64, device=dev, generator=gen)
    wf = torch.randn(K, dtype=torch.float64, device=dev, generator=gen)
    u = torch.empty(int(b.x_off[-1]), dtype=torch.float64, device=dev)

    def vjp():
        A.acopf_batch_vjp(b, x, wf, wc, u, stream)

    warm_to_steady(vjp, stream)
    vms = time_calls(vjp, stream, steps)
    vbytes = product_bytes(w)["vjp"]
    res["vjp"] = {"ms_per_step": vms, "algorithmic_bytes": vbytes,
                  "achieved_GBps": vbytes / (vms / 1e3) / 1e9,
                  "frac": vbytes / (vms / 1e3) / 1e9 / HBM_PEAK_GBS}
    log(f"[bench] uneven vjp: {vms:.4f} ms/step, frac {res['vjp']['frac']:.3f}")
    del outs, x, lam, u, wc
    b.close()
    for n in nets:
        n.close()
    return res


def make_nets(A, w, model):
    """(base or None, one net per instance) of the workload for a model."""
    opts = model_opts(A, model)
    if w["kind"] == "outage":
        base = A.acopf_net_create_opts(w["base"], opts)
        return base, [A.acopf_net_create_outage(base, int(l)) for l in w["outages"]]
    return None, [A.acopf_net_create_opts(g, opts) for g in w["grids"]]


def packed_inputs(w, batch, model):
    """Host x and lambda of every instance packed at the batch's offsets."""
    import torch
    x = torch.empty(int(batch.x_off[-1]), dtype=torch.float64)
    lam = torch.empty(int(batch.c_off[-1]), dtype=torch.float64)
    for k in range(count(w)):
        xk, lk, _ = model_iterate(w, k, model)
        x[batch.x_off[k]:batch.x_off[k + 1]] = torch.from_numpy(np.ascontiguousarray(xk))
        lam[batch.c_off[k]:batch.c_off[k + 1]] = torch.from_numpy(np.ascontiguousarray(lk))
    return x, lam


def variant_bench(A, w, model, sched, sigma, nbus_total, args, dev, stream):
    """The workload in another model, timed like the headline step (same
    schedule, steps and warmup; all outputs)."""
    import torch
    K = count(w)
    vbase, vnets = make_nets(A, w, model)
    vb = A.acopf_batch_create(vnets, **sched)
    vx, vl = packed_inputs(w, vb, model)
    vx, vl = vx.to(dev), vl.to(dev)
    outs = [torch.empty(n, dtype=torch.float64, device=dev)
            for n in (K, int(vb.x_off[-1]), int(vb.c_off[-1]), int(vb.j_off[-1]),
                      int(vb.h_off[-1]))]

    def vstep():
        A.acopf_batch_eval(vb, vx, sigma, vl, *outs, A.ACOPF_ALL, stream)

    for _ in range(args.warmup):
        vstep()
    warm_to_steady(vstep, stream)
    ms = time_calls(vstep, stream, args.steps)
    alg = algorithmic_bytes(w, model_opts(A, model))
    label = LABELS[model]
    res = {"formulation": label, "ms_per_step": ms, "value": nbus_total / (ms / 1e3),
           "unit": "bus-evals/s", "algorithmic_bytes": alg,
           "achieved_GBps": alg / (ms / 1e3) / 1e9, "frac": alg / (ms / 1e3) / 1e9 / HBM_PEAK_GBS,
           "traffic": load_traffic("k_eval_all", traffic_key(w, model))}
    log(f"[bench] {label}: {ms:.4f} ms/step, {res['value']:.4e} bus-evals/s, frac {res['frac']:.3f}")
    del outs, vx, vl
    vb.close()
    for n in vnets:
        n.close()
    if vbase is not None:
        vbase.close()
    return res


def main():
    global WARM_MS
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=50,
                    help="untimed steps first (the GPU needs ~10 ms of work to reach steady clocks)")
    ap.add_argument("--workload", default="n1", choices=["n1", "grid10k", "uneven", "served"],
                    help="n1: 1,000 N-1 outages of a 2,000-bus grid (default); grid10k: one "
                         "10,000-bus grid; uneven: 512 scenario grids of 200..25,000 buses; "
                         "served: Poisson requests over four resident grids")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="length of the served Poisson trace (the served workload is 60 s)")
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--serve-gc-on", dest="serve_gc_off", action="store_false",
                    help="keep Python's garbage collector running during the served trace (by "
                         "default it is off there: its generation-2 pauses, up to ~70 ms with "
                         "120,000 live requests, stall the serving loop)")
    ap.add_argument("--plain-steps", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--model", default="polar", choices=list(MODELS),
                    help="formulation of the timed step: polar (default), cartesian, or polar "
                         "with load-loss and power-imbalance slacks")
    ap.add_argument("--no-variants", dest="variants", action="store_false",
                    help="skip timing the workload in the other formulations, the "
                         "batched products (VJP, HVP, JVP), the persistent graph-replayed "
                         "schedule and the uneven scenario grids")
    ap.add_argument("--warm-ms", type=float, default=WARM_MS,
                    help="GPU time of untimed work before each timed region (0 for profiled "
                         "runs, where every dispatch is recorded)")
    ap.add_argument("--no-uneven", dest="uneven", action="store_false",
                    help="skip the uneven scenario grids (512 grids of 200..25,000 buses "
                         "with their VJP) in the default line")
    ap.add_argument("--tile-be", type=int, default=0)
    ap.add_argument("--grid-mult", type=int, default=-1)
    ap.add_argument("--xcd", type=int, default=-1)
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--autotune", action="store_true",
                    help="time every schedule on this workload's batch, cache the fastest "
                         "(paper_2203_10587_amd/tune.py; $ACOPF_TUNE_CACHE overrides the file) and exit")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a device-to-device copy of MIB MiB five times (the "
                         "reference kernel for scaling HBM traffic counters)")
    args = ap.parse_args()
    WARM_MS = args.warm_ms
    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 8
        src = torch.rand(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        for _ in range(5):
            dst.copy_(src)
        e.record()
        torch.cuda.synchronize()
        ms = s.elapsed_time(e) / 5
        print(json.dumps({"copy_bytes_each_way": n * 8, "ms": ms,
                          "GBps_read_plus_write": 2 * n * 8 / ms / 1e6}), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this library has no multi-GPU path "
              "(instances would shard across GPUs with no exchange); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "served":
        import torch
        torch.cuda.set_device(0)
        st = served(args.serve_seconds, args.serve_rate, gc_off=args.serve_gc_off)
        out = {"metric": METRIC, "value": st["bus_evals_per_s"], "unit": "bus-evals/s", "n_gpus": 1,
               "steps": st["done"], "warmup": 4, "ms_per_step": 1e3 / max(st["throughput_rps"], 1e-9),
               "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
               "data": "synthetic",
               "config": {"workload": "served_poisson_4grids", "rate_rps": args.serve_rate,
                          "seconds": args.serve_seconds, "grids_buses": st["grids_buses"]},
               "latency_ms": {"p50": st["p50_ms"], "p99": st["p99_ms"]}, "serving": st,
               "roofline": None, "cpu_baseline": None}
        print(json.dumps(out), flush=True)
        return

    t0 = time.time()
    w = {"grid10k": workload_grid10k, "n1": workload_n1, "uneven": workload_uneven}[args.workload]()
    log(f"[bench] workload {w['name']}: {count(w)} instances, generated in {time.time() - t0:.1f}s")
    cpu = None if (args.no_cpu or args.autotune) else cpu_baseline(w, args.model)
    if cpu:
        log(f"[bench] cpu oracle: {cpu['value']:.3e} bus-evals/s ({cpu['sample']})")
        cpu["pool"] = cpu_pool_baseline(w, args.model)
        log(f"[bench] cpu oracle pool: {cpu['pool']['value']:.3e} bus-evals/s "
            f"({cpu['pool']['sample']})")

    import torch
    from paper_2203_10587_amd import acopf as A
    from paper_2203_10587_amd import tune

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    K = count(w)
    base, nets = make_nets(A, w, args.model)
    if args.autotune:
        ts = torch.tensor([it.sigma for it in w["iterates"]], dtype=torch.float64)
        bx = A.acopf_batch_create(nets, **tune.DEFAULT)
        nx_, nc_ = int(bx.x_off[-1]), int(bx.c_off[-1])
        xt, lt = packed_inputs(w, bx, args.model)
        outs = [torch.empty(n, dtype=torch.float64, device=dev)
                for n in (K, nx_, nc_, int(bx.j_off[-1]), int(bx.h_off[-1]))]
        bx.close()
        best = tune.autotune(nets, xt.to(dev), ts.to(dev), lt.to(dev), outs, reps=20, progress=log)
        print(json.dumps({"autotune": best, "bucket": tune.bucket(nets),
                          "cache": tune.cache_path()}), flush=True)
        return
    sched = tune.lookup_or_default(nets)
    if args.tile_be:
        sched["tile_be"] = args.tile_be
    if args.grid_mult >= 0:
        sched["grid_mult"] = args.grid_mult
    if args.xcd >= 0:
        sched["xcd_group"] = args.xcd
    if args.no_graph:
        sched["no_graph"] = 1
    batch = A.acopf_batch_create(nets, **sched)
    nx, nc = int(batch.x_off[-1]), int(batch.c_off[-1])
    nj, nh = int(batch.j_off[-1]), int(batch.h_off[-1])
    x, lam = packed_inputs(w, batch, args.model)
    x, lam = x.to(dev), lam.to(dev)
    sigma = torch.tensor([it.sigma for it in w["iterates"]], dtype=torch.float64, device=dev)
    f = torch.empty(K, dtype=torch.float64, device=dev)
    gf = torch.empty(nx, dtype=torch.float64, device=dev)
    c = torch.empty(nc, dtype=torch.float64, device=dev)
    jv = torch.empty(nj, dtype=torch.float64, device=dev)
    hv = torch.empty(nh, dtype=torch.float64, device=dev)
    nbus_total = sum(int(n.dims.nbus) for n in nets)
    stream = torch.cuda.current_stream()

    def step():
        A.acopf_batch_eval(batch, x, sigma, lam, f, gf, c, jv, hv, A.ACOPF_ALL, stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # then untimed steps until the GPU has run WARM_MS of work, so that the
    # timed region starts at steady clocks however small --warmup is
    warm_extra = warm_to_steady(step, stream)
    log(f"[bench] extra warm-up: {warm_extra['calls']} steps, {warm_extra['gpu_ms']:.0f} ms of GPU time")
    # the timed region: K steps back to back between two events on the
    # launch stream (throughput and the roofline's per-launch time)
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    start.record(stream)
    for k in range(args.steps):
        step()
    end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = start.elapsed_time(end)
    # per-step latency (p50/p99) from at least LAT_SAMPLES more steps, each
    # between its own events (which serialise the stream, so they stay out of
    # the timed region)
    n_lat = max(args.steps, LAT_SAMPLES)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(n_lat)]
    for k in range(n_lat):
        ev[k][0].record(stream)
        step()
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    lat = np.array([a.elapsed_time(b) for a, b in ev])
    value = nbus_total * args.steps / (total_ms / 1e3)
    log(f"[bench] batched: {total_ms / args.steps:.4f} ms/step, {value:.4e} bus-evals/s "
        f"(wall {wall:.3f}s)")

    # coupling rows over the same batch: a contingency star joining every
    # other instance to instance 0 (Pg of each generator), values and the
    # Jacobian's +-1 entries, timed like the batched step
    coupled = None
    if K > 1 and len({int(n.dims.ngen) for n in nets}) == 1:  # links need equal generator sets
        cp = A.acopf_couple_create(batch, list(range(1, K)), [0] * (K - 1))
        cc = torch.empty(cp.rows, dtype=torch.float64, device=dev)
        cj = torch.empty(cp.nnz, dtype=torch.float64, device=dev)
        for _ in range(3):
            A.acopf_couple_eval(cp, x, cc, cj, stream)
        cs_, ce_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        cs_.record(stream)
        for _ in range(args.steps):
            A.acopf_couple_eval(cp, x, cc, cj, stream)
        ce_.record(stream)
        torch.cuda.synchronize()
        cms = cs_.elapsed_time(ce_) / args.steps
        cbytes = 40 * cp.rows  # reads 2 x 8 B of x, writes 8 B of c and 2 x 8 B of J per row
        coupled = {"links": K - 1, "rows": cp.rows, "ms": cms,
                   "rows_per_s": cp.rows / (cms / 1e3),
                   "achieved_GBps": cbytes / (cms / 1e3) / 1e9,
                   "frac": cbytes / (cms / 1e3) / 1e9 / HBM_PEAK_GBS,
                   "algorithmic_bytes": cbytes}
        log(f"[bench] coupled: {cp.rows} rows in {cms * 1e3:.1f} us")
        cp.close()

    # the same workload in the other model variants: the power-balance-cartesian
    # representation, and the polar one with both slack blocks (load loss and
    # power imbalance); each has its own nets, batch and seeded iterates
    # the batched products over the same batch and iterates
    products = None
    if args.variants:
        products = products_bench(A, w, args.model, batch, x, sigma, lam, nbus_total, args.steps,
                                  dev, stream)

    # the same step with a persistent grid replayed from a HIP graph: the
    # tuner's best such schedule, beside the tuned (direct) one
    persistent = None
    if args.variants and not sched.get("grid_mult", 0):
        persistent = persistent_graph_bench(A, w, nets, sched, x, sigma, lam, nbus_total,
                                            args.steps, dev, stream)

    variants = {}
    if args.variants:
        for mname in MODELS:
            if mname != args.model:
                variants[mname] = variant_bench(A, w, mname, sched, sigma, nbus_total, args, dev,
                                                stream)

    # plain path: the same kernels, one instance per launch, into the same buffers
    L = A.lib()
    import ctypes as C
    xp, lp = x.data_ptr(), lam.data_ptr()
    ptrs = []
    for k, n in enumerate(nets):
        xo, co, jo, ho = (int(batch.x_off[k]), int(batch.c_off[k]), int(batch.j_off[k]),
                          int(batch.h_off[k]))
        ptrs.append((n.handle, C.c_void_p(xp + 8 * xo), C.c_double(w["iterates"][k].sigma),
                     C.c_void_p(lp + 8 * co), C.c_void_p(f.data_ptr() + 8 * k),
                     C.c_void_p(gf.data_ptr() + 8 * xo), C.c_void_p(c.data_ptr() + 8 * co),
                     C.c_void_p(jv.data_ptr() + 8 * jo), C.c_void_p(hv.data_ptr() + 8 * ho)))
    sp = C.c_void_p(stream.cuda_stream)

    def plain_step():
        for p in ptrs:
            rc = L.acopf_eval_all(*p, A.ACOPF_ALL, sp)
            if rc:
                raise RuntimeError(L.acopf_last_error().decode())

    plain = None
    if args.plain_steps > 0:
        plain_step()
        torch.cuda.synchronize()
        ps, pe = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ps.record(stream)
        for _ in range(args.plain_steps):
            plain_step()
        pe.record(stream)
        torch.cuda.synchronize()
        plain_ms = ps.elapsed_time(pe) / args.plain_steps
        plain_value = nbus_total / (plain_ms / 1e3)
        plain = {"value": plain_value, "unit": "bus-evals/s", "ms_per_step": plain_ms,
                 "launches_per_step": K}
        log(f"[bench] plain: {plain_ms:.3f} ms/step, {plain_value:.4e} bus-evals/s")

    serving = None
    if args.serve_seconds > 0:
        log(f"[bench] served workload: {args.serve_seconds:.0f} s of Poisson arrivals at "
            f"{args.serve_rate:.0f}/s")
        serving = served(args.serve_seconds, args.serve_rate, gc_off=args.serve_gc_off)
        log(f"[bench] served: {serving['done']} requests, p50 {serving['p50_ms']:.3f} ms, "
            f"p99 {serving['p99_ms']:.3f} ms")

    uneven = None
    if args.variants and args.uneven and args.workload == "n1" and args.model == "polar":
        uneven = uneven_bench(A, args.steps, dev, stream)

    alg = algorithmic_bytes(w, model_opts(A, args.model))
    avg_ms = total_ms / args.steps  # per launch of the step, over the timed region
    achieved = alg / (avg_ms / 1e3) / 1e9
    traffic = load_traffic("k_eval_all", traffic_key(w, args.model))
    out = {
        "metric": METRIC, "value": value, "unit": "bus-evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": total_ms / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w["name"], "formulation": LABELS[args.model], "instances": K,
                   "buses_per_step": nbus_total,
                   "outputs": "f, grad_f, c, J, H", "schedule": sched},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "samples": int(len(lat))},
        "warmup_extra": warm_extra,
        "plain": plain,
        "persistent_graph": persistent,
        "uneven": uneven,
        "coupled": coupled,
        "products": products,
        "variants": variants or None,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_GBps": None if traffic is None else traffic / (avg_ms / 1e3) / 1e9,
                     "algorithmic_bytes": alg, "kernel_ms": avg_ms},
        "cpu_baseline": cpu,
        "serving": serving,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
