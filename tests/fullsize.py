"""The 1,000-outage workload (2,000-bus / 3,000-branch grid) at full size in
the launch configuration the benchmark times (the tuned schedule for that
batch), for any formulation: build, evaluate all outputs in one launch, and
hand back sampled instances with their grids and inputs."""
import numpy as np

from paper_2203_10587_amd import synth as S
from tests.parity import log


def run(A, opts, draw, samples=(0, 1, 499, 998, 999)):
    """draw(k, grid_k, polar_iterate_k) -> (x, lam, sigma) of instance k.
    Returns (outputs per sampled k, grids, inputs, nets, batch)."""
    import torch
    from paper_2203_10587_amd import tune
    os_ = S.n1_security_set(0)
    base = A.acopf_net_create_opts(os_.base, opts)
    nets = [A.acopf_net_create_outage(base, int(l)) for l in os_.outages]
    sched = tune.lookup_or_default(nets)
    log(f"[full size] schedule {sched}")
    b = A.acopf_batch_create(nets, **sched)
    K = b.count
    x = np.empty(int(b.x_off[-1]))
    lam = np.empty(int(b.c_off[-1]))
    sig = np.empty(K)
    keep = {}
    for k in range(K):
        g2, it = S.n1_instance(os_, k)
        xk, lk, sk = draw(k, g2, it)
        x[b.x_off[k]:b.x_off[k + 1]] = xk
        lam[b.c_off[k]:b.c_off[k + 1]] = lk
        sig[k] = sk
        if k in samples:
            keep[k] = (g2, xk, lk, sk)
    d = lambda a: torch.as_tensor(a, dtype=torch.float64, device="cuda")
    nan = lambda n: torch.full((int(n),), np.nan, dtype=torch.float64, device="cuda")
    f, gf, c = nan(K), nan(b.x_off[-1]), nan(b.c_off[-1])
    jv, hv = nan(b.j_off[-1]), nan(b.h_off[-1])
    A.acopf_batch_eval(b, d(x), d(sig), d(lam), f, gf, c, jv, hv, A.ACOPF_ALL)
    torch.cuda.synchronize()
    host = [t.cpu().numpy() for t in (f, gf, c, jv, hv)]
    assert all(np.all(np.isfinite(h)) for h in host), "a full-size output is not finite"
    out = {}
    for k in samples:
        s = lambda h, o: h[int(o[k]):int(o[k + 1])]
        out[k] = {"f": float(host[0][k]), "grad_f": s(host[1], b.x_off), "c": s(host[2], b.c_off),
                  "jac_val": s(host[3], b.j_off), "hess_val": s(host[4], b.h_off)}
    return out, keep, nets, b, base
