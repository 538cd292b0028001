"""Batched evaluation on the GPU: parity with the oracle, bitwise identity
with the one-instance-per-launch path and across every schedule, HIP-graph
replays, and the two batched workloads at full size (1,000 N-1 outages of a
2,000-bus grid; 512 uneven scenario grids of 200..25,000 buses)."""
import numpy as np
import pytest

import oracle as O
from paper_2203_10587_amd import synth as S
from tests.parity import assert_close, compare_outputs, log, oracle_all

pytestmark = pytest.mark.gpu


def _t():
    import torch
    return torch


class Packed:
    """Packed device buffers of a batch, filled from per-instance iterates."""

    def __init__(self, A, batch, iterates, w_f=None, w_c=None):
        torch = _t()
        self.A, self.b = A, batch
        K = batch.count
        nx, nc = int(batch.x_off[-1]), int(batch.c_off[-1])
        x = np.empty(nx)
        lam = np.empty(nc)
        for k, it in enumerate(iterates):
            x[batch.x_off[k]:batch.x_off[k + 1]] = it.x
            lam[batch.c_off[k]:batch.c_off[k + 1]] = it.lam
        d = lambda a: torch.as_tensor(a, dtype=torch.float64, device="cuda")
        self.x, self.lam = d(x), d(lam)
        self.sigma = d([it.sigma for it in iterates])
        nan = lambda n: torch.full((n,), np.nan, dtype=torch.float64, device="cuda")
        self.f, self.gf, self.c = nan(K), nan(nx), nan(nc)
        self.jv, self.hv = nan(int(batch.j_off[-1])), nan(int(batch.h_off[-1]))
        self.u = nan(nx)
        if w_c is not None:
            wc = np.empty(nc)
            for k in range(K):
                wc[batch.c_off[k]:batch.c_off[k + 1]] = w_c[k]
            self.wc, self.wf = d(wc), d(w_f)

    def eval(self, what=None, stream=None):
        A = self.A
        A.acopf_batch_eval(self.b, self.x, self.sigma, self.lam, self.f, self.gf, self.c,
                           self.jv, self.hv, A.ACOPF_ALL if what is None else what, stream)

    def vjp(self):
        self.A.acopf_batch_vjp(self.b, self.x, self.wf, self.wc, self.u)

    def instance(self, k):
        b = self.b
        h = lambda t, o: t[int(o[k]):int(o[k + 1])].cpu().numpy()
        out = {"f": float(self.f[k].cpu()), "grad_f": h(self.gf, b.x_off), "c": h(self.c, b.c_off),
               "jac_val": h(self.jv, b.j_off), "hess_val": h(self.hv, b.h_off)}
        if hasattr(self, "wc"):
            out["u"] = h(self.u, b.x_off)
        return out


def plain(A, net, it, w_f=None, w_c=None):
    torch = _t()
    d = lambda a: torch.as_tensor(np.asarray(a, dtype=np.float64), device="cuda")
    z = lambda n: torch.full((n,), np.nan, dtype=torch.float64, device="cuda")
    f, gf, c, jv, hv = z(1), z(net.n), z(net.m), z(net.nnz_jac), z(net.nnz_hess)
    A.acopf_eval_all(net, d(it.x), it.sigma, d(it.lam), f, gf, c, jv, hv)
    out = {"f": float(f.cpu()[0]), "grad_f": gf.cpu().numpy(), "c": c.cpu().numpy(),
           "jac_val": jv.cpu().numpy(), "hess_val": hv.cpu().numpy()}
    if w_c is not None:
        u = z(net.n)
        A.acopf_vjp(net, d(it.x), w_f, d(w_c), u)
        out["u"] = u.cpu().numpy()
    return out


def same(a, b, tag):
    for k in a:
        np.testing.assert_array_equal(np.asarray(a[k]), np.asarray(b[k]), err_msg=f"{tag}:{k}")


@pytest.fixture(scope="module")
def small_n1():
    os_ = S.n1_security_set(0, nb=300, nl=450, count=40)
    rng = np.random.default_rng(5)
    w_c = [rng.standard_normal(it.lam.shape) for it in os_.iterates]
    w_f = rng.standard_normal(len(w_c))
    return os_, w_f, w_c


def _nets(A, os_):
    base = A.acopf_net_create(os_.base)
    return base, [A.acopf_net_create_outage(base, int(l)) for l in os_.outages]


def test_batch_equals_plain_and_oracle(gpu_lib, small_n1):
    from paper_2203_10587_amd import acopf as A
    os_, w_f, w_c = small_n1
    base, nets = _nets(A, os_)
    b = A.acopf_batch_create(nets)
    P = Packed(A, b, os_.iterates, w_f, w_c)
    P.eval()
    P.vjp()
    _t().cuda.synchronize()
    for k in range(len(nets)):
        log(f"[batch vs plain] instance {k} outage {int(os_.outages[k])}")
        got = P.instance(k)
        ref_plain = plain(A, nets[k], os_.iterates[k], float(w_f[k]), w_c[k])
        same(got, ref_plain, f"inst{k}")
        if k % 8 == 0:
            g2, it = S.n1_instance(os_, k)
            compare_outputs(f"n1-{k}", got, oracle_all(g2, it, float(w_f[k]), w_c[k]))


def test_schedules_bitwise_identical(gpu_lib, small_n1):
    """Every schedule (tile class, persistent grid, XCD grouping, graph or
    direct launch) gives the same bits, for the evaluation and for the
    batched VJP, HVP and JVP."""
    from paper_2203_10587_amd import acopf as A
    from paper_2203_10587_amd import tune
    torch = _t()
    os_, w_f, w_c = small_n1
    base, nets = _nets(A, os_)
    ref = None
    for cand in tune.CANDIDATES + [dict(tune.DEFAULT, no_graph=1)]:
        log(f"[schedule] {cand}")
        b = A.acopf_batch_create(nets, **cand)
        P = Packed(A, b, os_.iterates, w_f, w_c)
        P.eval()
        P.vjp()
        nx, nc = int(b.x_off[-1]), int(b.c_off[-1])
        d = torch.as_tensor(np.random.default_rng(3).standard_normal(nx), device="cuda")
        hd = torch.full((nx,), np.nan, dtype=torch.float64, device="cuda")
        jd = torch.full((nc,), np.nan, dtype=torch.float64, device="cuda")
        A.acopf_batch_hvp(b, P.x, P.sigma, P.lam, d, hd)
        A.acopf_batch_jvp(b, P.x, d, jd)
        torch.cuda.synchronize()
        outs = [P.instance(k) for k in (0, 17, 39)] + [{"hd": hd.cpu().numpy(), "jd": jd.cpu().numpy()}]
        if ref is None:
            ref = outs
        else:
            for k, (a, r) in enumerate(zip(outs, ref)):
                same(a, r, f"{cand}:{k}")
        b.close()


def test_batch_variants_match_full(gpu_lib, small_n1):
    from paper_2203_10587_amd import acopf as A
    os_, _, _ = small_n1
    base, nets = _nets(A, os_)
    b = A.acopf_batch_create(nets)
    full = Packed(A, b, os_.iterates)
    full.eval()
    _t().cuda.synchronize()
    ref = [full.instance(k) for k in range(0, 40, 13)]
    for what, keys in ((A.ACOPF_J, ["jac_val"]), (A.ACOPF_H, ["hess_val"]),
                       (A.ACOPF_F | A.ACOPF_GRADF | A.ACOPF_C, ["f", "grad_f", "c"]),
                       (A.ACOPF_C | A.ACOPF_H, ["c", "hess_val"])):
        P = Packed(A, b, os_.iterates)
        P.eval(what)
        _t().cuda.synchronize()
        for i, k in enumerate(range(0, 40, 13)):
            got = P.instance(k)
            for key in keys:
                np.testing.assert_array_equal(np.asarray(got[key]), np.asarray(ref[i][key]),
                                              err_msg=f"what={what} {key}")


def test_graph_replays_match_eager(gpu_lib, small_n1):
    """Replay the captured graph several times with eager work and
    synchronisations in between; every replay equals the eager launch."""
    from paper_2203_10587_amd import acopf as A
    torch = _t()
    os_, _, _ = small_n1
    base, nets = _nets(A, os_)
    eager_b = A.acopf_batch_create(nets, no_graph=1)
    E = Packed(A, eager_b, os_.iterates)
    E.eval()
    torch.cuda.synchronize()
    ref = [E.instance(k) for k in range(40)]
    gb = A.acopf_batch_create(nets)
    G = Packed(A, gb, os_.iterates)
    for rep in range(4):
        for t in (G.f, G.gf, G.c, G.jv, G.hv):
            t.fill_(np.nan)
        G.eval()
        junk = torch.randn(1 << 20, dtype=torch.float64, device="cuda")
        _ = (junk * 2.0).sum().item()
        E.eval()  # eager launch of the same kernel between replays
        torch.cuda.synchronize()
        for k in range(40):
            same(G.instance(k), ref[k], f"replay{rep}:{k}")
    # a second buffer set goes through its own cached graph
    G2 = Packed(A, gb, os_.iterates)
    G2.eval()
    torch.cuda.synchronize()
    same(G2.instance(5), ref[5], "second-buffers")


def test_n1_security_set_full_size(gpu_lib):
    """1,000 N-1 outages of the 2,000-bus grid in one launch: sampled
    instances against the oracle and against the plain path; the
    angle-reference property (theta-columns of every J row sum to zero) on
    all instances."""
    from paper_2203_10587_amd import acopf as A
    from paper_2203_10587_amd import tune
    os_ = S.n1_security_set(0)
    base, nets = _nets(A, os_)
    b = A.acopf_batch_create(nets, **tune.lookup_or_default(nets))  # the benchmark's launch
    P = Packed(A, b, os_.iterates)
    P.eval()
    _t().cuda.synchronize()
    for k in (0, 1, 499, 998, 999):
        log(f"[n1_security_set] oracle instance {k}")
        g2, it = S.n1_instance(os_, k)
        got = P.instance(k)
        compare_outputs(f"n1-{k}", got, oracle_all(g2, it))
        same(got, plain(A, nets[k], it), f"c2 plain {k}")
    jv = P.jv.cpu().numpy()
    assert np.all(np.isfinite(jv)) and np.all(np.isfinite(P.hv.cpu().numpy()))
    for k in range(0, 1000, 37):
        jp, jc, hp, hc = A.acopf_pattern(nets[k])
        vals = jv[int(b.j_off[k]):int(b.j_off[k + 1])]
        nb = os_.base.nbus
        rows = np.repeat(np.arange(len(jp) - 1), np.diff(jp))
        th = jc < nb
        sums = np.bincount(rows[th], weights=vals[th], minlength=len(jp) - 1)
        scale = np.maximum.reduceat(np.abs(vals), jp[:-1])
        assert np.all(np.abs(sums) <= 1e-12 * scale * 8), k


def test_n1_products_full_size(gpu_lib):
    """The batched VJP, HVP and JVP over the 1,000 N-1 outages of the
    2,000-bus grid in the benchmark's launch: sampled instances against the
    oracle's gradient and matrices (H full and symmetric), with the rounding
    scales of the single-instance product tests."""
    torch = _t()
    from paper_2203_10587_amd import acopf as A
    from paper_2203_10587_amd import tune
    os_ = S.n1_security_set(0)
    base, nets = _nets(A, os_)
    b = A.acopf_batch_create(nets, **tune.lookup_or_default(nets))
    rng = np.random.default_rng(11)
    K = len(nets)
    w_c = [rng.standard_normal(it.lam.shape) for it in os_.iterates]
    w_f = rng.standard_normal(K)
    P = Packed(A, b, os_.iterates, w_f, w_c)
    nx, nc = int(b.x_off[-1]), int(b.c_off[-1])
    dh = rng.standard_normal(nx)
    dt = torch.as_tensor(dh, device="cuda")
    hd = torch.full((nx,), np.nan, dtype=torch.float64, device="cuda")
    jd = torch.full((nc,), np.nan, dtype=torch.float64, device="cuda")
    P.vjp()
    A.acopf_batch_hvp(b, P.x, P.sigma, P.lam, dt, hd)
    A.acopf_batch_jvp(b, P.x, dt, jd)
    torch.cuda.synchronize()
    u, hd, jd = P.u.cpu().numpy(), hd.cpu().numpy(), jd.cpu().numpy()
    assert np.all(np.isfinite(u)) and np.all(np.isfinite(hd)) and np.all(np.isfinite(jd))
    for k in (0, 1, 500, 999):
        log(f"[n1_products] oracle instance {k}")
        g2, it = S.n1_instance(os_, k)
        mdl = O.prepare(g2)
        xs, cs = slice(int(b.x_off[k]), int(b.x_off[k + 1])), slice(int(b.c_off[k]), int(b.c_off[k + 1]))
        d = dh[xs]
        out = O.evaluate(mdl, it.x, it.sigma, it.lam)
        J = O.jacobian_matrix(mdl, it.x)
        H = O.hessian_matrix(mdl, it.x, it.sigma, it.lam)
        want_u = O.vjp(mdl, it.x, float(w_f[k]), w_c[k])
        assert_close(f"vjp {k}", u[xs], want_u, O.vjp_scale(mdl, it.x, float(w_f[k]), w_c[k]))
        sj = O.jacobian_row_scales(mdl, it.x, out["jac_val"])
        rows = np.repeat(np.arange(mdl.m), np.diff(mdl.jac_rowptr))
        jscale = np.bincount(rows, weights=sj * np.abs(d[mdl.jac_col]), minlength=mdl.m)
        assert_close(f"jvp {k}", jd[cs], J @ d, jscale)
        Habs = abs(H).tocsr()
        rowmax = Habs.max(axis=1).toarray().ravel()
        assert_close(f"hvp {k}", hd[xs], H @ d, rowmax * ((Habs > 0).astype(float) @ np.abs(d)))


def test_uneven_scenarios_subset(gpu_lib):
    """The uneven scenario workload: a 64-instance draw spanning the size
    range, batched with VJP; smallest, median and largest instances against
    the oracle."""
    from paper_2203_10587_amd import acopf as A
    sizes = S.uneven_scenario_sizes(0)
    order = np.argsort(sizes)
    pick = sorted(set(order[::8].tolist()) | {int(order[0]), int(order[-1])})
    inst = S.uneven_scenarios(0, only=pick)
    nets = [A.acopf_net_create(g) for _, g, _ in inst]
    rng = np.random.default_rng(9)
    w_c = [rng.standard_normal(g.m) for _, g, _ in inst]
    w_f = rng.standard_normal(len(inst))
    b = A.acopf_batch_create(nets)
    P = Packed(A, b, [it for _, _, it in inst], w_f, w_c)
    P.eval()
    P.vjp()
    _t().cuda.synchronize()
    sz = [g.nbus for _, g, _ in inst]
    chk = {int(np.argmin(sz)), int(np.argmax(sz)), int(np.argsort(sz)[len(sz) // 2])}
    for i in sorted(chk):
        k, g, it = inst[i]
        log(f"[uneven_scenarios] instance {k} nb={g.nbus}")
        compare_outputs(f"uneven-{k}", P.instance(i), oracle_all(g, it, float(w_f[i]), w_c[i]))
    # f of every instance, one-chunk and several-chunk nets mixed in the
    # batch, bit for bit against the plain path
    fb = P.f.cpu().numpy()
    for i, (k, g, it) in enumerate(inst):
        assert fb[i] == plain(A, nets[i], it)["f"], (k, g.ngen)


def test_flow_limits_of_nets_and_children(gpu_lib, small_n1):
    """h+ from a device net and its N-1 children equals the host rule."""
    from paper_2203_10587_amd import acopf as A
    os_, _, _ = small_n1
    base, nets = _nets(A, os_)
    np.testing.assert_array_equal(A.acopf_flow_limits(base), A.acopf_flow_limits_host(os_.base))
    for k in (0, 7, 39):
        l = int(os_.outages[k])
        np.testing.assert_array_equal(A.acopf_flow_limits(nets[k]),
                                      A.acopf_flow_limits_host(os_.base, l))
        assert nets[k].dims.m_eq == 2 * os_.base.nbus


def test_batch_xdot_matches_exact_sums(gpu_lib):
    """Per-instance dot products over the packed x layout, against exactly
    rounded sums (math.fsum), within 1e-12 of the sum of |products|; uneven
    instance sizes from 9 to 4,200 buses, and bitwise repeatable."""
    import math
    from paper_2203_10587_amd import acopf as A
    torch = _t()
    grids = [S.ring9(0)[0], S.rgg_grid(4200, seed=7), S.random_grid(30, 50, 11, seed=3),
             S.rgg_grid(700, seed=2)]
    nets = [A.acopf_net_create(g) for g in grids]
    b = A.acopf_batch_create(nets)
    nx = int(b.x_off[-1])
    rng = np.random.default_rng(4)
    a, v = rng.standard_normal(nx), rng.standard_normal(nx)
    ta = torch.as_tensor(a, device="cuda")
    tv = torch.as_tensor(v, device="cuda")
    out = torch.full((b.count,), np.nan, dtype=torch.float64, device="cuda")
    out2 = torch.full_like(out, np.nan)
    log("[xdot] 4 instances")
    A.acopf_batch_xdot(b, ta, tv, out)
    A.acopf_batch_xdot(b, ta, tv, out2)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    np.testing.assert_array_equal(got, out2.cpu().numpy())
    for k in range(b.count):
        seg = slice(int(b.x_off[k]), int(b.x_off[k + 1]))
        prod = a[seg] * v[seg]
        want = math.fsum(prod)
        assert abs(got[k] - want) <= 1e-12 * np.abs(prod).sum(), (k, got[k], want)


@pytest.mark.parametrize("form", ["polar", "cartesian"])
def test_product_groups_bitwise(gpu_lib, form):
    """The batched VJP, HVP and JVP group the instances of one base network
    into shared product tiles (four at a time, the remainder in a smaller
    group, a lone instance on its own).  Bases with 7, 3, 2 and 1 outage
    children, interleaved in the batch, give groups of every size; every
    instance's products equal its one-instance launch bit for bit."""
    torch = _t()
    from paper_2203_10587_amd import acopf as A
    sets = [S.n1_security_set(s, nb=300, nl=450, count=n) for s, n in ((1, 7), (2, 3), (3, 2), (4, 1))]
    kind = A.ACOPF_CARTESIAN if form == "cartesian" else A.ACOPF_POLAR
    bases = [A.acopf_net_create_form(o.base, kind) for o in sets]
    kids = [[A.acopf_net_create_outage(bn, int(l)) for l in o.outages] for bn, o in zip(bases, sets)]
    nets = []
    for j in range(max(len(k) for k in kids)):  # interleave the bases
        nets += [k[j] for k in kids if j < len(k)]
    b = A.acopf_batch_create(nets)
    rng = np.random.default_rng(21)
    nx, nc = int(b.x_off[-1]), int(b.c_off[-1])
    dev = lambda a: torch.as_tensor(np.asarray(a, dtype=np.float64), device="cuda")
    nan = lambda n: torch.full((int(n),), np.nan, dtype=torch.float64, device="cuda")
    x = rng.uniform(0.9, 1.1, nx)
    lam, wc, d = rng.standard_normal(nc), rng.standard_normal(nc), rng.standard_normal(nx)
    wf, sig = rng.standard_normal(b.count), rng.uniform(0.5, 2.0, b.count)
    u, hd, jd = nan(nx), nan(nx), nan(nc)
    log(f"[groups] {form}: {b.count} instances")
    A.acopf_batch_vjp(b, dev(x), dev(wf), dev(wc), u)
    A.acopf_batch_hvp(b, dev(x), dev(sig), dev(lam), dev(d), hd)
    A.acopf_batch_jvp(b, dev(x), dev(d), jd)
    torch.cuda.synchronize()
    u, hd, jd = u.cpu().numpy(), hd.cpu().numpy(), jd.cpu().numpy()
    for k, net in enumerate(nets):
        xs, cs = slice(int(b.x_off[k]), int(b.x_off[k + 1])), slice(int(b.c_off[k]), int(b.c_off[k + 1]))
        u1, h1, j1 = nan(net.n), nan(net.n), nan(net.m)
        A.acopf_vjp(net, dev(x[xs]), float(wf[k]), dev(wc[cs]), u1)
        A.acopf_hvp(net, dev(x[xs]), float(sig[k]), dev(lam[cs]), dev(d[xs]), h1)
        A.acopf_jvp(net, dev(x[xs]), dev(d[xs]), j1)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(u[xs], u1.cpu().numpy(), err_msg=f"vjp {k}")
        np.testing.assert_array_equal(hd[xs], h1.cpu().numpy(), err_msg=f"hvp {k}")
        np.testing.assert_array_equal(jd[cs], j1.cpu().numpy(), err_msg=f"jvp {k}")
    b.close()


def test_product_graph_replays_match_eager(gpu_lib, small_n1):
    """The batched VJP, HVP and JVP replayed from their captured graphs four
    times, with eager launches and synchronisations in between: every replay
    equals the direct launch bit for bit."""
    from paper_2203_10587_amd import acopf as A
    torch = _t()
    os_, w_f, w_c = small_n1
    base, nets = _nets(A, os_)

    def run(b, P, d, out):
        u, hd, jd = out
        A.acopf_batch_vjp(b, P.x, P.wf, P.wc, u)
        A.acopf_batch_hvp(b, P.x, P.sigma, P.lam, d, hd)
        A.acopf_batch_jvp(b, P.x, d, jd)

    eb = A.acopf_batch_create(nets, no_graph=1)
    E = Packed(A, eb, os_.iterates, w_f, w_c)
    nx, nc = int(eb.x_off[-1]), int(eb.c_off[-1])
    d = torch.as_tensor(np.random.default_rng(9).standard_normal(nx), device="cuda")
    nan = lambda n: torch.full((n,), np.nan, dtype=torch.float64, device="cuda")
    eout = (nan(nx), nan(nx), nan(nc))
    run(eb, E, d, eout)
    torch.cuda.synchronize()
    ref = [t.cpu().numpy() for t in eout]
    gb = A.acopf_batch_create(nets)  # graph replay
    G = Packed(A, gb, os_.iterates, w_f, w_c)
    gout = (nan(nx), nan(nx), nan(nc))
    for rep in range(4):
        for t in gout:
            t.fill_(np.nan)
        run(gb, G, d, gout)
        junk = torch.randn(1 << 20, dtype=torch.float64, device="cuda")
        _ = (junk * 2.0).sum().item()
        run(eb, E, d, eout)  # direct launches between the replays
        torch.cuda.synchronize()
        for name, got, want in zip(("vjp", "hvp", "jvp"), gout, ref):
            np.testing.assert_array_equal(got.cpu().numpy(), want, err_msg=f"replay{rep}:{name}")


def test_autotune_picks_one_of_its_candidates(gpu_lib, small_n1, tmp_path, monkeypatch):
    """The autotuner (device warm-up, then every candidate timed) returns one
    of its candidates and, with save=False, leaves the cache alone."""
    from paper_2203_10587_amd import acopf as A
    from paper_2203_10587_amd import tune
    monkeypatch.setenv("ACOPF_TUNE_CACHE", str(tmp_path / "cache.json"))
    monkeypatch.setattr(tune, "WARM_MS", 20.0)
    os_, _, _ = small_n1
    base, nets = _nets(A, os_)
    b = A.acopf_batch_create(nets, no_graph=1)
    P = Packed(A, b, os_.iterates)
    cands = [dict(tune.DEFAULT, no_graph=1), dict(tune.DEFAULT, tile_be=128, no_graph=1)]
    best = tune.autotune(nets, P.x, P.sigma, P.lam, [P.f, P.gf, P.c, P.jv, P.hv], reps=2,
                         candidates=cands, save=False)
    assert best in cands
    assert not (tmp_path / "cache.json").exists()
    b.close()
