"""The adjoint kernel behind torch.autograd: gradcheck against central
finite differences of the forward kernels, batched directional finite
differences on uneven grids, and the VJP against the oracle's J' w."""
import numpy as np
import pytest

import oracle as O
from paper_2203_10587_amd import synth as S
from tests.parity import assert_close, log

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("seed,nb,nl,ng", [(1, 9, 12, 3), (2, 20, 30, 6), (3, 40, 55, 12)])
def test_gradcheck_single(gpu_lib, seed, nb, nl, ng):
    import torch
    from paper_2203_10587_amd import acopf as A
    from paper_2203_10587_amd.autograd import AcopfEval
    g = S.random_grid(nb, nl, ng, seed=seed, parallel=1)
    it = S.draw_iterate(g, np.random.default_rng(seed))
    net = A.acopf_net_create(g)
    x = torch.as_tensor(it.x, device="cuda").requires_grad_(True)
    log(f"[gradcheck] nb={nb}")
    assert torch.autograd.gradcheck(lambda z: AcopfEval.apply(z, net), (x,), eps=1e-6,
                                    atol=1e-6, rtol=1e-5)


def test_backward_matches_oracle(gpu_lib):
    import torch
    from paper_2203_10587_amd import acopf as A
    from paper_2203_10587_amd.autograd import AcopfEval
    g = S.rgg_grid(500, 650, seed=3)
    it = S.draw_iterate(g, np.random.default_rng(4))
    net = A.acopf_net_create(g)
    rng = np.random.default_rng(5)
    wc = rng.standard_normal(g.m)
    wf = 0.37
    x = torch.as_tensor(it.x, device="cuda").requires_grad_(True)
    f, c = AcopfEval.apply(x, net)
    (wf * f.sum() + (c * torch.as_tensor(wc, device="cuda")).sum()).backward()
    mdl = O.prepare(g)
    assert_close("autograd.u", x.grad.cpu().numpy(), O.vjp(mdl, it.x, wf, wc),
                 O.vjp_scale(mdl, it.x, wf, wc))


def test_batched_directional_fd(gpu_lib):
    """Uneven scenario grids (log-uniform sizes), random cotangents through
    AcopfBatchEval: per instance, w'(c(x+hv) - c(x-hv))/2h + w_f (f(x+hv) -
    f(x-hv))/2h against u'v."""
    import torch
    from paper_2203_10587_amd import acopf as A
    from paper_2203_10587_amd.autograd import AcopfBatchEval
    inst = S.uneven_scenarios(0, count=12, lo=200, hi=25_000)
    nets = [A.acopf_net_create(g) for _, g, _ in inst]
    b = A.acopf_batch_create(nets)
    K = len(nets)
    x = torch.cat([torch.as_tensor(it.x) for _, _, it in inst]).cuda().requires_grad_(True)
    rng = np.random.default_rng(0)
    wc = torch.as_tensor(rng.standard_normal(int(b.c_off[-1])), device="cuda")
    wf = torch.as_tensor(rng.standard_normal(K), device="cuda")
    f, c = AcopfBatchEval.apply(x, b)
    ((f * wf).sum() + (c * wc).sum()).backward()
    u = x.grad.detach()
    v = torch.as_tensor(rng.standard_normal(x.numel()), device="cuda")
    # keep angles and voltages physical: scale the direction
    h = 1e-6
    with torch.no_grad():
        fp, cp = AcopfBatchEval.apply(x + h * v, b)
        fm, cm = AcopfBatchEval.apply(x - h * v, b)
    for k in range(K):
        xs = slice(int(b.x_off[k]), int(b.x_off[k + 1]))
        cs = slice(int(b.c_off[k]), int(b.c_off[k + 1]))
        fd = float((wc[cs] * (cp[cs] - cm[cs])).sum() + wf[k] * (fp[k] - fm[k])) / (2 * h)
        an = float((u[xs] * v[xs]).sum())
        scale = float((u[xs].abs() * v[xs].abs()).sum())
        log(f"[batched fd] inst {k} nb={nets[k].dims.nbus} fd={fd:.6e} an={an:.6e}")
        assert abs(fd - an) <= 1e-6 * scale


def test_hvp_and_jvp_match_oracle(gpu_lib):
    """H d (full symmetric H) and J d against the oracle's matrices, on a
    grid with shunts, parallel branches and phase shifters, and on an N-1
    child."""
    import torch
    from paper_2203_10587_amd import acopf as A
    from tests.parity import assert_close
    g = S.random_grid(60, 95, 20, seed=5, parallel=3)
    base = A.acopf_net_create(g)
    for net, grid in ((base, g), (A.acopf_net_create_outage(base, 7), S.remove_branch(g, 7))):
        it = S.draw_iterate(grid, np.random.default_rng(3), sigma=0.7)
        d = np.random.default_rng(4).standard_normal(grid.n)
        T = lambda a: torch.as_tensor(np.asarray(a, dtype=np.float64), device="cuda")
        hv = torch.empty(net.n, dtype=torch.float64, device="cuda")
        jv = torch.empty(net.m, dtype=torch.float64, device="cuda")
        A.acopf_hvp(net, T(it.x), it.sigma, T(it.lam), T(d), hv)
        A.acopf_jvp(net, T(it.x), T(d), jv)
        mdl = O.prepare(grid)
        H = O.hessian_matrix(mdl, it.x, it.sigma, it.lam)
        J = O.jacobian_matrix(mdl, it.x)
        out = O.evaluate(mdl, it.x, it.sigma, it.lam)
        sj = O.jacobian_row_scales(mdl, it.x, out["jac_val"])
        rows = np.repeat(np.arange(mdl.m), np.diff(mdl.jac_rowptr))
        jscale = np.bincount(rows, weights=sj * np.abs(d[mdl.jac_col]), minlength=mdl.m)
        assert_close("jvp", jv.cpu().numpy(), J @ d, jscale)
        # each H entry sums per-branch terms that may cancel: bound the
        # rounding by the row's largest entry times the sum of |d| it touches
        Habs = abs(H).tocsr()
        rowmax = Habs.max(axis=1).toarray().ravel()
        hscale = rowmax * ((Habs > 0).astype(float) @ np.abs(d))
        assert_close("hvp", hv.cpu().numpy(), H @ d, hscale)


def test_double_backward(gpu_lib):
    """gradgradcheck: the VJP's own derivatives (HVP, JVP) against finite
    differences of the VJP."""
    import torch
    from paper_2203_10587_amd import acopf as A
    from paper_2203_10587_amd.autograd import AcopfEval
    g = S.random_grid(12, 18, 4, seed=2, parallel=1)
    it = S.draw_iterate(g, np.random.default_rng(1))
    net = A.acopf_net_create(g)
    x = torch.as_tensor(it.x, device="cuda").requires_grad_(True)
    assert torch.autograd.gradgradcheck(lambda z: AcopfEval.apply(z, net), (x,), eps=1e-6,
                                        atol=1e-5, rtol=1e-4)


@pytest.mark.parametrize("form,slacks", [(1, 0), (0, 3), (1, 3)])
def test_gradcheck_formulations(gpu_lib, form, slacks):
    """gradcheck and gradgradcheck through the adjoint, HVP and JVP kernels in
    the cartesian formulation and with slack blocks."""
    import torch
    from paper_2203_10587_amd import acopf as A
    from paper_2203_10587_amd.autograd import AcopfEval
    g = S.random_grid(12, 18, 4, seed=5, parallel=1)
    rng = np.random.default_rng(6)
    it = S.draw_iterate_cartesian(g, rng) if form else S.draw_iterate(g, rng)
    net = A.acopf_net_create_opts(g, A.net_opts(form, slacks, (0.3, 20.0), (0.8, 50.0)))
    xs = np.concatenate([it.x, rng.uniform(0.0, 0.2, net.n - len(it.x))])
    x = torch.as_tensor(xs, device="cuda").requires_grad_(True)
    log(f"[gradcheck] form={form} slacks={slacks} n={net.n} m={net.m}")
    fn = lambda z: AcopfEval.apply(z, net)
    assert torch.autograd.gradcheck(fn, (x,), eps=1e-6, atol=1e-6, rtol=1e-5)
    assert torch.autograd.gradgradcheck(fn, (x,), eps=1e-6, atol=1e-5, rtol=1e-4)
