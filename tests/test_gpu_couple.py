"""Coupling rows between batch instances on the GPU (paper: SCOPFLOW,
TCOPFLOW and SOPFLOW coupling constraints): a contingency star (N-1
children coupled to their base case) and a multi-period chain (each period
coupled to the one before, so inner periods are both child and parent).
The rows, their Jacobian values and pattern are compared with the oracle
exactly; the assembled problem's J, H and VJP within the parity tolerance."""
import numpy as np
import pytest

import oracle as O
from oracle import coupled as OC
from paper_2203_10587_amd import synth as S
from tests.parity import assert_close, log

pytestmark = pytest.mark.gpu


def _star():
    g = S.random_grid(60, 95, 20, seed=5, parallel=3)
    outs = [3, 7, 11, 19, 40, 52]
    grids = [g] + [S.remove_branch(g, l) for l in outs]
    return g, outs, grids, [(k, 0) for k in range(1, len(grids))]


def _chain():
    g = S.rgg_grid(300, 420, seed=4)
    grids = [S.scale_loads(g, s) for s in (0.9, 0.95, 1.0, 1.05, 1.1, 1.0)]
    return grids, [(t, t - 1) for t in range(1, len(grids))]


def _setup(A, nets, grids, links, seed):
    import torch
    b = A.acopf_batch_create(nets, tile_be=256, grid_mult=0)
    cp = A.acopf_couple_create(b, [a for a, _ in links], [p for _, p in links])
    rng = np.random.default_rng(seed)
    its = [S.draw_iterate(g, rng) for g in grids]
    x = torch.as_tensor(np.concatenate([i.x for i in its]), device="cuda")
    return b, cp, its, x


def _check(A, b, cp, grids, its, x, links, name):
    import torch
    models = [O.prepare(g) for g in grids]
    xs = [i.x for i in its]
    # pattern (bit-exact) and values (exact: one subtraction each side)
    rp, col = A.acopf_couple_pattern(cp)
    Jc = OC.coupling_matrix(models, links).tocsr()
    Jc.sort_indices()
    np.testing.assert_array_equal(rp, Jc.indptr)
    np.testing.assert_array_equal(col, Jc.indices)
    c = torch.full((cp.rows,), np.nan, dtype=torch.float64, device="cuda")
    jv = torch.full((cp.nnz,), np.nan, dtype=torch.float64, device="cuda")
    A.acopf_couple_eval(cp, x, c, jv)
    np.testing.assert_array_equal(c.cpu().numpy(), OC.coupling_rows(models, xs, links))
    np.testing.assert_array_equal(jv.cpu().numpy(), Jc.data)
    # JVP: exact
    d = torch.as_tensor(np.random.default_rng(2).standard_normal(x.numel()), device="cuda")
    out = torch.empty(cp.rows, dtype=torch.float64, device="cuda")
    A.acopf_couple_jvp(cp, d, out)
    np.testing.assert_array_equal(out.cpu().numpy(), Jc @ d.cpu().numpy())
    log(f"[{name}] rows={cp.rows} links={len(links)}")
    return models


def _check_assembled(A, b, cp, models, its, x, links, name):
    """The assembled problem: global J and H values on the global pattern,
    and u = sum_k w_f,k grad f_k + J' w over the whole problem."""
    import torch
    from paper_2203_10587_amd.coupled import global_pattern
    K = b.count
    nx, nc = int(b.x_off[-1]), int(b.c_off[-1])
    nj, nh = int(b.j_off[-1]), int(b.h_off[-1])
    sig = torch.as_tensor([i.sigma for i in its], dtype=torch.float64, device="cuda")
    lam = torch.as_tensor(np.concatenate([i.lam for i in its]), device="cuda")
    T = lambda n: torch.empty(n, dtype=torch.float64, device="cuda")
    f, gf, c, jv, hv = T(K), T(nx), T(nc), T(nj), T(nh)
    A.acopf_batch_eval(b, x, sig, lam, f, gf, c, jv, hv, A.ACOPF_ALL)
    cc, cj = T(cp.rows), T(cp.nnz)
    A.acopf_couple_eval(cp, x, cc, cj)
    jrp, jcl, hrp, hcl = global_pattern(b, cp)
    ref = OC.assemble(models, [i.x for i in its], [i.sigma for i in its], [i.lam for i in its],
                      links)
    J, H = ref["J"].tocsr(), ref["H"].tocsr()
    # the expected structure: each instance's structural pattern shifted to
    # its block, then the coupling rows
    xo, _ = OC.offsets(models)
    erp, ecl, hrp_e, hcl_e, jb, hb = [np.zeros(1, np.int64)], [], [np.zeros(1, np.int64)], [], 0, 0
    for k, m in enumerate(models):
        erp.append(m.jac_rowptr[1:].astype(np.int64) + jb)
        ecl.append(m.jac_col.astype(np.int64) + xo[k])
        hrp_e.append(m.hess_rowptr[1:].astype(np.int64) + hb)
        hcl_e.append(m.hess_col.astype(np.int64) + xo[k])
        jb += int(m.jac_rowptr[-1])
        hb += int(m.hess_rowptr[-1])
    Jc = ref["J_couple"].tocsr()
    Jc.sort_indices()
    erp.append(Jc.indptr[1:].astype(np.int64) + jb)
    ecl.append(Jc.indices.astype(np.int64))
    erp, ecl = np.concatenate(erp), np.concatenate(ecl)
    hrp_e, hcl_e = np.concatenate(hrp_e), np.concatenate(hcl_e)
    np.testing.assert_array_equal(jrp, erp)
    np.testing.assert_array_equal(jcl, ecl)
    np.testing.assert_array_equal(hrp, hrp_e)
    np.testing.assert_array_equal(hcl, hcl_e)
    # values at those positions
    jrow = np.repeat(np.arange(erp.size - 1), np.diff(erp))
    jref = np.asarray(J[jrow, ecl]).ravel()
    hrow = np.repeat(np.arange(hrp_e.size - 1), np.diff(hrp_e))
    href = np.asarray(H[hrow, hcl_e]).ravel()
    # per-instance scales of the parity rule; the coupling rows are exact
    sj, sh = [], []
    for m, it in zip(models, its):
        o = O.evaluate(m, it.x, it.sigma, it.lam)
        sc = O.scales(m, it.x, o, it.sigma, it.lam)
        sj.append(sc["jac_val"])
        sh.append(sc["hess_val"])
    sj.append(np.zeros(Jc.nnz))
    jall = np.concatenate([jv.cpu().numpy(), cj.cpu().numpy()])
    assert_close(f"{name}.J", jall, jref, np.concatenate(sj))
    assert_close(f"{name}.H", hv.cpu().numpy(), href, np.concatenate(sh))
    # VJP over the whole problem: the batch's blocks, then the coupling rows
    rng = np.random.default_rng(9)
    wf = rng.standard_normal(K)
    wc = rng.standard_normal(nc)
    wr = rng.standard_normal(cp.rows)
    u = T(nx)
    A.acopf_batch_vjp(b, x, torch.as_tensor(wf, device="cuda"), torch.as_tensor(wc, device="cuda"), u)
    A.acopf_couple_vjp(cp, torch.as_tensor(wr, device="cuda"), u)
    gref = np.concatenate([O.objective(m, i.x)[1] for m, i in zip(models, its)])
    wfx = np.concatenate([np.full(m.n, wf[k]) for k, m in enumerate(models)])
    w = np.concatenate([wc, wr])
    uref = wfx * gref + J.T @ w
    scale = wfx * np.abs(gref) + abs(J).T @ np.abs(w)
    assert_close(f"{name}.u", u.cpu().numpy(), uref, scale)


def test_contingency_star(gpu_lib):
    from paper_2203_10587_amd import acopf as A
    g, outs, grids, links = _star()
    base = A.acopf_net_create(g)
    nets = [base] + [A.acopf_net_create_outage(base, l) for l in outs]
    b, cp, its, x = _setup(A, nets, grids, links, 1)
    models = _check(A, b, cp, grids, its, x, links, "star")
    _check_assembled(A, b, cp, models, its, x, links, "star")


def test_multiperiod_chain(gpu_lib):
    from paper_2203_10587_amd import acopf as A
    grids, links = _chain()
    nets = [A.acopf_net_create(g) for g in grids]
    b, cp, its, x = _setup(A, nets, grids, links, 2)
    models = _check(A, b, cp, grids, its, x, links, "chain")
    _check_assembled(A, b, cp, models, its, x, links, "chain")


def test_coupling_errors(gpu_lib):
    from paper_2203_10587_amd import acopf as A
    g1 = S.random_grid(12, 18, 4, seed=1)
    g2 = S.random_grid(12, 18, 5, seed=1)
    nets = [A.acopf_net_create(g1), A.acopf_net_create(g2), A.acopf_net_create(g1)]
    b = A.acopf_batch_create(nets, tile_be=256, grid_mult=0)
    for ch, pa, msg in (([1], [0], "generator"), ([0], [0], "itself"), ([3], [0], "range")):
        with pytest.raises(A.AcopfError) as e:
            A.acopf_couple_create(b, ch, pa)
        assert msg in str(e.value)
    cp = A.acopf_couple_create(b, [2], [0])
    with pytest.raises(A.AcopfError) as e:
        b.close()  # a coupling still uses the batch
    assert "couplings" in str(e.value)
    cp.close()
    b.close()
