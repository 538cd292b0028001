"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Tolerance: the row-scaled relative rule with tol = 1e-12; CSR index arrays
bit-exact.  Sizes run from the 9-bus ring to the 10,000-bus grid, with
irregular grids (shunts, parallel branches, phase shifters, several
generators per bus, a star bus, no generators, isolated buses) and N-1
outages including outages of parallel branches."""
import numpy as np
import pytest

import oracle as O
from paper_2203_10587_amd import synth as S
from tests.parity import TOL, compare_outputs, log, oracle_all

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def dev(a):
    torch = _torch()
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def gpu_eval(A, net, it, w_f=None, w_c=None, separate=True):
    """All outputs of one instance; by the separate entry points or eval_all."""
    torch = _torch()
    x, lam = dev(it.x), dev(it.lam)
    f = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
    gf = torch.full((net.n,), np.nan, dtype=torch.float64, device="cuda")
    c = torch.full((net.m,), np.nan, dtype=torch.float64, device="cuda")
    jv = torch.full((net.nnz_jac,), np.nan, dtype=torch.float64, device="cuda")
    hv = torch.full((net.nnz_hess,), np.nan, dtype=torch.float64, device="cuda")
    if separate:
        A.acopf_eval_f_g(net, x, f, gf, c)
        A.acopf_eval_jac(net, x, jv)
        A.acopf_eval_hess(net, x, it.sigma, lam, hv)
    else:
        A.acopf_eval_all(net, x, it.sigma, lam, f, gf, c, jv, hv)
    out = {"f": float(host(f)[0]), "grad_f": host(gf), "c": host(c), "jac_val": host(jv),
           "hess_val": host(hv)}
    if w_c is not None:
        u = torch.full((net.n,), np.nan, dtype=torch.float64, device="cuda")
        A.acopf_vjp(net, x, w_f, dev(w_c), u)
        out["u"] = host(u)
    torch.cuda.synchronize()
    return out


def small_cases():
    yield "ring9", S.ring9(0)[0]
    yield "rand12_par", S.random_grid(12, 20, 5, seed=1, parallel=2)
    yield "rand60", S.random_grid(60, 95, 20, seed=5, parallel=3)
    yield "star120", S.random_grid(121, 125, 10, seed=8, star=True, parallel=1)
    yield "nogen", S.random_grid(15, 18, 0, seed=2)
    yield "onebus", S.Grid(**{**S.random_grid(2, 1, 1, seed=3).__dict__, "nbus": 1,
                              "br_from": np.zeros(0, np.int32), "br_to": np.zeros(0, np.int32),
                              "br_r": np.zeros(0), "br_x": np.zeros(0), "br_b": np.zeros(0),
                              "br_tap": np.zeros(0), "br_shift": np.zeros(0),
                              "br_rate": np.zeros(0), "bus_pd": np.array([0.5]),
                              "bus_qd": np.array([0.1]), "bus_gs": np.array([0.02]),
                              "bus_bs": np.array([0.05]), "gen_bus": np.zeros(1, np.int32)})
    yield "isolated", S.Grid(**{**S.random_grid(6, 5, 2, seed=4).__dict__, "nbus": 8,
                                "bus_pd": np.ones(8) * .2, "bus_qd": np.ones(8) * .1,
                                "bus_gs": np.ones(8) * .01, "bus_bs": np.ones(8) * .02})
    yield "rgg700", S.rgg_grid(700, 910, seed=11)         # several tiles + ragged tail
    yield "rand600_shift", S.random_grid(600, 900, 300, seed=9, parallel=5)


@pytest.mark.parametrize("name,g", list(small_cases()), ids=lambda v: v if isinstance(v, str) else "")
def test_plain_parity(gpu_lib, name, g):
    from paper_2203_10587_amd import acopf as A
    log(f"[plain parity] {name} nb={g.nbus} nl={g.nbranch} ng={g.ngen}")
    rng = np.random.default_rng(17)
    it = S.draw_iterate(g, rng, sigma=0.73)
    w_c = rng.standard_normal(g.m)
    ref = oracle_all(g, it, 1.3, w_c)
    net = A.acopf_net_create(g)
    jp, jc, hp, hc = A.acopf_pattern(net)
    mdl = ref["mdl"]
    np.testing.assert_array_equal(jp, mdl.jac_rowptr)
    np.testing.assert_array_equal(jc, mdl.jac_col)
    np.testing.assert_array_equal(hp, mdl.hess_rowptr)
    np.testing.assert_array_equal(hc, mdl.hess_col)
    out = gpu_eval(A, net, it, 1.3, w_c)
    r = compare_outputs(name, out, ref)
    log(f"   worst error / tolerance: {max(r.values()):.3e}")
    fused = gpu_eval(A, net, it, separate=False)
    for k in ("grad_f", "c", "jac_val", "hess_val"):
        np.testing.assert_array_equal(fused[k], out[k], err_msg=k)
    assert fused["f"] == out["f"]


def test_grid_10k_parity(gpu_lib):
    from paper_2203_10587_amd import acopf as A
    g, it = S.grid_10k(0)
    log(f"[grid_10k] nb={g.nbus} nl={g.nbranch}")
    rng = np.random.default_rng(3)
    w_c = rng.standard_normal(g.m)
    ref = oracle_all(g, it, 0.9, w_c)
    net = A.acopf_net_create(g)
    out = gpu_eval(A, net, it, 0.9, w_c)
    r = compare_outputs("grid_10k", out, ref)
    log(f"   worst error / tolerance: {max(r.values()):.3e}")


def test_repeat_bitwise(gpu_lib):
    from paper_2203_10587_amd import acopf as A
    g = S.rgg_grid(3000, 3900, seed=4)
    it = S.draw_iterate(g, np.random.default_rng(1))
    net = A.acopf_net_create(g)
    a = gpu_eval(A, net, it)
    for _ in range(3):
        b = gpu_eval(A, net, it)
        for k in a:
            np.testing.assert_array_equal(np.asarray(a[k]), np.asarray(b[k]), err_msg=k)


def test_outage_parity(gpu_lib):
    """N-1 children against the oracle on the grid with the branch removed,
    including outages of parallel branches (slot kept) and branch 0 / last."""
    from paper_2203_10587_amd import acopf as A
    for name, g in (("rand60", S.random_grid(60, 95, 20, seed=5, parallel=3)),
                    ("rgg700", S.rgg_grid(700, 910, seed=11))):
        base = A.acopf_net_create(g)
        pairs = {}
        for l in range(g.nbranch):
            pairs.setdefault(frozenset((int(g.br_from[l]), int(g.br_to[l]))), []).append(l)
        par = [l for ls in pairs.values() if len(ls) > 1 for l in ls]
        picks = sorted(set([0, g.nbranch - 1, g.nbranch // 2] + par[:4]))
        for l in picks:
            log(f"[outage parity] {name} branch {l}")
            g2 = S.remove_branch(g, l)
            rng = np.random.default_rng(l)
            it = S.draw_iterate(g2, rng, sigma=1.1)
            w_c = rng.standard_normal(g2.m)
            ref = oracle_all(g2, it, 0.4, w_c)
            child = A.acopf_net_create_outage(base, l)
            jp, jc, hp, hc = A.acopf_pattern(child)
            np.testing.assert_array_equal(jc, ref["mdl"].jac_col)
            np.testing.assert_array_equal(hc, ref["mdl"].hess_col)
            np.testing.assert_array_equal(jp, ref["mdl"].jac_rowptr)
            np.testing.assert_array_equal(hp, ref["mdl"].hess_rowptr)
            out = gpu_eval(A, child, it, 0.4, w_c)
            compare_outputs(f"{name}-{l}", out, ref)
            child.close()


def test_tile_capacity_error(gpu_lib):
    """A bus with more branch ends than a bus tile holds is refused cleanly."""
    from paper_2203_10587_amd import acopf as A
    g = S.random_grid(600, 600, 3, seed=1, star=True, parallel=1)  # a 600-end star bus
    with pytest.raises(A.AcopfError) as ei:
        A.acopf_net_create(g)
    assert ei.value.code == A.ACOPF_EINVAL and "branch ends" in str(ei.value)
