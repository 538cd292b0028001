"""Pins for the CPU oracle: closed forms, invariants, finite differences, an
independent autograd model, a power-flow solve, pattern brute force and
planted mistakes.  None of these compare the oracle with itself."""
import json
import os

import numpy as np
import pytest

import oracle as O
from paper_2203_10587_amd import synth as S
from tests import rectform as R

HERE = os.path.dirname(os.path.abspath(__file__))


def small_grids():
    return [
        ("ring9", S.ring9(0)[0]),
        ("rand12", S.random_grid(12, 20, 5, seed=1, parallel=2)),
        ("rand25", S.random_grid(25, 40, 9, seed=7, parallel=1)),
        ("star8", S.random_grid(8, 9, 3, seed=4, star=True, parallel=1)),
    ]


def _it(g, seed=0, sigma=1.0):
    return S.draw_iterate(g, np.random.default_rng(seed), sigma)


def two_bus(r, x, b=0.0, tap=1.0, shift=0.0):
    z = lambda v: np.array([v], float)
    return S.Grid(nbus=2, br_from=np.array([0], np.int32), br_to=np.array([1], np.int32),
                  br_r=z(r), br_x=z(x), br_b=z(b), br_tap=z(tap), br_shift=z(shift),
                  br_rate=z(1.0), bus_pd=np.zeros(2), bus_qd=np.zeros(2),
                  bus_gs=np.zeros(2), bus_bs=np.zeros(2),
                  gen_bus=np.array([0], np.int32), gen_c2=z(0.05), gen_c1=z(20.0),
                  gen_c0=z(3.0), gen_pmin=z(0), gen_pmax=z(2), gen_qmin=z(-1), gen_qmax=z(1))


# --------------------------------------------------------------------------
# closed forms


@pytest.mark.parametrize("X,vf,vt,d", [(0.1, 1.0, 0.95, 0.1), (0.25, 1.04, 0.97, -0.3)])
def test_lossless_line_closed_form(X, vf, vt, d):
    """Textbook lossless-line transfer: P_f = vf vt sin(d)/X,
    Q_f = (vf^2 - vf vt cos d)/X, P_t = -P_f, Q_t = (vt^2 - vf vt cos d)/X."""
    g = two_bus(0.0, X)
    mdl = O.prepare(g)
    x = np.array([d, 0.0, vf, vt, 0.5, 0.1])
    _, Sf, St, _ = O.constraints(mdl, x)
    assert Sf[0].real == pytest.approx(vf * vt * np.sin(d) / X, rel=1e-14)
    assert Sf[0].imag == pytest.approx((vf ** 2 - vf * vt * np.cos(d)) / X, rel=1e-14)
    assert St[0].real == pytest.approx(-vf * vt * np.sin(d) / X, rel=1e-14)
    assert St[0].imag == pytest.approx((vt ** 2 - vf * vt * np.cos(d)) / X, rel=1e-14)


def test_line_charging_and_tap_closed_form():
    """Charging b/2 draws -b/2 v^2 of reactive power at each open end; an
    ideal tap N on an open-ended line scales the from-end charging by 1/N^2."""
    g = two_bus(0.01, 0.1, b=0.3, tap=1.05)
    g.br_x = np.array([1e12])  # effectively open series element
    mdl = O.prepare(g)
    x = np.array([0.2, -0.1, 1.02, 0.98, 0.0, 0.0])
    _, Sf, St, _ = O.constraints(mdl, x)
    assert Sf[0].imag == pytest.approx(-0.15 * 1.02 ** 2 / 1.05 ** 2, rel=1e-9)
    assert St[0].imag == pytest.approx(-0.15 * 0.98 ** 2, rel=1e-9)


def test_objective_closed_form():
    g = S.ring9(0)[0]
    mdl = O.prepare(g)
    it = _it(g, 3)
    f, grad, _ = O.objective(mdl, it.x)
    pg = it.x[2 * g.nbus:2 * g.nbus + g.ngen] * 100.0
    assert f == pytest.approx(float(np.sum(g.gen_c2 * pg ** 2 + g.gen_c1 * pg + g.gen_c0)), rel=1e-15)
    want = np.zeros(mdl.n)
    want[2 * g.nbus:2 * g.nbus + g.ngen] = (2 * g.gen_c2 * pg + g.gen_c1) * 100.0
    np.testing.assert_allclose(grad, want, rtol=1e-15)


# --------------------------------------------------------------------------
# invariants


@pytest.mark.parametrize("name,g", small_grids())
def test_series_losses(name, g):
    """P_f + P_t equals r |y_s|^2 |V_f/N - V_t|^2 >= 0 on every branch."""
    mdl = O.prepare(g)
    it = _it(g, 5)
    _, Sf, St, V = O.constraints(mdl, it.x)
    N = g.br_tap * np.exp(1j * g.br_shift)
    Vs = V[g.br_from] / N - V[g.br_to]
    loss = g.br_r / (g.br_r ** 2 + g.br_x ** 2) * np.abs(Vs) ** 2
    np.testing.assert_allclose(Sf.real + St.real, loss, rtol=1e-11, atol=1e-14)
    assert np.all(loss >= 0)


@pytest.mark.parametrize("name,g", small_grids())
def test_zero_mismatch_at_constructed_power_flow_point(name, g):
    """Choose loads that balance the injections at x (computed by the
    independent rectangular model); the oracle's balance rows then vanish."""
    it = _it(g, 11)
    mdl = O.prepare(g)
    d = R.tensors(g)
    import torch
    xt = torch.as_tensor(it.x)
    Pf, Qf, Pt, Qt = (a.numpy() for a in R.flows(d, xt))
    nb, ng = g.nbus, g.ngen
    v = it.x[nb:2 * nb]
    Pinj = np.zeros(nb)
    Qinj = np.zeros(nb)
    np.add.at(Pinj, g.br_from, Pf)
    np.add.at(Pinj, g.br_to, Pt)
    np.add.at(Qinj, g.br_from, Qf)
    np.add.at(Qinj, g.br_to, Qt)
    Pinj += g.bus_gs * v * v
    Qinj -= g.bus_bs * v * v
    gen_p = np.zeros(nb)
    gen_q = np.zeros(nb)
    np.add.at(gen_p, g.gen_bus, it.x[2 * nb:2 * nb + ng])
    np.add.at(gen_q, g.gen_bus, it.x[2 * nb + ng:])
    g2 = S.Grid(**{**g.__dict__, "bus_pd": gen_p - Pinj, "bus_qd": gen_q - Qinj})
    mdl2 = O.prepare(g2)
    c, _, _, _ = O.constraints(mdl2, it.x)
    s = O.constraint_scales(mdl2, it.x)
    assert np.all(np.abs(c[:2 * nb]) <= 1e-14 * s[:2 * nb])


@pytest.mark.parametrize("name,g", small_grids())
def test_angle_reference_invariance(name, g):
    mdl = O.prepare(g)
    it = _it(g, 2, sigma=0.8)
    nb = g.nbus
    c0 = O.constraints(mdl, it.x)[0]
    x1 = it.x.copy()
    x1[:nb] += 0.37
    c1 = O.constraints(mdl, x1)[0]
    s = O.constraint_scales(mdl, it.x)
    assert np.all(np.abs(c1 - c0) <= 1e-13 * s)
    J = O.jacobian_matrix(mdl, it.x)
    ones = np.zeros(mdl.n)
    ones[:nb] = 1.0
    rs = np.abs(J).toarray().max(axis=1)
    assert np.all(np.abs(J @ ones) <= 1e-13 * np.maximum(rs, 1e-300))
    H = O.hessian_matrix(mdl, it.x, it.sigma, it.lam)
    hs = np.abs(H).toarray().max(axis=1)
    assert np.all(np.abs(H @ ones) <= 1e-13 * np.maximum(hs, 1e-300))


@pytest.mark.parametrize("name,g", small_grids())
def test_euler_homogeneity_in_v(name, g):
    """Bus injections are homogeneous of degree 2 in v and squared flows of
    degree 4, so sum_j v_j dc/dv_j = 2 (injection) or 4 h, and the v-blocks of
    the Hessian satisfy H_vv v = (deg - 1) grad_v and H_theta,v v = deg grad_theta."""
    mdl = O.prepare(g)
    it = _it(g, 8)
    nb, ng, nl = g.nbus, g.ngen, g.nbranch
    v = it.x[nb:2 * nb]
    c = O.constraints(mdl, it.x)[0]
    J = O.jacobian_matrix(mdl, it.x).toarray()
    gen = np.zeros(nb)
    np.add.at(gen, g.gen_bus, it.x[2 * nb:2 * nb + ng])
    genq = np.zeros(nb)
    np.add.at(genq, g.gen_bus, it.x[2 * nb + ng:])
    inj = np.concatenate([c[:nb] + gen - g.bus_pd, c[nb:2 * nb] + genq - g.bus_qd])
    ev = J[:, nb:2 * nb] @ v
    sc = np.abs(J[:, nb:2 * nb]).max(axis=1) * np.max(v)
    assert np.all(np.abs(ev[:2 * nb] - 2 * inj) <= 1e-13 * sc[:2 * nb])
    assert np.all(np.abs(ev[2 * nb:] - 4 * c[2 * nb:]) <= 1e-13 * sc[2 * nb:])
    rng = np.random.default_rng(1)
    for deg, sel in ((2, slice(0, 2 * nb)), (4, slice(2 * nb, 2 * nb + 2 * nl))):
        lam = np.zeros(mdl.m)
        lam[sel] = rng.standard_normal(lam[sel].shape)
        H = O.hessian_matrix(mdl, it.x, 0.0, lam).toarray()
        grad = J.T @ lam
        Hv = H[:, nb:2 * nb] @ v
        scale = np.abs(H).max() + np.abs(grad).max()
        assert np.abs(Hv[nb:2 * nb] - (deg - 1) * grad[nb:2 * nb]).max() <= 1e-12 * scale
        assert np.abs(Hv[:nb] - deg * grad[:nb]).max() <= 1e-12 * scale


# --------------------------------------------------------------------------
# derivatives against finite differences and an independent autograd model


def _fd_step(x):
    return 1e-6 * np.maximum(1.0, np.abs(x))


@pytest.mark.parametrize("name,g", small_grids())
def test_jacobian_central_differences(name, g):
    mdl = O.prepare(g)
    it = _it(g, 4)
    J = O.jacobian_matrix(mdl, it.x).toarray()
    hs = _fd_step(it.x)
    fd = np.zeros_like(J)
    for j in range(mdl.n):
        xp, xm = it.x.copy(), it.x.copy()
        xp[j] += hs[j]
        xm[j] -= hs[j]
        fd[:, j] = (O.constraints(mdl, xp)[0] - O.constraints(mdl, xm)[0]) / (2 * hs[j])
    rs = np.abs(J).max(axis=1, keepdims=True)
    assert np.all(np.abs(fd - J) <= 1e-6 * np.maximum(np.abs(J), rs))


@pytest.mark.parametrize("name,g", small_grids())
def test_hessian_central_differences_of_lagrangian_gradient(name, g):
    """Every Hessian entry against central differences of
    grad L = sigma grad f + J' lambda (which uses only first derivatives)."""
    mdl = O.prepare(g)
    it = _it(g, 6, sigma=1.7)
    H = O.hessian_matrix(mdl, it.x, it.sigma, it.lam).toarray()
    gl = lambda z: it.sigma * O.objective(mdl, z)[1] + O.jacobian_matrix(mdl, z).T @ it.lam
    hs = _fd_step(it.x)
    fd = np.zeros_like(H)
    for j in range(mdl.n):
        xp, xm = it.x.copy(), it.x.copy()
        xp[j] += hs[j]
        xm[j] -= hs[j]
        fd[:, j] = (gl(xp) - gl(xm)) / (2 * hs[j])
    rs = np.abs(H).max(axis=1, keepdims=True)
    assert np.all(np.abs(fd - H) <= 1e-6 * np.maximum(np.abs(H), rs))


@pytest.mark.parametrize("name,g", small_grids())
def test_against_independent_autograd_model(name, g):
    """Values, dense J and dense H against torch autograd of the rectangular
    model in tests/rectform.py (a different derivation route)."""
    mdl = O.prepare(g)
    it = _it(g, 9, sigma=0.6)
    c = O.constraints(mdl, it.x)[0]
    cr, fr = R.values(g, it.x)
    s = O.constraint_scales(mdl, it.x)
    assert np.all(np.abs(c - cr) <= 1e-13 * np.maximum(np.abs(cr), s))
    assert O.objective(mdl, it.x)[0] == pytest.approx(fr, rel=1e-14)
    J = O.jacobian_matrix(mdl, it.x).toarray()
    Jr = R.dense_jacobian(g, it.x)
    rs = np.abs(Jr).max(axis=1, keepdims=True)
    assert np.all(np.abs(J - Jr) <= 1e-13 * np.maximum(np.abs(Jr), rs))
    H = O.hessian_matrix(mdl, it.x, it.sigma, it.lam).toarray()
    Hr = R.dense_hessian(g, it.x, it.sigma, it.lam)
    hs = np.abs(Hr).max(axis=1, keepdims=True)
    assert np.all(np.abs(H - Hr) <= 1e-13 * np.maximum(np.abs(Hr), hs))


@pytest.mark.parametrize("name,g", small_grids())
def test_hessian_symmetric(name, g):
    mdl = O.prepare(g)
    it = _it(g, 12)
    H = O.hessian_matrix(mdl, it.x, it.sigma, it.lam)
    assert abs(H - H.T).max() <= 1e-14 * abs(H).max()


@pytest.mark.parametrize("name,g", small_grids())
def test_vjp_is_weighted_gradient(name, g):
    mdl = O.prepare(g)
    it = _it(g, 13)
    rng = np.random.default_rng(2)
    wc = rng.standard_normal(mdl.m)
    wf = 0.7
    u = O.vjp(mdl, it.x, wf, wc)
    Jr = R.dense_jacobian(g, it.x)
    d = R.tensors(g)
    import torch
    xt = torch.as_tensor(it.x).requires_grad_(True)
    R.objective(d, xt).backward()
    want = wf * xt.grad.numpy() + Jr.T @ wc
    sc = O.vjp_scale(mdl, it.x, wf, wc)
    assert np.all(np.abs(u - want) <= 1e-13 * np.maximum(np.abs(want), sc))


# --------------------------------------------------------------------------
# a Newton power flow driven by the oracle's Jacobian converges quadratically


def test_newton_power_flow_on_ring9():
    """AC power flow (the PFLOW application): slack bus 0 (theta = 0, v = 1,
    Pg_0 and Qg_0 free), PV buses 1, 2 (v = 1, Pg fixed, Qg free), PQ buses
    3..8.  Newton on the 18 balance rows with the oracle's Jacobian columns
    must converge quadratically.  Loads are halved: the random ring at full
    load lies beyond its loadability limit and has no solution."""
    g, _ = S.ring9(0)
    g = S.scale_loads(g, 0.5)
    mdl = O.prepare(g)
    nb, ng = g.nbus, g.ngen
    x = np.zeros(mdl.n)
    x[nb:2 * nb] = 1.0
    x[2 * nb + 1] = x[2 * nb + 2] = g.bus_pd.sum() / 3
    unk = (list(range(1, nb)) + list(range(nb + 3, 2 * nb))
           + [2 * nb, 2 * nb + ng, 2 * nb + ng + 1, 2 * nb + ng + 2])
    res = []
    for _ in range(12):
        c = O.constraints(mdl, x)[0][:2 * nb]
        res.append(np.abs(c).max())
        if res[-1] < 1e-12:
            break
        J = O.jacobian_matrix(mdl, x).toarray()[:2 * nb][:, unk]
        x[unk] -= np.linalg.solve(J, c)
    assert res[-1] < 1e-12
    assert len(res) <= 8
    # quadratic: once in the basin each residual is below C * previous^2
    k = next(i for i, r in enumerate(res) if r < 0.1)
    assert len(res) - k >= 3
    for a, b in zip(res[k:-1], res[k + 1:]):
        assert b <= 10.0 * a * a + 1e-13


# --------------------------------------------------------------------------
# pattern


def test_pattern_nnz_formulas():
    for g in [S.ring9(0)[0], S.random_grid(25, 40, 9, seed=7, parallel=1),
              S.rgg_grid(500, 650, seed=3)]:
        jp, jc, hp, hc = O.pattern(g)
        pairs = {frozenset((int(a), int(b))) for a, b in zip(g.br_from, g.br_to)}
        E, nb, ng, nl = len(pairs), g.nbus, g.ngen, g.nbranch
        assert jp[-1] == 4 * nb + 8 * E + 2 * ng + 8 * nl
        assert hp[-1] == 3 * nb + 4 * E + ng
        for p, c in ((jp, jc), (hp, hc)):
            for i in range(len(p) - 1):
                row = c[p[i]:p[i + 1]]
                assert np.all(np.diff(row) > 0)
        assert np.all(hc <= np.repeat(np.arange(len(hp) - 1), np.diff(hp)))


def test_config_sizes():
    g, it = S.ring9(0)
    jp, _, hp, _ = O.pattern(g)
    assert (g.n, g.m, jp[-1], hp[-1]) == (24, 42, 234, 78)


@pytest.mark.parametrize("name,g", small_grids())
def test_pattern_equals_structural_nonzeros(name, g):
    """Brute force: at a generic point the dense autograd J and lower H are
    nonzero exactly on the pattern."""
    it = _it(g, 21)
    Jr = R.dense_jacobian(g, it.x)
    Hr = np.tril(R.dense_hessian(g, it.x, 1.3, it.lam))
    jp, jc, hp, hc = O.pattern(g)
    for dense, p, c in ((Jr, jp, jc), (Hr, hp, hc)):
        mask = np.zeros(dense.shape, bool)
        mask[np.repeat(np.arange(len(p) - 1), np.diff(p)), c] = True
        assert np.all(dense[~mask] == 0.0)
        assert np.all(np.abs(dense[mask]) > 0.0)


def test_outage_removes_rows_and_slots():
    os_ = S.n1_security_set(0, nb=60, nl=90, count=5)
    base = O.pattern(os_.base)
    for k in range(5):
        l = int(os_.outages[k])
        g = S.remove_branch(os_.base, l)
        jp, _, hp, _ = O.pattern(g)
        assert g.m == os_.base.m - 2
        assert jp[-1] == base[0][-1] - 8 - 8   # 4 balance slots x2 rows, 8 flow entries
        assert hp[-1] == base[2][-1] - 4


# --------------------------------------------------------------------------
# frozen regression values for the 9-bus ring (written by tests/golden/make_golden.py)


def test_golden_ring9():
    with open(os.path.join(HERE, "golden", "ring9_seed0.json")) as fh:
        gold = json.load(fh)
    g, it = S.ring9(0)
    mdl = O.prepare(g)
    out = O.evaluate(mdl, it.x, it.sigma, it.lam)
    np.testing.assert_array_equal(mdl.jac_rowptr, gold["jac_rowptr"])
    np.testing.assert_array_equal(mdl.jac_col, gold["jac_col"])
    np.testing.assert_array_equal(mdl.hess_rowptr, gold["hess_rowptr"])
    np.testing.assert_array_equal(mdl.hess_col, gold["hess_col"])
    for k in ("grad_f", "c", "jac_val", "hess_val"):
        np.testing.assert_allclose(out[k], gold[k], rtol=1e-13, atol=1e-13)
    assert out["f"] == pytest.approx(gold["f"], rel=1e-14)


# --------------------------------------------------------------------------
# planted mistakes: each plausible error in the oracle must trip a pin


def _mutants():
    orig = O.acopf_oracle.branch_admittances

    def shift_sign(grid):
        Yff, Yft, Ytf, Ytt = orig(grid)
        ys = 1.0 / (grid.br_r + 1j * grid.br_x)
        return Yff, -ys / (grid.br_tap * np.exp(1j * grid.br_shift)), Ytf, Ytt

    def no_tap_square(grid):
        Yff, Yft, Ytf, Ytt = orig(grid)
        return Yff * grid.br_tap, Yft, Ytf, Ytt

    def dropped_charging(grid):
        Yff, Yft, Ytf, Ytt = orig(grid)
        return Yff, Yft, Ytf, Ytt - 1j * grid.br_b / 2

    def swapped_transfer(grid):
        Yff, Yft, Ytf, Ytt = orig(grid)
        return Yff, Ytf, Yft, Ytt

    return [shift_sign, no_tap_square, dropped_charging, swapped_transfer]


@pytest.mark.parametrize("mut", _mutants(), ids=lambda f: f.__name__)
def test_planted_admittance_mistakes_are_caught(monkeypatch, mut):
    g = S.random_grid(12, 20, 5, seed=1, parallel=2)
    it = _it(g, 9)
    monkeypatch.setattr(O.acopf_oracle, "branch_admittances", mut)
    mdl = O.prepare(g)
    c = O.constraints(mdl, it.x)[0]
    cr, _ = R.values(g, it.x)
    assert np.abs(c - cr).max() > 1e-6


def test_planted_hessian_mistake_is_caught(monkeypatch):
    """Dropping the mu * grad h grad h' term must fail the FD pin."""
    g = S.random_grid(12, 20, 5, seed=1, parallel=2)
    it = _it(g, 6)
    mdl = O.prepare(g)
    orig = O.acopf_oracle._branch_local_hessians

    def broken(mdl_, x, lam, magnitude=False):
        lam2 = lam.copy()
        lam2[2 * mdl_.nb:] = 0.0
        return orig(mdl_, x, lam2, magnitude)

    monkeypatch.setattr(O.acopf_oracle, "_branch_local_hessians", broken)
    H = O.hessian_matrix(mdl, it.x, it.sigma, it.lam).toarray()
    Hr = R.dense_hessian(g, it.x, it.sigma, it.lam)
    assert np.abs(H - Hr).max() > 1e-3


@pytest.mark.parametrize("cart", [False, True])
def test_hessian_magnitude_companion(cart):
    """The rounding companion of the Hessian scale (each entry's sum of
    absolute terms): at least the entry's magnitude everywhere, equal to it
    on the cost diagonal (one term per entry), and unchanged when every
    multiplier changes sign (which negates the network part of H)."""
    from oracle import cartesian as OC
    g = S.random_grid(14, 22, 5, seed=3, parallel=2)
    mdl = O.prepare(g)
    rng = np.random.default_rng(4)
    it = S.draw_iterate_cartesian(g, rng) if cart else S.draw_iterate(g, rng)
    lam = rng.standard_normal(mdl.m + (g.nbus if cart else 0))
    mod = OC if cart else O
    H = mod.hessian_matrix(mdl, it.x, 0.7, lam).toarray()
    M = mod.hessian_matrix(mdl, it.x, 0.7, lam, magnitude=True).toarray()
    assert np.all(M >= np.abs(H) * (1 - 1e-14) - 1e-300)
    nb = g.nbus
    k = 2 * nb + np.arange(g.ngen)
    np.testing.assert_allclose(M[k, k], np.abs(H[k, k]), rtol=1e-15)
    # flipping every multiplier's sign negates H but leaves M unchanged
    M2 = mod.hessian_matrix(mdl, it.x, 0.7, -lam, magnitude=True).toarray()
    np.testing.assert_allclose(M2[:2 * nb, :2 * nb], M[:2 * nb, :2 * nb], rtol=1e-14)
