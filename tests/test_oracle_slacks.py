"""Pins of the feasibility-slack oracle (no GPU).  The slack columns are
tied to the physics through the base oracle on modified data: an imbalance
"+" variable must move the balance rows exactly as extra generation at its
bus does, a "-" variable as extra load, a load-loss variable as a smaller
load.  The penalty is pinned by hand-computed values, the derivatives by
central differences, the pattern by its structure, and a planted sign error
must fail the generation pin."""
import numpy as np
import pytest

import oracle as O
from oracle import cartesian as OC
from oracle import slacks as OS
from paper_2203_10587_amd import synth as S

FULL = dict(imbalance=True, loadloss=True, imb_cost=(0.4, 30.0), loss_cost=(1.5, 90.0))


def _grid():
    return S.random_grid(14, 22, 6, seed=2, parallel=2)


def _point(g, spec, seed):
    rng = np.random.default_rng(seed)
    if spec.cartesian:
        it = S.draw_iterate_cartesian(g, rng)
    else:
        it = S.draw_iterate(g, rng)
    ns = len(OS.kinds(spec)) * g.nbus
    return np.concatenate([it.x, rng.uniform(0.0, 0.3, ns)]), rng


def _base_c(g, x, cart):
    mdl = O.prepare(g)
    return (OC if cart else O).constraints(mdl, x)[0]


@pytest.mark.parametrize("cart", [False, True])
def test_plus_imbalance_is_generation(cart):
    """dP+ (dQ+) at bus i changes c exactly as raising Pg (Qg) of a generator
    at bus i by the same amount."""
    g = _grid()
    spec = OS.Spec(**FULL, cartesian=cart)
    mdl = O.prepare(g)
    x, _ = _point(g, spec, 1)
    nb, ng = g.nbus, g.ngen
    n0 = mdl.n
    k = 0
    i = int(g.gen_bus[k])
    for slot, off in ((0, 2 * nb + k), (2, 2 * nb + ng + k)):   # dP+, dQ+
        xs = x.copy()
        xs[n0:] = 0.0
        t = 0.0625
        xs[n0 + slot * nb + i] = t
        xb = x[:n0].copy()
        xb[off] += t
        got = OS.constraints(mdl, spec, xs)
        want = _base_c(g, xb, cart)
        assert np.abs(got - want).max() <= 1e-14 * max(1.0, np.abs(want).max())


@pytest.mark.parametrize("cart", [False, True])
def test_minus_imbalance_and_load_loss_are_load(cart):
    """dP- (dQ-) = t at bus i is the load Pd_i + t (Qd_i + t); Pl (Ql) = t
    is the load Pd_i - t (Qd_i - t)."""
    g = _grid()
    spec = OS.Spec(**FULL, cartesian=cart)
    mdl = O.prepare(g)
    x, _ = _point(g, spec, 2)
    nb, n0 = g.nbus, mdl.n
    i, t = 5, 0.125
    for slot, field, sign in ((1, "bus_pd", 1.0), (3, "bus_qd", 1.0), (4, "bus_pd", -1.0),
                              (5, "bus_qd", -1.0)):
        xs = x.copy()
        xs[n0:] = 0.0
        xs[n0 + slot * nb + i] = t
        arr = getattr(g, field).copy()
        arr[i] += sign * t
        g2 = S.Grid(**{**g.__dict__, field: arr})
        want = _base_c(g2, x[:n0], cart)
        got = OS.constraints(mdl, spec, xs)
        assert np.abs(got - want).max() <= 1e-14 * max(1.0, np.abs(want).max()), OS.kinds(spec)[slot][0]


def test_penalty_hand_values():
    """B = 100 MVA, c2 = 0.5 $/MW^2, c1 = 10 $/MW, s = 0.1 pu = 10 MW:
    cost 0.5 * 100 + 10 * 10 = 150, d/ds = 100 (2 * 0.5 * 10 + 10) = 2000,
    d2/ds2 = 2 * 0.5 * 100^2 = 10000 (times sigma)."""
    g = S.Grid(**{**_grid().__dict__, "base_mva": 100.0})
    spec = OS.Spec(imbalance=False, loadloss=True, loss_cost=(0.5, 10.0))
    mdl = O.prepare(g)
    x, _ = _point(g, spec, 3)
    n0, nb = mdl.n, g.nbus
    x[n0:] = 0.0
    f0 = OS.objective(mdl, spec, x)[0]
    x[n0 + 3] = 0.1                 # Pl at bus 3
    x[n0 + nb + 7] = 0.1            # Ql at bus 7
    f1, grad, _ = OS.objective(mdl, spec, x)
    assert abs((f1 - f0) - 300.0) <= 1e-9
    assert abs(grad[n0 + 3] - 2000.0) <= 1e-9 and abs(grad[n0 + nb + 7] - 2000.0) <= 1e-9
    assert abs(grad[n0] - 1000.0) <= 1e-12          # s = 0: c1 B
    H = OS.hessian_matrix(mdl, spec, x, 0.75, np.zeros(mdl.m)).toarray()
    np.testing.assert_allclose(np.diag(H)[n0:], 0.75 * 10000.0, rtol=1e-15)


@pytest.mark.parametrize("cart", [False, True])
def test_differences(cart):
    g = S.random_grid(9, 12, 3, seed=1, parallel=1)
    spec = OS.Spec(**FULL, cartesian=cart)
    mdl = O.prepare(g)
    x, rng = _point(g, spec, 4)
    m = len(OS.constraints(mdl, spec, x))
    lam = rng.standard_normal(m)
    sigma = 0.8
    J = OS.jacobian_matrix(mdl, spec, x).toarray()
    H = OS.hessian_matrix(mdl, spec, x, sigma, lam).toarray()
    grad = OS.objective(mdl, spec, x)[1]
    h = 1e-6
    for j in range(len(x)):
        d = np.zeros(len(x))
        d[j] = h
        fd = (OS.constraints(mdl, spec, x + d) - OS.constraints(mdl, spec, x - d)) / (2 * h)
        assert np.abs(fd - J[:, j]).max() <= 1e-6 * max(1.0, np.abs(J[:, j]).max())
        fdf = (OS.objective(mdl, spec, x + d)[0] - OS.objective(mdl, spec, x - d)[0]) / (2 * h)
        assert abs(fdf - grad[j]) <= 1e-6 * max(1.0, abs(grad[j]))
        lg = lambda z: sigma * OS.objective(mdl, spec, z)[1] + OS.jacobian_matrix(mdl, spec, z).T @ lam
        fdh = (lg(x + d) - lg(x - d)) / (2 * h)
        assert np.abs(fdh - H[:, j]).max() <= 1e-5 * max(1.0, np.abs(H[:, j]).max())


@pytest.mark.parametrize("imb,loss", [(True, False), (False, True), (True, True)])
def test_pattern_structure(imb, loss):
    g = _grid()
    spec = OS.Spec(imbalance=imb, loadloss=loss, imb_cost=(0.3, 1.0), loss_cost=(0.0, 2.0))
    mdl = O.prepare(g)
    nb, n0 = g.nbus, mdl.n
    jp, jc, hp, hc = OS.pattern(mdl, spec)
    ks = OS.kinds(spec)
    nsp = sum(1 for k in ks if k[1] == 0)
    assert len(jc) == len(mdl.jac_col) + 2 * nsp * nb
    assert len(hc) == len(mdl.hess_col) + len(ks) * nb
    for i in (0, 4, nb - 1):
        for r in (0, 1):
            row = jc[jp[r * nb + i]:jp[r * nb + i + 1]]
            want = [n0 + k * nb + i for k, kd in enumerate(ks) if kd[1] == r]
            assert list(row[len(row) - len(want):]) == want
            assert np.all(np.diff(row) > 0)
    for q in range(len(ks) * nb):
        r = n0 + q
        assert list(hc[hp[r]:hp[r + 1]]) == [r]
    # every nonzero at a random point lies on the pattern
    x, _ = _point(g, spec, 6)
    J = OS.jacobian_matrix(mdl, spec, x).toarray()
    on = np.zeros_like(J, bool)
    on[np.repeat(np.arange(len(jp) - 1), np.diff(jp)), jc] = True
    assert not np.any((J != 0) & ~on)


def test_no_slacks_is_the_base_model():
    g = _grid()
    for cart in (False, True):
        spec = OS.Spec(cartesian=cart)
        mdl = O.prepare(g)
        rng = np.random.default_rng(7)
        it = S.draw_iterate_cartesian(g, rng) if cart else S.draw_iterate(g, rng)
        lam = rng.standard_normal(mdl.m + (g.nbus if cart else 0))
        a = OS.evaluate(mdl, spec, it.x, 0.9, lam)
        b = (OC if cart else O).evaluate(mdl, it.x, 0.9, lam)
        for k in ("grad_f", "c", "jac_val", "hess_val"):
            np.testing.assert_array_equal(a[k], b[k])
        assert a["f"] == b["f"]


def test_planted_sign_error_is_caught(monkeypatch):
    """dP+ entering with +1 (as load) breaks the generation pin."""
    g = _grid()
    monkeypatch.setattr(OS, "IMBALANCE", (("dP+", 0, 1.0),) + OS.IMBALANCE[1:])
    spec = OS.Spec(**FULL)
    mdl = O.prepare(g)
    x, _ = _point(g, spec, 1)
    n0, nb, k = mdl.n, g.nbus, 0
    i = int(g.gen_bus[k])
    xs = x.copy()
    xs[n0:] = 0.0
    xs[n0 + i] = 0.0625
    xb = x[:n0].copy()
    xb[2 * nb + k] += 0.0625
    assert np.abs(OS.constraints(mdl, spec, xs) - O.constraints(mdl, xb)[0]).max() > 0.1
