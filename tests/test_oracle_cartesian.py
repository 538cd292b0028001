"""Pins of the power-balance-cartesian oracle (no GPU).  The strongest ties
it to the polar oracle, which is pinned on its own: at e = v cos(theta),
f = v sin(theta) the two give the same constraints, and the first- and
second-order chain rules map the cartesian J and H onto the polar ones.
Central differences, the pattern and a planted sign error complete it."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from oracle import cartesian as OC
from paper_2203_10587_amd import synth as S

GRIDS = {
    "ring9": lambda: S.random_grid(9, 12, 3, seed=1, parallel=1),
    "parallel30": lambda: S.random_grid(30, 48, 9, seed=4, parallel=2),
}


def _polar_point(name, seed=0):
    g = GRIDS[name]()
    it = S.draw_iterate(g, np.random.default_rng(seed))
    mdl = O.prepare(g)
    nb = mdl.nb
    th, v = it.x[:nb], it.x[nb:2 * nb]
    xc = it.x.copy()
    xc[:nb], xc[nb:2 * nb] = v * np.cos(th), v * np.sin(th)
    lam_c = np.concatenate([it.lam, np.zeros(nb)])  # magnitude rows off for the comparison
    return g, it, mdl, xc, lam_c


def _transform(mdl, x_polar, xc):
    """T = d(e, f)/d(theta, v) (2nb x 2nb) and the second derivatives."""
    nb = mdl.nb
    th, v = x_polar[:nb], x_polar[nb:2 * nb]
    e, f = xc[:nb], xc[nb:2 * nb]
    T = sp.bmat([[sp.diags(-f), sp.diags(np.cos(th))], [sp.diags(e), sp.diags(np.sin(th))]],
                format="csr")
    return T, th, e, f


@pytest.mark.parametrize("name", sorted(GRIDS))
def test_values_match_polar(name):
    g, it, mdl, xc, _ = _polar_point(name)
    cp, _, _, _ = O.constraints(mdl, it.x)
    cc, _, _, _ = OC.constraints(mdl, xc)
    sc = O.constraint_scales(mdl, it.x)
    m = mdl.m
    assert np.all(np.abs(cc[:m] - cp) <= 1e-13 * np.maximum(np.abs(cp), sc))
    v = it.x[mdl.nb:2 * mdl.nb]
    assert np.allclose(cc[m:], v * v, rtol=1e-14, atol=0)


@pytest.mark.parametrize("name", sorted(GRIDS))
def test_first_order_chain_rule(name):
    g, it, mdl, xc, _ = _polar_point(name, 1)
    nb = mdl.nb
    Jp = O.jacobian_matrix(mdl, it.x).toarray()
    Jc = OC.jacobian_matrix(mdl, xc).toarray()[:mdl.m]
    T, *_ = _transform(mdl, it.x, xc)
    lhs = Jc[:, :2 * nb] @ T.toarray()
    scale = np.abs(Jc[:, :2 * nb]) @ np.abs(T.toarray()) + 1.0
    assert np.all(np.abs(lhs - Jp[:, :2 * nb]) <= 1e-12 * scale)
    np.testing.assert_array_equal(Jc[:, 2 * nb:], Jp[:, 2 * nb:])


@pytest.mark.parametrize("name", sorted(GRIDS))
def test_second_order_chain_rule(name):
    """H_polar = T' H_cart T + sum_i (dL/de_i) d2e_i + (dL/df_i) d2f_i, with
    d2e/dtheta2 = -e, d2e/dtheta dv = -sin(theta), d2f/dtheta2 = -f,
    d2f/dtheta dv = cos(theta) (the v-v second derivatives vanish)."""
    g, it, mdl, xc, lam_c = _polar_point(name, 2)
    nb = mdl.nb
    Hp = O.hessian_matrix(mdl, it.x, it.sigma, it.lam).toarray()
    Hc = OC.hessian_matrix(mdl, xc, it.sigma, lam_c).toarray()
    T, th, e, f = _transform(mdl, it.x, xc)
    Td = T.toarray()
    Hm = Td.T @ Hc[:2 * nb, :2 * nb] @ Td
    grad = OC.jacobian_matrix(mdl, xc).T @ lam_c  # the cost has no (e, f) part
    Ge, Gf = grad[:nb], grad[nb:2 * nb]
    i = np.arange(nb)
    Hm[i, i] += Ge * (-e) + Gf * (-f)
    cross = Ge * (-np.sin(th)) + Gf * np.cos(th)
    Hm[i, nb + i] += cross
    Hm[nb + i, i] += cross
    scale = np.abs(Td.T) @ np.abs(Hc[:2 * nb, :2 * nb]) @ np.abs(Td) + np.abs(Hp[:2 * nb, :2 * nb]) + 1.0
    assert np.all(np.abs(Hm - Hp[:2 * nb, :2 * nb]) <= 1e-11 * scale)
    np.testing.assert_allclose(Hc[2 * nb:, 2 * nb:], Hp[2 * nb:, 2 * nb:], rtol=1e-15, atol=0)


def test_differences_and_pattern():
    g = GRIDS["parallel30"]()
    mdl = O.prepare(g)
    rng = np.random.default_rng(5)
    it = S.draw_iterate(g, rng)
    nb = mdl.nb
    xc = it.x.copy()
    xc[:nb] = rng.uniform(0.9, 1.1, nb)
    xc[nb:2 * nb] = rng.uniform(-0.2, 0.2, nb)
    lam = rng.standard_normal(mdl.m + nb)
    J = OC.jacobian_matrix(mdl, xc).toarray()
    H = OC.hessian_matrix(mdl, xc, it.sigma, lam).toarray()
    h = 1e-6
    for j in range(mdl.n):
        d = np.zeros(mdl.n)
        d[j] = h
        fd = (OC.constraints(mdl, xc + d)[0] - OC.constraints(mdl, xc - d)[0]) / (2 * h)
        assert np.abs(fd - J[:, j]).max() <= 1e-6 * max(1.0, np.abs(J[:, j]).max())
        gp = it.sigma * O.objective(mdl, xc + d)[1] + OC.jacobian_matrix(mdl, xc + d).T @ lam
        gm = it.sigma * O.objective(mdl, xc - d)[1] + OC.jacobian_matrix(mdl, xc - d).T @ lam
        fdh = (gp - gm) / (2 * h)
        assert np.abs(fdh - H[:, j]).max() <= 1e-5 * max(1.0, np.abs(H[:, j]).max())
    # every nonzero lies on the pattern; the counts follow the polar ones
    jp, jc, hp, hc = OC.pattern(mdl)
    rows = np.repeat(np.arange(len(jp) - 1), np.diff(jp))
    on = np.zeros_like(J, bool)
    on[rows, jc] = True
    assert not np.any((J != 0) & ~on)
    assert len(jc) == len(mdl.jac_col) + 2 * nb
    Hl = np.tril(H)
    hrows = np.repeat(np.arange(len(hp) - 1), np.diff(hp))
    onh = np.zeros_like(Hl, bool)
    onh[hrows, hc] = True
    assert not np.any((Hl != 0) & ~onh)


def test_planted_sign_error_is_caught():
    """dV/df = -j instead of +j (the f columns negated) breaks the chain rule."""
    g, it, mdl, xc, _ = _polar_point("ring9", 3)
    nb = mdl.nb
    Jc = OC.jacobian_matrix(mdl, xc).toarray()[:mdl.m]
    Jc[:, nb:2 * nb] *= -1.0
    T, *_ = _transform(mdl, it.x, xc)
    Jp = O.jacobian_matrix(mdl, it.x).toarray()
    assert np.abs(Jc[:, :2 * nb] @ T.toarray() - Jp[:, :2 * nb]).max() > 1e-3
