"""Pins of the coupled-problem oracle (no GPU): the assembled Jacobian
against central differences of the assembled constraints, linearity and
zeros of the coupling rows, the transposed product against loops over the
links, and a planted sign error that the difference pin catches."""
import numpy as np
import pytest

import oracle as O
from oracle import coupled as OC
from paper_2203_10587_amd import synth as S


def _star(seed=3):
    """A base grid with parallel branches and shunts, two N-1 children, and a
    load-scaled copy: links child -> base and a chain copy -> child."""
    g = S.random_grid(12, 18, 4, seed=seed, parallel=2)
    grids = [g, S.remove_branch(g, 2), S.remove_branch(g, 5), S.scale_loads(g, 1.1)]
    models = [O.prepare(x) for x in grids]
    rng = np.random.default_rng(seed)
    its = [S.draw_iterate(x, rng) for x in grids]
    links = [(1, 0), (2, 0), (3, 1)]
    return models, its, links


def _c_global(models, xs, links):
    """The assembled constraints, written directly: each instance's c, then
    Pg(child) - Pg(parent) per link and generator."""
    parts = [O.constraints(m, x)[0] for m, x in zip(models, xs)]
    for a, b in links:
        ma, mb = models[a], models[b]
        parts.append(xs[a][2 * ma.nb: 2 * ma.nb + ma.ng] - xs[b][2 * mb.nb: 2 * mb.nb + mb.ng])
    return np.concatenate(parts)


def _split(models, xg):
    xo, _ = OC.offsets(models)
    return [xg[xo[k]:xo[k + 1]].copy() for k in range(len(models))]


def _fd_jacobian(models, xg, links, h=1e-6):
    cols = []
    for j in range(xg.size):
        e = np.zeros_like(xg)
        e[j] = h
        cp = _c_global(models, _split(models, xg + e), links)
        cm = _c_global(models, _split(models, xg - e), links)
        cols.append((cp - cm) / (2 * h))
    return np.array(cols).T


def test_assembled_jacobian_matches_differences():
    models, its, links = _star()
    out = OC.assemble(models, [i.x for i in its], [i.sigma for i in its], [i.lam for i in its],
                      links)
    fd = _fd_jacobian(models, out["x"], links)
    J = out["J"].toarray()
    assert J.shape == fd.shape
    assert np.abs(J - fd).max() <= 1e-6 * max(1.0, np.abs(fd).max())
    # block sizes: every instance's rows, then ng rows per link
    assert J.shape[0] == sum(m.m for m in models) + sum(models[a].ng for a, _ in links)


def test_coupling_rows_zero_and_linear():
    models, its, links = _star(5)
    xs = [i.x.copy() for i in its]
    # equal dispatch in every instance: every row vanishes
    base_pg = xs[0][2 * models[0].nb: 2 * models[0].nb + models[0].ng].copy()
    for k, m in enumerate(models):
        xs[k][2 * m.nb: 2 * m.nb + m.ng] = base_pg
    assert np.array_equal(OC.coupling_rows(models, xs, links), np.zeros(sum(models[a].ng for a, _ in links)))
    # linear: rows(x + t d) = rows(x) + t J_couple d, exactly for a power-of-two t
    rng = np.random.default_rng(0)
    xg = np.concatenate(xs)
    d = rng.standard_normal(xg.size)
    Jc = OC.coupling_matrix(models, links)
    t = 0.25
    lhs = OC.coupling_rows(models, _split(models, xg + t * d), links)
    rhs = OC.coupling_rows(models, xs, links) + t * (Jc @ d)
    assert np.abs(lhs - rhs).max() <= 1e-14 * max(1.0, np.abs(rhs).max())


def test_transposed_product_by_loops():
    models, its, links = _star(7)
    Jc = OC.coupling_matrix(models, links)
    xo, _ = OC.offsets(models)
    w = np.random.default_rng(1).standard_normal(Jc.shape[0])
    u = np.zeros(Jc.shape[1])
    r = 0
    for a, b in links:
        for k in range(models[a].ng):
            u[xo[a] + 2 * models[a].nb + k] += w[r]
            u[xo[b] + 2 * models[b].nb + k] -= w[r]
            r += 1
    assert np.abs(Jc.T @ w - u).max() <= 1e-15 * max(1.0, np.abs(u).max())


def test_planted_sign_error_is_caught():
    models, its, links = _star(9)
    xg = np.concatenate([i.x for i in its])
    fd = _fd_jacobian(models, xg, links)
    m0 = sum(m.m for m in models)
    wrong = OC.coupling_matrix(models, links).copy()
    wrong.data = -wrong.data  # parent +1, child -1
    assert np.abs(wrong.toarray() - fd[m0:]).max() > 0.5


def test_generator_mismatch_rejected():
    g1 = S.random_grid(12, 18, 4, seed=1)
    g2 = S.random_grid(12, 18, 5, seed=1)
    with pytest.raises(ValueError):
        OC.coupling_matrix([O.prepare(g1), O.prepare(g2)], [(1, 0)])
