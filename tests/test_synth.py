"""The seeded input generator: sizes, structure and reproducibility."""
import numpy as np
import pytest
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components

from paper_2203_10587_amd import synth as S


def _connected(nb, f, t):
    A = coo_matrix((np.ones(len(f)), (f, t)), shape=(nb, nb))
    return connected_components(A, directed=False)[0] == 1


def _simple(f, t):
    pairs = {frozenset((int(a), int(b))) for a, b in zip(f, t)}
    return len(pairs) == len(f) and np.all(f != t)


def test_ring9_structure():
    g, it = S.ring9(0)
    assert (g.nbus, g.nbranch, g.ngen) == (9, 12, 3)
    assert list(g.gen_bus) == [0, 1, 2]
    assert np.all(g.bus_pd[:3] == 0) and np.all(g.bus_pd[3:] > 0)
    np.testing.assert_allclose(g.bus_qd, 0.3 * g.bus_pd)
    assert _simple(g.br_from, g.br_to) and _connected(9, g.br_from, g.br_to)
    for l in range(9):
        assert {int(g.br_from[l]), int(g.br_to[l])} == {l, (l + 1) % 9}
    nb = 9
    assert np.all(np.abs(it.x[:nb]) <= 0.2) and np.all(np.abs(it.x[nb:2 * nb] - 1) <= 0.05)
    assert it.lam.shape == (g.m,)


def test_rgg_counts_and_structure():
    g = S.rgg_grid(2000, 3000, seed=5)
    assert (g.nbus, g.nbranch, g.ngen) == (2000, 3000, 500)
    assert int(np.sum(g.bus_pd > 0)) == 1400
    assert int(np.sum(g.br_tap != 1.0)) == 600
    assert np.all(g.br_from < g.br_to)
    assert _simple(g.br_from, g.br_to) and _connected(2000, g.br_from, g.br_to)
    key = g.br_from.astype(np.int64) * 2000 + g.br_to
    assert np.all(np.diff(key) > 0)


def test_grid_10k_sizes():
    g, it = S.grid_10k(0)
    assert (g.nbus, g.nbranch, g.ngen, int(np.sum(g.bus_pd > 0))) == (10000, 13000, 2500, 7000)
    assert int(np.sum(g.br_tap != 1.0)) == 2600
    assert it.x.shape == (25000,) and it.lam.shape == (46000,)


def test_bridges_brute_force():
    g = S.random_grid(30, 36, 4, seed=2, parallel=1)
    br = S.bridges(g.nbus, g.br_from, g.br_to)
    for l in range(g.nbranch):
        keep = np.arange(g.nbranch) != l
        assert br[l] == (not _connected(g.nbus, g.br_from[keep], g.br_to[keep]))


def test_n1_outages_are_non_bridges_and_distinct():
    os_ = S.n1_security_set(0, nb=200, nl=300, count=50)
    assert len(set(os_.outages.tolist())) == 50
    br = S.bridges(200, os_.base.br_from, os_.base.br_to)
    assert not np.any(br[os_.outages])
    for k in (0, 49):
        g, it = S.n1_instance(os_, k)
        assert g.nbranch == 299 and it.lam.shape == (g.m,)
        assert _connected(200, g.br_from, g.br_to)


def test_determinism_and_child_independence():
    a = S.uneven_scenarios(7, count=6, lo=200, hi=400, only=[1, 4])
    b = S.uneven_scenarios(7, count=6, lo=200, hi=400)
    for (k, ga, ia) in a:
        gb, ib = b[k][1], b[k][2]
        np.testing.assert_array_equal(ga.br_from, gb.br_from)
        np.testing.assert_array_equal(ia.x, ib.x)
        np.testing.assert_array_equal(ia.lam, ib.lam)
    g1, i1 = S.ring9(3)
    g2, i2 = S.ring9(3)
    np.testing.assert_array_equal(i1.lam, i2.lam)
    np.testing.assert_array_equal(g1.br_x, g2.br_x)


def test_uneven_scenario_size_distribution():
    sz = S.uneven_scenario_sizes(0)
    assert len(sz) == 512 and sz.min() >= 200 and sz.max() <= 25000
    assert 2.3e6 < sz.sum() < 3.0e6


@pytest.mark.parametrize("kw", [dict(), dict(star=True), dict(parallel=3)])
def test_random_grid_features(kw):
    g = S.random_grid(20, 30, 8, seed=1, **kw)
    assert _connected(20, g.br_from, g.br_to)
    assert np.all(g.br_from != g.br_to)
    if kw.get("parallel", 1):
        pairs = [frozenset((int(a), int(b))) for a, b in zip(g.br_from, g.br_to)]
        assert len(set(pairs)) < len(pairs)
