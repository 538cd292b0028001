"""The C-ABI library on the host: it loads, exports every function the header
declares, and its host-side pattern builder agrees bit for bit with the
oracle's structural rule (base nets and N-1 outages).  No GPU needed."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle as O
from paper_2203_10587_amd import acopf as A
from paper_2203_10587_amd import synth as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "acopf.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(acopf_\w+)\s*\(", txt, re.M)))


def test_library_exports_every_declared_function():
    names = header_functions()
    assert len(names) >= 18
    L = A.lib()
    for n in names:
        assert hasattr(L, n), n
        assert n in A._SIGS, f"binding lacks {n}"
    assert L.acopf_version() >= 10000


def _grids():
    yield "ring9", S.ring9(0)[0]
    yield "rand30", S.random_grid(30, 50, 11, seed=3, parallel=3)
    yield "star40", S.random_grid(40, 45, 6, seed=8, star=True, parallel=2)
    yield "rgg800", S.rgg_grid(800, 1040, seed=2)
    yield "nogen", S.random_grid(12, 15, 0, seed=1)
    yield "isolated", S.Grid(**{**S.random_grid(6, 5, 2, seed=4).__dict__, "nbus": 8,
                                "bus_pd": np.zeros(8), "bus_qd": np.zeros(8),
                                "bus_gs": np.zeros(8), "bus_bs": np.zeros(8)})


@pytest.mark.parametrize("name,g", list(_grids()))
def test_host_pattern_bit_exact(name, g):
    dims, jp, jc, hp, hc = A.acopf_pattern_host(g)
    ojp, ojc, ohp, ohc = O.pattern(g)
    np.testing.assert_array_equal(jp, ojp)
    np.testing.assert_array_equal(jc, ojc)
    np.testing.assert_array_equal(hp, ohp)
    np.testing.assert_array_equal(hc, ohc)
    assert (dims.n, dims.m) == (g.n, g.m)
    assert dims.outage == -1


@pytest.mark.parametrize("name,g", [x for x in _grids() if x[1].nbranch > 0])
def test_host_pattern_bit_exact_outages(name, g):
    rng = np.random.default_rng(0)
    picks = rng.choice(g.nbranch, min(g.nbranch, 12), replace=False)
    # include every parallel branch: the slot must survive their removal
    pairs = {}
    for l in range(g.nbranch):
        pairs.setdefault(frozenset((int(g.br_from[l]), int(g.br_to[l]))), []).append(l)
    par = [l for ls in pairs.values() if len(ls) > 1 for l in ls]
    for l in sorted(set(picks.tolist()) | set(par)):
        dims, jp, jc, hp, hc = A.acopf_pattern_host(g, int(l))
        g2 = S.remove_branch(g, int(l))
        ojp, ojc, ohp, ohc = O.pattern(g2)
        np.testing.assert_array_equal(jp, ojp)
        np.testing.assert_array_equal(jc, ojc)
        np.testing.assert_array_equal(hp, ohp)
        np.testing.assert_array_equal(hc, ohc)
        assert (dims.m, dims.nbranch, dims.outage) == (g2.m, g2.nbranch, l)


def _bad(g, **kw):
    return S.Grid(**{**g.__dict__, **kw})


@pytest.mark.parametrize("mut,msg", [
    (lambda g: _bad(g, br_to=np.where(np.arange(g.nbranch) == 2, g.br_from, g.br_to)), "from == to"),
    (lambda g: _bad(g, br_to=np.where(np.arange(g.nbranch) == 1, 99, g.br_to)), "out of range"),
    (lambda g: _bad(g, br_r=np.where(np.arange(g.nbranch) == 0, 0.0, g.br_r),
                    br_x=np.where(np.arange(g.nbranch) == 0, 0.0, g.br_x)), "zero impedance"),
    (lambda g: _bad(g, br_tap=np.where(np.arange(g.nbranch) == 3, 0.0, g.br_tap)), "tap"),
    (lambda g: _bad(g, bus_pd=np.where(np.arange(g.nbus) == 3, np.nan, g.bus_pd)), "non-finite"),
    (lambda g: _bad(g, gen_bus=np.array([0, 1, 12], np.int32)), "bus out of range"),
    (lambda g: _bad(g, base_mva=0.0), "base_mva"),
])
def test_validation_errors(mut, msg):
    g = mut(S.ring9(0)[0])
    with pytest.raises(A.AcopfError) as ei:
        A.acopf_pattern_host(g)
    assert ei.value.code == A.ACOPF_EINVAL
    assert msg in str(ei.value)


def test_outage_index_validation():
    g = S.ring9(0)[0]
    for bad in (-2, 12, 100):
        with pytest.raises(A.AcopfError):
            A.acopf_pattern_host(g, bad)


def test_null_arguments_return_einval():
    L = A.lib()
    assert L.acopf_net_create(None, None) == A.ACOPF_EINVAL
    assert L.acopf_eval_f_g(None, None, None, None, None, None) == A.ACOPF_EINVAL
    assert L.acopf_batch_create(None, 0, None, C.byref(C.c_void_p())) == A.ACOPF_EINVAL
    assert L.acopf_last_error()


@pytest.mark.parametrize("name,g", [x for x in _grids() if x[0] in ("ring9", "rand30", "star40", "nogen")])
def test_host_pattern_cartesian_bit_exact(name, g):
    """The cartesian representation: the polar rows with (e, f) in the places
    of (theta, v), then one (e_i, f_i) row per bus; the same H pattern."""
    from oracle import cartesian as OC
    dims, jp, jc, hp, hc = A.acopf_pattern_host_form(g, A.ACOPF_CARTESIAN)
    ojp, ojc, ohp, ohc = OC.pattern(O.prepare(g))
    for a, b in ((jp, ojp), (jc, ojc), (hp, ohp), (hc, ohc)):
        np.testing.assert_array_equal(a, b)
    assert (dims.n, dims.m) == (g.n, g.m + g.nbus)
    if g.nbranch:
        for l in (0, g.nbranch - 1):
            dims, jp, jc, hp, hc = A.acopf_pattern_host_form(g, A.ACOPF_CARTESIAN, l)
            ojp, ojc, ohp, ohc = OC.pattern(O.prepare(S.remove_branch(g, l)))
            for a, b in ((jp, ojp), (jc, ojc), (hp, ohp), (hc, ohc)):
                np.testing.assert_array_equal(a, b)
            assert dims.m == g.m - 2 + g.nbus


def test_form_validation():
    g = S.ring9(0)[0]
    with pytest.raises(A.AcopfError) as ei:
        A.acopf_pattern_host_form(g, 2)
    assert ei.value.code == A.ACOPF_EINVAL
    # the polar entry point is the polar form
    a = A.acopf_pattern_host(g)
    b = A.acopf_pattern_host_form(g, A.ACOPF_POLAR)
    for x, y in zip(a[1:], b[1:]):
        np.testing.assert_array_equal(x, y)


@pytest.mark.parametrize("slacks", [1, 2, 3])
@pytest.mark.parametrize("cart", [False, True])
def test_host_pattern_slacks_bit_exact(slacks, cart):
    """Slack blocks: each balance row gains its slack columns after the
    generators; H gains one diagonal entry per slack column."""
    from oracle import slacks as OS
    for name, g in _grids():
        if name not in ("ring9", "rand30", "nogen", "isolated"):
            continue
        spec = OS.Spec(imbalance=bool(slacks & 1), loadloss=bool(slacks & 2), cartesian=cart)
        opts = A.net_opts(A.ACOPF_CARTESIAN if cart else A.ACOPF_POLAR, slacks)
        dims, jp, jc, hp, hc = A.acopf_pattern_host_opts(g, opts)
        for a, b in zip((jp, jc, hp, hc), OS.pattern(O.prepare(g), spec)):
            np.testing.assert_array_equal(a, b)
        ns = len(OS.kinds(spec))
        assert (dims.n, dims.m) == (g.n + ns * g.nbus, g.m + (g.nbus if cart else 0))
        if g.nbranch:
            l = g.nbranch // 2
            dims, jp, jc, hp, hc = A.acopf_pattern_host_opts(g, opts, l)
            for a, b in zip((jp, jc, hp, hc), OS.pattern(O.prepare(S.remove_branch(g, l)), spec)):
                np.testing.assert_array_equal(a, b)


def test_opts_validation():
    g = S.ring9(0)[0]
    for bad in (A.net_opts(3, 0), A.net_opts(0, 4), A.net_opts(0, 1, (float("nan"), 0.0))):
        with pytest.raises(A.AcopfError) as ei:
            A.acopf_pattern_host_opts(g, bad)
        assert ei.value.code == A.ACOPF_EINVAL
    a = A.acopf_pattern_host(g)
    b = A.acopf_pattern_host_opts(g, None)
    for x, y in zip(a[1:], b[1:]):
        np.testing.assert_array_equal(x, y)


@pytest.mark.parametrize("name,g", [x for x in _grids() if x[1].nbranch > 0])
def test_flow_limits_are_rate_squared(name, g):
    """h+ of each flow row: rate^2 of its branch (from ends, then to ends),
    unlimited for rate <= 0; an outage drops its branch's two rows."""
    rate = np.asarray(g.br_rate, dtype=np.float64).copy()
    rate[::5] = 0.0  # some unlimited branches
    g = S.Grid(**{**g.__dict__, "br_rate": rate})
    want = np.where(rate > 0, rate * rate, np.inf)
    np.testing.assert_array_equal(A.acopf_flow_limits_host(g), np.concatenate([want, want]))
    l = g.nbranch // 2
    keep = np.arange(g.nbranch) != l
    np.testing.assert_array_equal(A.acopf_flow_limits_host(g, l),
                                  np.concatenate([want[keep], want[keep]]))


def test_dims_report_equality_rows():
    g = S.random_grid(30, 50, 11, seed=3, parallel=3)
    for form in (A.ACOPF_POLAR, A.ACOPF_CARTESIAN):
        dims, *_ = A.acopf_pattern_host_form(g, form)
        assert dims.m_eq == 2 * g.nbus
        assert dims.m == 2 * g.nbus + 2 * g.nbranch + (g.nbus if form == A.ACOPF_CARTESIAN else 0)


def test_non_finite_rate_is_rejected():
    g = S.ring9(0)[0]
    rate = np.asarray(g.br_rate, dtype=np.float64).copy()
    rate[3] = np.nan
    with pytest.raises(A.AcopfError) as ei:
        A.acopf_pattern_host(S.Grid(**{**g.__dict__, "br_rate": rate}))
    assert ei.value.code == A.ACOPF_EINVAL and "branch 3" in str(ei.value)
