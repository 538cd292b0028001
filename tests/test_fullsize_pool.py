"""The host-side pool that checks full-size batches against the oracle (no
GPU): oracle outputs fed back to it pass, a planted one-entry mistake and a
wrong pattern are reported with the instance they belong to."""
import numpy as np

import oracle as O
from paper_2203_10587_amd import synth as S
from tests import fullsize_pool as FP


def _item(os_, k, w=None, corrupt=None, bad_pattern=False, prod=False):
    g, it = S.n1_instance(os_, k)
    mdl = O.prepare(g)
    out = O.evaluate(mdl, it.x, it.sigma, it.lam)
    got = {k2: (np.array(v, copy=True) if k2 != "f" else v) for k2, v in out.items()}
    if w is not None:
        got["u"] = O.vjp(mdl, it.x, *w)
    if prod:  # H d and J d along the instance's seeded direction
        d = FP.direction(k, len(it.x))
        got["hd"] = O.hessian_matrix(mdl, it.x, it.sigma, it.lam) @ d
        got["jd"] = O.jacobian_matrix(mdl, it.x) @ d
    if corrupt:
        got[corrupt][3] += 1e-6 * (1 + abs(got[corrupt][3]))
    pat = [mdl.jac_rowptr, mdl.jac_col, mdl.hess_rowptr, mdl.hess_col.copy()]
    if bad_pattern:
        pat[3][5] += 1
    return k, got, pat, w, prod


def test_pool_accepts_oracle_outputs_and_flags_mistakes():
    os_ = S.n1_security_set(0)
    rng = np.random.default_rng(1)
    w = (0.7, rng.standard_normal(os_.iterates[2].lam.shape))
    items = [_item(os_, 0), _item(os_, 1, corrupt="jac_val"), _item(os_, 2, w=w),
             _item(os_, 3, bad_pattern=True), _item(os_, 4, corrupt="hess_val"),
             _item(os_, 5, prod=True), _item(os_, 6, prod=True, corrupt="hd")]
    res, bad = FP.check_all("n1", "polar", items, nproc=2)
    assert sorted(r[0] for r in res) == [0, 2, 5]
    assert sorted(r[0] for r in bad) == [1, 3, 4, 6]
    msgs = {r[0]: r[2] for r in bad}
    assert "jac_val" in msgs[1] and "hess_col" in msgs[3] and "hess_val" in msgs[4]
    assert ".hd" in msgs[6]
    assert {"hd", "jd"} <= set(next(r[2] for r in res if r[0] == 5))
    assert all(v == 0.0 for r in res for v in r[2].values())
