"""CPU oracle for the feasibility slack variables: load loss and power
imbalance.

TEST INFRASTRUCTURE: imported only by tests/ (never by the HIP path).

Paper: OPFLOW section, its table of formulation features, which lists
feasibility variables for load loss and power imbalance beside the standard
ACOPF and gives no equations for them.  Reading taken here:
  * power imbalance: four non-negative variables per bus, dP+ and dP- in the
    bus's active balance row, dQ+ and dQ- in its reactive row; the "+"
    variable supplies power (it enters the row as generation does, with -1),
    the "-" variable absorbs it (as load does, with +1);
  * load loss: two variables per bus, Pl and Ql, the part of the bus load
    that is shed (coefficient -1: the load Pd - Pl remains);
  * each kind is penalised on MW like the generator cost,
    c2 (B s)^2 + c1 (B s) with B the base MVA, one (c2, c1) for the
    imbalance variables and one for load loss; the bounds (s >= 0,
    Pl <= Pd) are the solver's;
  * the variables follow Qg as blocks of nb, in the order dP+, dP-, dQ+,
    dQ-, Pl, Ql (enabled kinds only); they apply to either representation
    (polar or cartesian), whose own rows are unchanged.

Written from that definition, over x = [x_base; s]:
    f = f_base(x_base) + sum over slacks of c2 (B s)^2 + c1 B s
    c = c_base(x_base) + S s       (S: one +-1 per slack, in its bus's row)
    J = [J_base, S]
    H = blockdiag(H_base, sigma diag(2 c2 B^2))
Patterns: the base pattern with each slack's column appended to its bus's
row (slack columns exceed every base column, so rows stay ascending); the
Hessian gains one diagonal row entry per slack column, explicit zeros kept.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from . import acopf_oracle as P
from . import cartesian as C

# name, balance row (0 active, 1 reactive), coefficient in that row
IMBALANCE = (("dP+", 0, -1.0), ("dP-", 0, 1.0), ("dQ+", 1, -1.0), ("dQ-", 1, 1.0))
LOADLOSS = (("Pl", 0, -1.0), ("Ql", 1, -1.0))


@dataclass
class Spec:
    imbalance: bool = False
    loadloss: bool = False
    imb_cost: tuple = (0.0, 0.0)    # (c2, c1) per MW
    loss_cost: tuple = (0.0, 0.0)
    cartesian: bool = False


def kinds(spec: Spec):
    """(name, row, coef, c2, c1) of each slack block, in layout order."""
    out = []
    if spec.imbalance:
        out += [(nm, r, cf) + tuple(spec.imb_cost) for nm, r, cf in IMBALANCE]
    if spec.loadloss:
        out += [(nm, r, cf) + tuple(spec.loss_cost) for nm, r, cf in LOADLOSS]
    return out


def _base(spec):
    return C if spec.cartesian else P


def base_sizes(mdl, spec):
    """(n, m) of the representation without slacks."""
    return mdl.n, mdl.m + (mdl.nb if spec.cartesian else 0)


def base_pattern(mdl, spec):
    if spec.cartesian:
        return C.pattern(mdl)
    return mdl.jac_rowptr, mdl.jac_col, mdl.hess_rowptr, mdl.hess_col


def split(mdl, spec, x):
    n0, _ = base_sizes(mdl, spec)
    return np.asarray(x[:n0]), np.asarray(x[n0:])


def slack_matrix(mdl, spec) -> sp.csr_matrix:
    """S (m_base x ns nb): slack (kind k, bus i) in row (row_k nb + i)."""
    nb = mdl.nb
    _, m0 = base_sizes(mdl, spec)
    ks = kinds(spec)
    rows, cols, vals = [], [], []
    for k, (_, r, cf, _, _) in enumerate(ks):
        rows.append(r * nb + np.arange(nb))
        cols.append(k * nb + np.arange(nb))
        vals.append(np.full(nb, cf))
    if not ks:
        return sp.csr_matrix((m0, 0))
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(m0, len(ks) * nb))


def _penalty(mdl, spec, s):
    """Per-slack cost terms, their gradient and their second derivative."""
    B = mdl.grid.base_mva
    ks = kinds(spec)
    c2 = np.repeat([k[3] for k in ks], mdl.nb) if ks else np.zeros(0)
    c1 = np.repeat([k[4] for k in ks], mdl.nb) if ks else np.zeros(0)
    terms = c2 * (B * s) ** 2 + c1 * (B * s)
    grad = 2.0 * c2 * B * B * s + c1 * B
    return terms, grad, 2.0 * c2 * B * B


def objective(mdl, spec, x):
    xb, s = split(mdl, spec, x)
    fb, gb, fs = P.objective(mdl, xb)
    terms, gs, _ = _penalty(mdl, spec, s)
    return (fb + float(np.sum(terms)), np.concatenate([gb, gs]),
            fs + float(np.sum(np.abs(terms))))


def constraints(mdl, spec, x):
    xb, s = split(mdl, spec, x)
    cb = _base(spec).constraints(mdl, xb)[0]
    return cb + slack_matrix(mdl, spec) @ s


def jacobian_matrix(mdl, spec, x) -> sp.csr_matrix:
    xb, _ = split(mdl, spec, x)
    return sp.hstack([_base(spec).jacobian_matrix(mdl, xb), slack_matrix(mdl, spec)],
                     format="csr")


def hessian_matrix(mdl, spec, x, sigma, lam, magnitude: bool = False) -> sp.csr_matrix:
    """Full symmetric Hessian of sigma f + lam' c (with magnitude=True, the
    base representation's sum of absolute terms per entry)."""
    xb, s = split(mdl, spec, x)
    _, m0 = base_sizes(mdl, spec)
    Hb = _base(spec).hessian_matrix(mdl, xb, sigma, np.asarray(lam)[:m0], magnitude=magnitude)
    _, _, d2 = _penalty(mdl, spec, s)
    d = np.abs(sigma * d2) if magnitude else sigma * d2
    return sp.block_diag([Hb, sp.diags(d)], format="csr")


def pattern(mdl, spec):
    """J and lower-H patterns (int32 rowptr / col)."""
    jp, jc, hp, hc = base_pattern(mdl, spec)
    n0, m0 = base_sizes(mdl, spec)
    ns = slack_matrix(mdl, spec).shape[1]
    Jb = sp.csr_matrix((np.ones(len(jc)), np.asarray(jc), np.asarray(jp)), shape=(m0, n0))
    Jf = sp.hstack([Jb, abs(slack_matrix(mdl, spec))], format="csr")
    Jf.sort_indices()
    Hb = sp.csr_matrix((np.ones(len(hc)), np.asarray(hc), np.asarray(hp)), shape=(n0, n0))
    Hf = sp.block_diag([Hb, sp.identity(ns)], format="csr")
    Hf.sort_indices()
    return (Jf.indptr.astype(np.int32), Jf.indices.astype(np.int32),
            Hf.indptr.astype(np.int32), Hf.indices.astype(np.int32))


def evaluate(mdl, spec, x, sigma=1.0, lam=None):
    jp, jc, hp, hc = pattern(mdl, spec)
    f, grad, _ = objective(mdl, spec, x)
    out = {"f": f, "grad_f": grad, "c": constraints(mdl, spec, x),
           "jac_val": P._values_at(jacobian_matrix(mdl, spec, x), jp, jc)}
    if lam is not None:
        out["hess_val"] = P._values_at(hessian_matrix(mdl, spec, x, sigma, lam), hp, hc)
    return out


def vjp(mdl, spec, x, w_f, w_c):
    _, grad, _ = objective(mdl, spec, x)
    return w_f * grad + jacobian_matrix(mdl, spec, x).T @ w_c


def scales(mdl, spec, x, out, sigma=None, lam=None):
    """The base representation's scales, widened by the slack terms: the
    balance rows by |S| |s|, J rows by their +-1 entries, f by the
    penalty terms' magnitudes; H entries, given sigma and lambda, at least
    the sum of the absolute values of their terms."""
    xb, s = split(mdl, spec, x)
    base = _base(spec)
    jpb, jcb, _, _ = base_pattern(mdl, spec)
    ob = base.evaluate(mdl, xb)
    sb = base.scales(mdl, xb, ob)
    Sm = slack_matrix(mdl, spec)
    jp, _, hp, _ = pattern(mdl, spec)
    nz = np.diff(jpb) > 0
    row_b = np.zeros(len(jpb) - 1)
    row_b[nz] = np.maximum.reduceat(sb["jac_val"], np.asarray(jpb)[:-1][nz])
    row_s = np.asarray(abs(Sm).max(axis=1).todense()).ravel() if Sm.shape[1] else 0.0
    _, _, fs = objective(mdl, spec, x)
    res = {"f": fs, "grad_f": np.abs(out["grad_f"]),
           "c": sb["c"] + abs(Sm) @ np.abs(s),
           "jac_val": np.repeat(np.maximum(row_b, row_s), np.diff(jp))}
    if "hess_val" in out:
        res["hess_val"] = P._row_absmax(hp, out["hess_val"])
        if lam is not None:
            Hm = hessian_matrix(mdl, spec, x, sigma, lam, magnitude=True)
            res["hess_val"] = np.maximum(res["hess_val"], P._values_at(Hm, hp, pattern(mdl, spec)[3]))
    return res


def vjp_scale(mdl, spec, x, w_f, w_c):
    _, grad, _ = objective(mdl, spec, x)
    jp, jc, _, _ = pattern(mdl, spec)
    jv = P._values_at(jacobian_matrix(mdl, spec, x), jp, jc)
    sj = scales(mdl, spec, x, {"jac_val": jv, "grad_f": grad})["jac_val"]
    rows = np.repeat(np.arange(len(jp) - 1), np.diff(jp))
    Sj = sp.csr_matrix((sj, (rows, jc)), shape=(len(jp) - 1, len(grad)))
    return abs(w_f) * np.abs(grad) + Sj.T @ np.abs(w_c)
