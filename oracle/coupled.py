"""CPU oracle for the coupled multi-instance problem.

TEST INFRASTRUCTURE: imported only by tests/ (never by the HIP path).

Paper: SCOPFLOW, TCOPFLOW and SOPFLOW sections.  Subproblems (a base case
and its contingencies, consecutive time periods, scenarios) are joined into
one block-structured problem by coupling constraints
    -delta <= x_a - x_b <= delta,
written for a contingency against its base case, a period against the one
before it and a scenario against the base; the paper's example of the
coupled quantity is generator real power.  Reading taken here: each link
(child a, parent b) contributes one row per generator k,
    r = Pg_k(a) - Pg_k(b),
blocks in link order, generators in index order; the bounds +-delta belong to
the solver, and the rows are linear, so they contribute nothing to the
Hessian.

The assembled problem, over x = [x_0; x_1; ...; x_{K-1}] (instance blocks in
order):
    c = [c_0; ...; c_{K-1}; coupling rows],
    J = [blockdiag(J_0, ..., J_{K-1}); J_couple],
    H = blockdiag(H_0, ..., H_{K-1}).
Everything here is written from that definition with scipy.sparse; the
per-instance blocks come from acopf_oracle.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import acopf_oracle as O


def offsets(models):
    """Start of each instance block in the global x and c (length K + 1)."""
    xo = np.concatenate([[0], np.cumsum([m.n for m in models])]).astype(np.int64)
    co = np.concatenate([[0], np.cumsum([m.m for m in models])]).astype(np.int64)
    return xo, co


def coupling_matrix(models, links) -> sp.csr_matrix:
    """J_couple over the global x: one +1 (child) and one -1 (parent) per row."""
    xo, _ = offsets(models)
    rows, cols, vals = [], [], []
    r = 0
    for a, b in links:
        ma, mb = models[a], models[b]
        if ma.ng != mb.ng:
            raise ValueError("coupled instances need the same generators")
        for k in range(ma.ng):
            rows += [r, r]
            cols += [xo[a] + 2 * ma.nb + k, xo[b] + 2 * mb.nb + k]
            vals += [1.0, -1.0]
            r += 1
    return sp.csr_matrix((vals, (rows, cols)), shape=(r, int(xo[-1])))


def coupling_rows(models, xs, links) -> np.ndarray:
    """Row values Pg(child) - Pg(parent), link by link, generator by generator."""
    out = []
    for a, b in links:
        ma, mb = models[a], models[b]
        pa = np.asarray(xs[a])[2 * ma.nb: 2 * ma.nb + ma.ng]
        pb = np.asarray(xs[b])[2 * mb.nb: 2 * mb.nb + mb.ng]
        out.append(pa - pb)
    return np.concatenate(out) if out else np.zeros(0)


def assemble(models, xs, sigmas, lams, links):
    """The coupled problem at the instances' iterates: dict with the global
    x, f (sum of the instances' objectives), c, J and H (scipy CSR)."""
    blocksJ, blocksH, cs, f = [], [], [], 0.0
    for mdl, x, s, lam in zip(models, xs, sigmas, lams):
        fk, _, _ = O.objective(mdl, x)
        f += fk
        ck, _, _, _ = O.constraints(mdl, x)
        cs.append(ck)
        blocksJ.append(O.jacobian_matrix(mdl, x))
        blocksH.append(O.hessian_matrix(mdl, x, s, lam))
    Jc = coupling_matrix(models, links)
    J = sp.vstack([sp.block_diag(blocksJ, format="csr"), Jc], format="csr")
    H = sp.block_diag(blocksH, format="csr")
    c = np.concatenate(cs + [coupling_rows(models, xs, links)])
    return {"x": np.concatenate([np.asarray(x) for x in xs]), "f": f, "c": c, "J": J, "H": H,
            "J_couple": Jc}
