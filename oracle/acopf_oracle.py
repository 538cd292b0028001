"""FP64 CPU oracle for the polar ACOPF model evaluation.

TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import or run this module.  It shares no
code with the HIP path and must never be used to produce product results.

What it computes (OPFLOW section: the compact problem min f(x) s.t. g(x) = 0,
h- <= h(x) <= h+, x- <= x <= x+, in the power-balance-polar representation).
The paper leaves the ACOPF formulation to its references; the reading taken
here is the standard polar pi-model formulation in per unit:

  variables     x = [theta (nb), v (nb), Pg (ng), Qg (ng)]
  objective     f = sum_k c2_k (B Pg_k)^2 + c1_k (B Pg_k) + c0_k,  B = base MVA
  equalities    g = [Re S_bus - Cg' Pg + Pd ;  Im S_bus - Cg' Qg + Qd]
                S_bus = V o conj(Y_bus V),  V = v o exp(j theta)
                (bus shunts Gs + j Bs sit on the diagonal of Y_bus)
  inequalities  h = [|S_f|^2 ; |S_t|^2],  S_f = (C_f V) o conj(Y_f V), likewise t
  Lagrangian    L = sigma f + lambda' [g ; h]
  outputs       f, grad f, c = [g ; h], J = dc/dx on the fixed pattern,
                lower triangle of the Lagrangian Hessian on its fixed pattern,
                VJP u = w_f grad f + J' w_c.

Branch model: series admittance y_s = 1/(r + j x), total charging b split in
halves at both ends, and an ideal transformer of complex ratio
N = tap exp(j shift) on the from side, so that
  I_f = (y_s + j b/2)/tap^2 V_f - y_s/conj(N) V_t
  I_t = -y_s/N V_f + (y_s + j b/2) V_t.

Routes: values and first derivatives come from the complex bus-injection form
(matrix derivatives of V o conj(Y V) by the product rule); the Hessian is the
per-branch complex product rule applied to S = V conj(I) in the four local
variables (theta_f, theta_t, v_f, v_t), assembled as a full symmetric matrix,
checked for symmetry and only then cut to its lower triangle.

Sparsity patterns follow a purely structural rule (never numeric; explicit
zeros are kept, parallel branches share a slot):
  J row g^P_i : theta_j, v_j for j in {i} u N(i) ascending, then Pg_k at bus i
  J row g^Q_i : the same with Qg
  J flow rows : theta_f, theta_t, v_f, v_t in ascending column order
  H row theta_i : theta_j, j <= i, j in {i} u N(i)
  H row v_i     : theta_j for all j in {i} u N(i), then v_j for j <= i
  H row Pg_k    : Pg_k (diagonal);  H rows Qg_k are empty.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


# ---------------------------------------------------------------------------
# network preparation (not part of the timed evaluation)


def branch_admittances(grid):
    """Per-branch (Y_ff, Y_ft, Y_tf, Y_tt) of the pi model with a from-side
    ideal transformer (see the module docstring)."""
    ys = 1.0 / (grid.br_r + 1j * grid.br_x)
    N = grid.br_tap * np.exp(1j * grid.br_shift)
    ysh = 1j * grid.br_b / 2.0
    Yff = (ys + ysh) / (grid.br_tap ** 2)
    Yft = -ys / np.conj(N)
    Ytf = -ys / N
    Ytt = ys + ysh
    return Yff, Yft, Ytf, Ytt


@dataclass
class Model:
    grid: object
    nb: int
    nl: int
    ng: int
    n: int
    m: int
    Yff: np.ndarray
    Yft: np.ndarray
    Ytf: np.ndarray
    Ytt: np.ndarray
    Cf: sp.csr_matrix
    Ct: sp.csr_matrix
    Cg: sp.csr_matrix      # ng x nb
    Yf: sp.csr_matrix
    Yt: sp.csr_matrix
    Ybus: sp.csr_matrix
    jac_rowptr: np.ndarray
    jac_col: np.ndarray
    hess_rowptr: np.ndarray
    hess_col: np.ndarray


def pattern(grid):
    """CSR patterns (int32 rowptr/col) of J and of the lower Hessian, built
    from the structural rule in the module docstring."""
    nb, nl, ng = grid.nbus, len(grid.br_from), len(grid.gen_bus)
    nbr = [set() for _ in range(nb)]
    for l in range(nl):
        a, b = int(grid.br_from[l]), int(grid.br_to[l])
        nbr[a].add(b)
        nbr[b].add(a)
    gens_at = [[] for _ in range(nb)]
    for k in range(ng):
        gens_at[int(grid.gen_bus[k])].append(k)
    th = lambda j: j
    vv = lambda j: nb + j
    pg = lambda k: 2 * nb + k
    qg = lambda k: 2 * nb + ng + k

    jrows = []
    for block in ("P", "Q"):
        for i in range(nb):
            s = sorted(nbr[i] | {i})
            cols = [th(j) for j in s] + [vv(j) for j in s]
            cols += [pg(k) if block == "P" else qg(k) for k in sorted(gens_at[i])]
            jrows.append(cols)
    for _side in ("f", "t"):
        for l in range(nl):
            a, b = sorted((int(grid.br_from[l]), int(grid.br_to[l])))
            jrows.append([th(a), th(b), vv(a), vv(b)])

    hrows = []
    for i in range(nb):
        s = sorted(nbr[i] | {i})
        hrows.append([th(j) for j in s if j <= i])
    for i in range(nb):
        s = sorted(nbr[i] | {i})
        hrows.append([th(j) for j in s] + [vv(j) for j in s if j <= i])
    for k in range(ng):
        hrows.append([pg(k)])
    for k in range(ng):
        hrows.append([])

    def csr(rows):
        ptr = np.zeros(len(rows) + 1, dtype=np.int64)
        ptr[1:] = np.cumsum([len(r) for r in rows])
        col = np.fromiter((c for r in rows for c in r), dtype=np.int64, count=int(ptr[-1]))
        return ptr.astype(np.int32), col.astype(np.int32)

    jp, jc = csr(jrows)
    hp, hc = csr(hrows)
    return jp, jc, hp, hc


def prepare(grid) -> Model:
    """Admittance matrices, incidence matrices and patterns for a grid."""
    nb, nl, ng = grid.nbus, len(grid.br_from), len(grid.gen_bus)
    Yff, Yft, Ytf, Ytt = branch_admittances(grid)
    rows = np.arange(nl)
    Cf = sp.csr_matrix((np.ones(nl), (rows, grid.br_from)), shape=(nl, nb))
    Ct = sp.csr_matrix((np.ones(nl), (rows, grid.br_to)), shape=(nl, nb))
    Cg = sp.csr_matrix((np.ones(ng), (np.arange(ng), grid.gen_bus)), shape=(ng, nb))
    Yf = sp.diags(Yff) @ Cf + sp.diags(Yft) @ Ct
    Yt = sp.diags(Ytf) @ Cf + sp.diags(Ytt) @ Ct
    Ybus = (Cf.T @ Yf + Ct.T @ Yt + sp.diags(grid.bus_gs + 1j * grid.bus_bs)).tocsr()
    jp, jc, hp, hc = pattern(grid)
    return Model(grid=grid, nb=nb, nl=nl, ng=ng, n=2 * nb + 2 * ng, m=2 * nb + 2 * nl,
                 Yff=Yff, Yft=Yft, Ytf=Ytf, Ytt=Ytt, Cf=Cf.tocsr(), Ct=Ct.tocsr(),
                 Cg=Cg.tocsr(), Yf=Yf.tocsr(), Yt=Yt.tocsr(), Ybus=Ybus,
                 jac_rowptr=jp, jac_col=jc, hess_rowptr=hp, hess_col=hc)


# ---------------------------------------------------------------------------
# evaluation


def _split(mdl: Model, x):
    nb, ng = mdl.nb, mdl.ng
    th, v = x[:nb], x[nb:2 * nb]
    pg, qg = x[2 * nb:2 * nb + ng], x[2 * nb + ng:]
    return th, v, pg, qg


def objective(mdl: Model, x):
    """f and grad f of the quadratic cost on MW (B = base MVA)."""
    g = mdl.grid
    B = g.base_mva
    _, _, pg, _ = _split(mdl, x)
    terms = g.gen_c2 * (B * pg) ** 2 + g.gen_c1 * (B * pg) + g.gen_c0
    grad = np.zeros(mdl.n)
    grad[2 * mdl.nb:2 * mdl.nb + mdl.ng] = 2.0 * g.gen_c2 * B * B * pg + g.gen_c1 * B
    return float(np.sum(terms)), grad, float(np.sum(np.abs(terms)))


def constraints(mdl: Model, x):
    """c = [g^P; g^Q; h^f; h^t] and the flows used to build it."""
    g = mdl.grid
    th, v, pg, qg = _split(mdl, x)
    V = v * np.exp(1j * th)
    Sbus = V * np.conj(mdl.Ybus @ V)
    gen_p = mdl.Cg.T @ pg
    gen_q = mdl.Cg.T @ qg
    gP = Sbus.real - gen_p + g.bus_pd
    gQ = Sbus.imag - gen_q + g.bus_qd
    Sf = (mdl.Cf @ V) * np.conj(mdl.Yf @ V)
    St = (mdl.Ct @ V) * np.conj(mdl.Yt @ V)
    hf = Sf.real ** 2 + Sf.imag ** 2
    ht = St.real ** 2 + St.imag ** 2
    return np.concatenate([gP, gQ, hf, ht]), Sf, St, V


def _branch_companions(mdl: Model, x):
    """Absolute companions of the branch flows: a = |Y_self| v_e^2 +
    |Y_transfer| v_f v_t bounds the size of the products that S_e is summed
    from (they cancel to a much smaller |S_e| on short lines); d bounds the
    products in its first derivatives."""
    th, v, _, _ = _split(mdl, x)
    g = mdl.grid
    vf, vt = v[g.br_from], v[g.br_to]
    af = np.abs(mdl.Yff) * vf * vf + np.abs(mdl.Yft) * vf * vt
    at = np.abs(mdl.Ytt) * vt * vt + np.abs(mdl.Ytf) * vf * vt
    df = 2 * np.abs(mdl.Yff) * vf + np.abs(mdl.Yft) * (vf + vt + vf * vt)
    dt = 2 * np.abs(mdl.Ytt) * vt + np.abs(mdl.Ytf) * (vf + vt + vf * vt)
    return af, at, df, dt


def constraint_scales(mdl: Model, x):
    """Absolute-sum companion of each constraint row.  Balance row: the sum of
    |products| the row is built from (branch terms, shunt, generation, load).
    Flow row h = P^2 + Q^2: h + 2 (|P| + |Q|) a + eps a^2, its first-order
    sensitivity to rounding in P and Q."""
    g = mdl.grid
    c, Sf, St, V = constraints(mdl, x)
    v = np.abs(V)
    _, _, pg, qg = _split(mdl, x)
    af, at, _, _ = _branch_companions(mdl, x)
    base = mdl.Cf.T @ af + mdl.Ct.T @ at
    sP = base + np.abs(g.bus_gs) * v * v + mdl.Cg.T @ np.abs(pg) + np.abs(g.bus_pd)
    sQ = base + np.abs(g.bus_bs) * v * v + mdl.Cg.T @ np.abs(qg) + np.abs(g.bus_qd)
    eps = np.finfo(float).eps
    hf = c[2 * mdl.nb:2 * mdl.nb + mdl.nl] + 2 * (np.abs(Sf.real) + np.abs(Sf.imag)) * af + eps * af * af
    ht = c[2 * mdl.nb + mdl.nl:] + 2 * (np.abs(St.real) + np.abs(St.imag)) * at + eps * at * at
    return np.concatenate([sP, sQ, hf, ht])


def jacobian_row_scales(mdl: Model, x, jac_val):
    """Per-entry scale of J values: the row's max |entry|; flow rows add
    2 a d, the companion of 2 (P dP + Q dQ) when |S| is much below a."""
    s = _row_absmax(mdl.jac_rowptr, jac_val)
    af, at, df, dt = _branch_companions(mdl, x)
    nb, nl = mdl.nb, mdl.nl
    extra = np.zeros(mdl.m)
    extra[2 * nb:2 * nb + nl] = 2 * af * df
    extra[2 * nb + nl:] = 2 * at * dt
    return s + np.repeat(extra, np.diff(mdl.jac_rowptr))


def jacobian_matrix(mdl: Model, x) -> sp.csr_matrix:
    """dc/dx as a sparse matrix, from complex matrix derivatives of
    S = V o conj(Y V) (product rule; dV/dtheta = j diag(V), dV/dv = diag(E),
    E = exp(j theta))."""
    th, v, pg, qg = _split(mdl, x)
    nb, ng = mdl.nb, mdl.ng
    V = v * np.exp(1j * th)
    E = np.exp(1j * th)
    dV = sp.diags(V)
    dE = sp.diags(E)
    Ibus = mdl.Ybus @ V
    dSb_dth = 1j * dV @ (sp.diags(np.conj(Ibus)) - (mdl.Ybus @ dV).conj())
    dSb_dv = dV @ (mdl.Ybus @ dE).conj() + sp.diags(np.conj(Ibus)) @ dE

    def branch_side(C, Y):
        I = Y @ V
        CV = C @ V
        d_th = sp.diags(np.conj(I)) @ C @ (1j * dV) + sp.diags(CV) @ (Y @ (1j * dV)).conj()
        d_v = sp.diags(np.conj(I)) @ C @ dE + sp.diags(CV) @ (Y @ dE).conj()
        S = CV * np.conj(I)
        P, Q = sp.diags(S.real), sp.diags(S.imag)
        dh_th = 2.0 * (P @ d_th.real + Q @ d_th.imag)
        dh_v = 2.0 * (P @ d_v.real + Q @ d_v.imag)
        return dh_th, dh_v

    hf_th, hf_v = branch_side(mdl.Cf, mdl.Yf)
    ht_th, ht_v = branch_side(mdl.Ct, mdl.Yt)
    mCgT = -mdl.Cg.T
    Z = lambda r, c: sp.csr_matrix((r, c))
    nl = mdl.nl
    J = sp.bmat([
        [dSb_dth.real, dSb_dv.real, mCgT, Z(nb, ng)],
        [dSb_dth.imag, dSb_dv.imag, Z(nb, ng), mCgT],
        [hf_th, hf_v, Z(nl, ng), Z(nl, ng)],
        [ht_th, ht_v, Z(nl, ng), Z(nl, ng)],
    ], format="csr")
    return J


def _branch_local_hessians(mdl: Model, x, lam, magnitude: bool = False):
    """Per branch, the 4x4 Hessian of its share of lambda'c in the local
    variables z = (theta_f, theta_t, v_f, v_t), by the complex product rule
    on S_f = V_f conj(I_f), S_t = V_t conj(I_t).  With magnitude=True, the
    same sum with every term replaced by its absolute value (the companion
    of the parity rule's Hessian scale)."""
    g = mdl.grid
    nb, nl = mdl.nb, mdl.nl
    th, v, _, _ = _split(mdl, x)
    f = g.br_from.astype(np.int64)
    t = g.br_to.astype(np.int64)
    Ef, Et = np.exp(1j * th[f]), np.exp(1j * th[t])
    Vf, Vt = v[f] * Ef, v[t] * Et
    # first derivatives of V_f, V_t w.r.t. z: shape (nl, 4)
    dVf = np.zeros((nl, 4), complex)
    dVt = np.zeros((nl, 4), complex)
    dVf[:, 0] = 1j * Vf
    dVf[:, 2] = Ef
    dVt[:, 1] = 1j * Vt
    dVt[:, 3] = Et
    # second derivatives: shape (nl, 4, 4)
    d2Vf = np.zeros((nl, 4, 4), complex)
    d2Vt = np.zeros((nl, 4, 4), complex)
    d2Vf[:, 0, 0] = -Vf
    d2Vf[:, 0, 2] = d2Vf[:, 2, 0] = 1j * Ef
    d2Vt[:, 1, 1] = -Vt
    d2Vt[:, 1, 3] = d2Vt[:, 3, 1] = 1j * Et

    def end(Vs, dVs, d2Vs, Ya, Yb):
        # S = Vs conj(I), I = Ya V_f + Yb V_t
        I = Ya * Vf + Yb * Vt
        dI = Ya[:, None] * dVf + Yb[:, None] * dVt
        d2I = Ya[:, None, None] * d2Vf + Yb[:, None, None] * d2Vt
        S = Vs * np.conj(I)
        dS = dVs * np.conj(I)[:, None] + Vs[:, None] * np.conj(dI)
        d2S = (d2Vs * np.conj(I)[:, None, None]
               + dVs[:, :, None] * np.conj(dI)[:, None, :]
               + dVs[:, None, :] * np.conj(dI)[:, :, None]
               + Vs[:, None, None] * np.conj(d2I))
        return S, dS, d2S

    Sf, dSf, d2Sf = end(Vf, dVf, d2Vf, mdl.Yff, mdl.Yft)
    St, dSt, d2St = end(Vt, dVt, d2Vt, mdl.Ytf, mdl.Ytt)
    lP, lQ = lam[:nb], lam[nb:2 * nb]
    mu_f, mu_t = lam[2 * nb:2 * nb + nl], lam[2 * nb + nl:]

    def weight(S, dS, d2S, lp, lq, mu):
        P, Q = S.real, S.imag
        dP, dQ = dS.real, dS.imag
        d2P, d2Q = d2S.real, d2S.imag
        if magnitude:
            a = np.abs
            return (a(lp)[:, None, None] * a(d2P) + a(lq)[:, None, None] * a(d2Q)
                    + 2.0 * a(mu)[:, None, None] * (a(dP[:, :, None] * dP[:, None, :])
                                                    + a(dQ[:, :, None] * dQ[:, None, :])
                                                    + a(P)[:, None, None] * a(d2P)
                                                    + a(Q)[:, None, None] * a(d2Q)))
        Hb = lp[:, None, None] * d2P + lq[:, None, None] * d2Q
        # mu * Hessian of (P^2 + Q^2)
        Hh = 2.0 * (dP[:, :, None] * dP[:, None, :] + dQ[:, :, None] * dQ[:, None, :]
                    + P[:, None, None] * d2P + Q[:, None, None] * d2Q)
        return Hb + mu[:, None, None] * Hh

    H = weight(Sf, dSf, d2Sf, lP[f], lQ[f], mu_f) + weight(St, dSt, d2St, lP[t], lQ[t], mu_t)
    idx = np.stack([f, t, nb + f, nb + t], axis=1)
    return H, idx


def hessian_matrix(mdl: Model, x, sigma, lam, magnitude: bool = False) -> sp.csr_matrix:
    """Full symmetric Hessian of L = sigma f + lambda'c (sparse).  With
    magnitude=True, each entry is instead the sum of the absolute values of
    the terms it adds up (its rounding companion)."""
    g = mdl.grid
    nb, ng, n = mdl.nb, mdl.ng, mdl.n
    Hl, idx = _branch_local_hessians(mdl, x, lam, magnitude)
    rows = np.repeat(idx, 4, axis=1).reshape(-1)
    cols = np.tile(idx, (1, 4)).reshape(-1)
    vals = Hl.reshape(-1)
    # bus shunts: lambda_P Gs v^2 - lambda_Q Bs v^2
    if magnitude:
        sh = 2.0 * (np.abs(lam[:nb] * g.bus_gs) + np.abs(lam[nb:2 * nb] * g.bus_bs))
    else:
        sh = 2.0 * (lam[:nb] * g.bus_gs - lam[nb:2 * nb] * g.bus_bs)
    # cost: sigma * 2 c2 B^2 on (Pg_k, Pg_k)
    B = g.base_mva
    cost = sigma * 2.0 * g.gen_c2 * B * B
    if magnitude:
        cost = np.abs(cost)
    rows = np.concatenate([rows, nb + np.arange(nb), 2 * nb + np.arange(ng)])
    cols = np.concatenate([cols, nb + np.arange(nb), 2 * nb + np.arange(ng)])
    vals = np.concatenate([vals, sh, cost])
    return sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()


def _values_at(M: sp.spmatrix, rowptr, col):
    """Entries of sparse M at the CSR coordinates (rowptr, col); coordinates
    M does not store read as 0."""
    M = M.tocoo()
    M.sum_duplicates()
    ncol = M.shape[1]
    key = M.row.astype(np.int64) * ncol + M.col
    order = np.argsort(key)
    key, data = key[order], M.data[order]
    rows = np.repeat(np.arange(len(rowptr) - 1, dtype=np.int64), np.diff(rowptr))
    want = rows * ncol + col.astype(np.int64)
    pos = np.searchsorted(key, want)
    pos_c = np.minimum(pos, max(len(key) - 1, 0))
    hit = (pos < len(key)) & (key[pos_c] == want) if len(key) else np.zeros(len(want), bool)
    out = np.zeros(len(want))
    out[hit] = data[pos_c[hit]]
    return out


def _row_absmax(rowptr, vals):
    a = np.abs(vals)
    out = np.zeros(len(rowptr) - 1)
    nz = np.diff(rowptr) > 0
    out[nz] = np.maximum.reduceat(a, rowptr[:-1][nz])
    return np.repeat(out, np.diff(rowptr))


def evaluate(mdl: Model, x, sigma=1.0, lam=None, hess_check: bool = True):
    """Full evaluation: dict with f, grad_f, c, jac_val, hess_val (values on
    the model's patterns)."""
    f, grad, _ = objective(mdl, x)
    c, _, _, _ = constraints(mdl, x)
    J = jacobian_matrix(mdl, x)
    out = {"f": f, "grad_f": grad, "c": c,
           "jac_val": _values_at(J, mdl.jac_rowptr, mdl.jac_col)}
    if lam is not None:
        H = hessian_matrix(mdl, x, sigma, lam)
        if hess_check:
            asym = abs(H - H.T).max() if H.nnz else 0.0
            scale = abs(H).max() if H.nnz else 1.0
            if asym > 1e-14 * max(scale, 1.0):
                raise AssertionError(f"Hessian not symmetric: {asym} vs scale {scale}")
        out["hess_val"] = _values_at(H, mdl.hess_rowptr, mdl.hess_col)
    return out


def vjp(mdl: Model, x, w_f, w_c):
    """u = w_f grad f + J' w_c (plain definition through the sparse J)."""
    _, grad, _ = objective(mdl, x)
    J = jacobian_matrix(mdl, x)
    return w_f * grad + J.T @ w_c


def vjp_scale(mdl: Model, x, w_f, w_c):
    """Companion |w_f| |grad f| + sum_r |w_r| s_r over the rows r that touch
    each column, with s_r the Jacobian row scale."""
    _, grad, _ = objective(mdl, x)
    J = jacobian_matrix(mdl, x)
    jv = _values_at(J, mdl.jac_rowptr, mdl.jac_col)
    sj = jacobian_row_scales(mdl, x, jv)
    rows = np.repeat(np.arange(mdl.m), np.diff(mdl.jac_rowptr))
    Sj = sp.csr_matrix((sj, (rows, mdl.jac_col)), shape=(mdl.m, mdl.n))
    return abs(w_f) * np.abs(grad) + Sj.T @ np.abs(w_c)


def scales(mdl: Model, x, out, sigma=None, lam=None):
    """Per-entry scales for the row-scaled relative parity rule:
    |gpu - oracle| <= tol * max(|oracle|, scale).  A Hessian entry's scale is
    its row's largest |entry| and, given the sigma and lambda it was
    evaluated with, at least the sum of the absolute values of the terms it
    adds up: an entry whose terms cancel is rounded relative to the terms."""
    _, _, fs = objective(mdl, x)
    s = {"f": fs, "c": constraint_scales(mdl, x), "grad_f": np.abs(out["grad_f"]),
         "jac_val": jacobian_row_scales(mdl, x, out["jac_val"])}
    if "hess_val" in out:
        s["hess_val"] = _row_absmax(mdl.hess_rowptr, out["hess_val"])
        if lam is not None:
            Hm = hessian_matrix(mdl, x, sigma, lam, magnitude=True)
            s["hess_val"] = np.maximum(s["hess_val"],
                                       _values_at(Hm, mdl.hess_rowptr, mdl.hess_col))
    return s
