"""FP64 CPU oracle for the power-balance-cartesian representation.

TEST INFRASTRUCTURE: imported only by tests/ (never by the HIP path).

The paper (OPFLOW section) names two representations of the network
equations, power-balance-polar and power-balance-cartesian, and leaves the
formulation to its references.  Reading taken here: the same problem as the
polar oracle (acopf_oracle), with rectangular voltage components
  variables     x = [e (nb), f (nb), Pg (ng), Qg (ng)],  V = e + j f
  objective     as polar (cost on MW)
  equalities    g = [Re S_bus - Cg' Pg + Pd ; Im S_bus - Cg' Qg + Qd]
  inequalities  h = [|S_f|^2 ; |S_t|^2 ; |V|^2]: the magnitude is no longer a
                variable, so its bounds act on a row e_i^2 + f_i^2 (the bounds
                themselves are the solver's)
  lambda        ordered like c = [g ; h]
Patterns: those of the polar representation with (e, f) in the places of
(theta, v), plus the magnitude rows, each (e_i, f_i); the Hessian pattern is
unchanged (the magnitude and shunt terms fall on existing diagonal entries).

Routes: J from complex matrix derivatives of S = V o conj(Y V) with
dV/de = 1, dV/df = j; H by the per-branch complex product rule in the four
local variables (e_f, e_t, f_f, f_t) (V is linear in them, so only the
first-derivative cross terms remain), assembled as a full symmetric matrix.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import acopf_oracle as P


def pattern(mdl):
    """J pattern (int32 rowptr/col) of the cartesian representation: the
    polar rows, then one row (e_i, f_i) per bus; the H pattern of polar."""
    nb = mdl.nb
    jp = np.concatenate([mdl.jac_rowptr, mdl.jac_rowptr[-1] + 2 * np.arange(1, nb + 1)])
    jc = np.concatenate([mdl.jac_col, np.stack([np.arange(nb), nb + np.arange(nb)], 1).ravel()])
    return jp.astype(np.int32), jc.astype(np.int32), mdl.hess_rowptr, mdl.hess_col


def _split(mdl, x):
    nb = mdl.nb
    return x[:nb], x[nb:2 * nb]


def constraints(mdl, x):
    g = mdl.grid
    e, f = _split(mdl, x)
    _, _, pg, qg = P._split(mdl, x)
    V = e + 1j * f
    Sbus = V * np.conj(mdl.Ybus @ V)
    gP = Sbus.real - mdl.Cg.T @ pg + g.bus_pd
    gQ = Sbus.imag - mdl.Cg.T @ qg + g.bus_qd
    Sf = (mdl.Cf @ V) * np.conj(mdl.Yf @ V)
    St = (mdl.Ct @ V) * np.conj(mdl.Yt @ V)
    hf = Sf.real ** 2 + Sf.imag ** 2
    ht = St.real ** 2 + St.imag ** 2
    return np.concatenate([gP, gQ, hf, ht, e * e + f * f]), Sf, St, V


def jacobian_matrix(mdl, x) -> sp.csr_matrix:
    nb, ng, nl = mdl.nb, mdl.ng, mdl.nl
    e, f = _split(mdl, x)
    V = e + 1j * f
    dV = sp.diags(V)
    Ibus = mdl.Ybus @ V
    cI = sp.diags(np.conj(Ibus))
    YbC = mdl.Ybus.conj()
    dSb_de = cI + dV @ YbC
    dSb_df = 1j * cI - 1j * (dV @ YbC)

    def branch_side(C, Y):
        I = Y @ V
        CV = C @ V
        cIb = sp.diags(np.conj(I))
        dCV = sp.diags(CV)
        d_e = cIb @ C + dCV @ Y.conj()
        d_f = 1j * (cIb @ C) - 1j * (dCV @ Y.conj())
        S = CV * np.conj(I)
        Pd, Qd = sp.diags(S.real), sp.diags(S.imag)
        return 2.0 * (Pd @ d_e.real + Qd @ d_e.imag), 2.0 * (Pd @ d_f.real + Qd @ d_f.imag)

    hf_e, hf_f = branch_side(mdl.Cf, mdl.Yf)
    ht_e, ht_f = branch_side(mdl.Ct, mdl.Yt)
    mCgT = -mdl.Cg.T
    Z = lambda r, c: sp.csr_matrix((r, c))
    return sp.bmat([
        [dSb_de.real, dSb_df.real, mCgT, Z(nb, ng)],
        [dSb_de.imag, dSb_df.imag, Z(nb, ng), mCgT],
        [hf_e, hf_f, Z(nl, ng), Z(nl, ng)],
        [ht_e, ht_f, Z(nl, ng), Z(nl, ng)],
        [sp.diags(2.0 * e), sp.diags(2.0 * f), Z(nb, ng), Z(nb, ng)],
    ], format="csr")


def hessian_matrix(mdl, x, sigma, lam, magnitude: bool = False) -> sp.csr_matrix:
    """Full symmetric Hessian of L = sigma f + lambda'c.  With
    magnitude=True, each entry is instead the sum of the absolute values of
    the terms it adds up (its rounding companion)."""
    g = mdl.grid
    nb, nl, ng, n = mdl.nb, mdl.nl, mdl.ng, mdl.n
    e, f_ = _split(mdl, x)
    V = e + 1j * f_
    fb = g.br_from.astype(np.int64)
    tb = g.br_to.astype(np.int64)
    Vf, Vt = V[fb], V[tb]
    # local z = (e_f, e_t, f_f, f_t): constant first derivatives of V_f, V_t
    dVf = np.zeros((nl, 4), complex)
    dVt = np.zeros((nl, 4), complex)
    dVf[:, 0], dVf[:, 2] = 1.0, 1j
    dVt[:, 1], dVt[:, 3] = 1.0, 1j

    def end(Vs, dVs, Ya, Yb):
        I = Ya * Vf + Yb * Vt
        dI = Ya[:, None] * dVf + Yb[:, None] * dVt
        S = Vs * np.conj(I)
        dS = dVs * np.conj(I)[:, None] + Vs[:, None] * np.conj(dI)
        d2S = dVs[:, :, None] * np.conj(dI)[:, None, :] + dVs[:, None, :] * np.conj(dI)[:, :, None]
        return S, dS, d2S

    Sf, dSf, d2Sf = end(Vf, dVf, mdl.Yff, mdl.Yft)
    St, dSt, d2St = end(Vt, dVt, mdl.Ytf, mdl.Ytt)
    lP, lQ = lam[:nb], lam[nb:2 * nb]
    mu_f, mu_t = lam[2 * nb:2 * nb + nl], lam[2 * nb + nl:2 * nb + 2 * nl]
    lV = lam[2 * nb + 2 * nl:]

    def weight(S, dS, d2S, lp, lq, mu):
        Pv, Qv = S.real, S.imag
        dP, dQ = dS.real, dS.imag
        d2P, d2Q = d2S.real, d2S.imag
        if magnitude:
            a = np.abs
            return (a(lp)[:, None, None] * a(d2P) + a(lq)[:, None, None] * a(d2Q)
                    + 2.0 * a(mu)[:, None, None] * (a(dP[:, :, None] * dP[:, None, :])
                                                    + a(dQ[:, :, None] * dQ[:, None, :])
                                                    + a(Pv)[:, None, None] * a(d2P)
                                                    + a(Qv)[:, None, None] * a(d2Q)))
        Hb = lp[:, None, None] * d2P + lq[:, None, None] * d2Q
        Hh = 2.0 * (dP[:, :, None] * dP[:, None, :] + dQ[:, :, None] * dQ[:, None, :]
                    + Pv[:, None, None] * d2P + Qv[:, None, None] * d2Q)
        return Hb + mu[:, None, None] * Hh

    Hl = weight(Sf, dSf, d2Sf, lP[fb], lQ[fb], mu_f) + weight(St, dSt, d2St, lP[tb], lQ[tb], mu_t)
    idx = np.stack([fb, tb, nb + fb, nb + tb], axis=1)
    rows = np.repeat(idx, 4, axis=1).reshape(-1)
    cols = np.tile(idx, (1, 4)).reshape(-1)
    vals = Hl.reshape(-1)
    # shunts (P += Gs |V|^2, Q -= Bs |V|^2) and the magnitude rows, on the
    # (e_i, e_i) and (f_i, f_i) diagonals
    d = 2.0 * (lP * g.bus_gs - lQ * g.bus_bs) + 2.0 * lV
    B = g.base_mva
    cost = sigma * 2.0 * g.gen_c2 * B * B
    if magnitude:
        d = 2.0 * (np.abs(lP * g.bus_gs) + np.abs(lQ * g.bus_bs)) + 2.0 * np.abs(lV)
        cost = np.abs(cost)
    ar = np.arange(nb)
    rows = np.concatenate([rows, ar, nb + ar, 2 * nb + np.arange(ng)])
    cols = np.concatenate([cols, ar, nb + ar, 2 * nb + np.arange(ng)])
    vals = np.concatenate([vals, d, d, cost])
    return sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()


def evaluate(mdl, x, sigma=1.0, lam=None):
    """f, grad_f, c, jac_val (cartesian pattern), hess_val (if lam)."""
    jp, jc, hp, hc = pattern(mdl)
    fval, grad, _ = P.objective(mdl, x)
    c, _, _, _ = constraints(mdl, x)
    out = {"f": fval, "grad_f": grad, "c": c,
           "jac_val": P._values_at(jacobian_matrix(mdl, x), jp, jc)}
    if lam is not None:
        H = hessian_matrix(mdl, x, sigma, lam)
        asym = abs(H - H.T).max() if H.nnz else 0.0
        if asym > 1e-14 * max(abs(H).max() if H.nnz else 1.0, 1.0):
            raise AssertionError(f"Hessian not symmetric: {asym}")
        out["hess_val"] = P._values_at(H, hp, hc)
    return out


def vjp(mdl, x, w_f, w_c):
    _, grad, _ = P.objective(mdl, x)
    return w_f * grad + jacobian_matrix(mdl, x).T @ w_c


def _companions(mdl, x):
    """Companions of the branch flows in the magnitudes |V| (as in polar,
    with the transfer terms counted by both rectangular products)."""
    g = mdl.grid
    e, f = _split(mdl, x)
    v = np.hypot(e, f)
    vf, vt = v[g.br_from], v[g.br_to]
    af = np.abs(mdl.Yff) * vf * vf + 2 * np.abs(mdl.Yft) * vf * vt
    at = np.abs(mdl.Ytt) * vt * vt + 2 * np.abs(mdl.Ytf) * vf * vt
    df = 2 * np.abs(mdl.Yff) * vf + 2 * np.abs(mdl.Yft) * (vf + vt)
    dt = 2 * np.abs(mdl.Ytt) * vt + 2 * np.abs(mdl.Ytf) * (vf + vt)
    return v, af, at, df, dt


def scales(mdl, x, out, sigma=None, lam=None):
    """Per-entry scales of the parity rule, as for polar: balance rows by the
    absolute products they sum, flow rows h + 2(|P|+|Q|) a + eps a^2,
    magnitude rows their value, J and H rows by their largest entry (J flow
    rows add 2 a d); given sigma and lambda, an H entry's scale is at least
    the sum of the absolute values of its terms."""
    g = mdl.grid
    nb, nl = mdl.nb, mdl.nl
    c, Sf, St, _ = constraints(mdl, x)
    v, af, at, df, dt = _companions(mdl, x)
    _, _, pg, qg = P._split(mdl, x)
    base = mdl.Cf.T @ af + mdl.Ct.T @ at
    sP = base + np.abs(g.bus_gs) * v * v + mdl.Cg.T @ np.abs(pg) + np.abs(g.bus_pd)
    sQ = base + np.abs(g.bus_bs) * v * v + mdl.Cg.T @ np.abs(qg) + np.abs(g.bus_qd)
    eps = np.finfo(float).eps
    hf = c[2 * nb:2 * nb + nl] + 2 * (np.abs(Sf.real) + np.abs(Sf.imag)) * af + eps * af * af
    ht = c[2 * nb + nl:2 * nb + 2 * nl] + 2 * (np.abs(St.real) + np.abs(St.imag)) * at + eps * at * at
    jp, _, hp, _ = pattern(mdl)
    sj = P._row_absmax(jp, out["jac_val"])
    extra = np.zeros(len(jp) - 1)
    extra[2 * nb:2 * nb + nl] = 2 * af * df
    extra[2 * nb + nl:2 * nb + 2 * nl] = 2 * at * dt
    s = {"f": P.objective(mdl, x)[2], "grad_f": np.abs(out["grad_f"]),
         "c": np.concatenate([sP, sQ, hf, ht, v * v]),
         "jac_val": sj + np.repeat(extra, np.diff(jp))}
    if "hess_val" in out:
        s["hess_val"] = P._row_absmax(hp, out["hess_val"])
        if lam is not None:
            Hm = hessian_matrix(mdl, x, sigma, lam, magnitude=True)
            s["hess_val"] = np.maximum(s["hess_val"], P._values_at(Hm, hp, mdl.hess_col))
    return s


def vjp_scale(mdl, x, w_f, w_c):
    _, grad, _ = P.objective(mdl, x)
    jp, jc, _, _ = pattern(mdl)
    jv = P._values_at(jacobian_matrix(mdl, x), jp, jc)
    sj = scales(mdl, x, {"jac_val": jv, "grad_f": grad})["jac_val"]
    rows = np.repeat(np.arange(len(jp) - 1), np.diff(jp))
    Sj = sp.csr_matrix((sj, (rows, jc)), shape=(len(jp) - 1, mdl.n))
    return abs(w_f) * np.abs(grad) + Sj.T @ np.abs(w_c)
