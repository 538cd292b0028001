"""An independent value-only model of the ACOPF constraints for the oracle's
self-tests, written in real arithmetic on rectangular voltages
(e + j f = v exp(j theta)) with torch so that autograd can produce dense
first and second derivatives.  It shares nothing with the oracle beyond the
physical model: a pi-model branch with series admittance 1/(r + j x), charging
b/2 at each end and an ideal transformer of ratio tap*exp(j shift) on the from
side; bus shunts Gs + j Bs; generation subtracted and load added in the
balance rows; squared apparent power in the flow rows.
"""
import torch


def _cm(a, b):
    return (a[0] * b[0] - a[1] * b[1], a[0] * b[1] + a[1] * b[0])


def _cconj(a):
    return (a[0], -a[1])


def _cdiv(a, b):
    den = b[0] * b[0] + b[1] * b[1]
    return ((a[0] * b[0] + a[1] * b[1]) / den, (a[1] * b[0] - a[0] * b[1]) / den)


def _cadd(a, b):
    return (a[0] + b[0], a[1] + b[1])


def _csub(a, b):
    return (a[0] - b[0], a[1] - b[1])


def tensors(grid):
    T = lambda a: torch.as_tensor(a, dtype=torch.float64)
    L = lambda a: torch.as_tensor(a, dtype=torch.long)
    return dict(f=L(grid.br_from), t=L(grid.br_to), r=T(grid.br_r), x=T(grid.br_x),
                b=T(grid.br_b), tap=T(grid.br_tap), sh=T(grid.br_shift),
                pd=T(grid.bus_pd), qd=T(grid.bus_qd), gs=T(grid.bus_gs), bs=T(grid.bus_bs),
                gb=L(grid.gen_bus), c2=T(grid.gen_c2), c1=T(grid.gen_c1), c0=T(grid.gen_c0),
                nb=grid.nbus, ng=len(grid.gen_bus), base=float(grid.base_mva))


def flows(d, x):
    """(P_f, Q_f, P_t, Q_t) per branch, rectangular route."""
    nb = d["nb"]
    th, v = x[:nb], x[nb:2 * nb]
    e, fi = v * torch.cos(th), v * torch.sin(th)
    Vf = (e[d["f"]], fi[d["f"]])
    Vt = (e[d["t"]], fi[d["t"]])
    one = torch.ones_like(d["r"])
    zero = torch.zeros_like(d["r"])
    ys = _cdiv((one, zero), (d["r"], d["x"]))
    N = (d["tap"] * torch.cos(d["sh"]), d["tap"] * torch.sin(d["sh"]))
    half_b = (zero, d["b"] / 2)
    # the from terminal sees V_f / N on the network side of the ideal transformer
    Vf_in = _cdiv(Vf, N)
    Is = _cm(ys, _csub(Vf_in, Vt))               # series current, from -> to
    If_in = _cadd(Is, _cm(half_b, Vf_in))        # current leaving the transformer
    If = _cdiv(If_in, _cconj(N))                 # power-conserving ratio on currents
    It = _cadd(_cm(ys, _csub(Vt, Vf_in)), _cm(half_b, Vt))
    Sf = _cm(Vf, _cconj(If))
    St = _cm(Vt, _cconj(It))
    return Sf[0], Sf[1], St[0], St[1]


def constraints(d, x):
    nb, ng = d["nb"], d["ng"]
    v = x[nb:2 * nb]
    pg, qg = x[2 * nb:2 * nb + ng], x[2 * nb + ng:]
    Pf, Qf, Pt, Qt = flows(d, x)
    P = torch.zeros(nb, dtype=x.dtype).index_add(0, d["f"], Pf).index_add(0, d["t"], Pt)
    Q = torch.zeros(nb, dtype=x.dtype).index_add(0, d["f"], Qf).index_add(0, d["t"], Qt)
    P = P + d["gs"] * v * v
    Q = Q - d["bs"] * v * v
    GP = torch.zeros(nb, dtype=x.dtype).index_add(0, d["gb"], pg)
    GQ = torch.zeros(nb, dtype=x.dtype).index_add(0, d["gb"], qg)
    gP = P - GP + d["pd"]
    gQ = Q - GQ + d["qd"]
    return torch.cat([gP, gQ, Pf * Pf + Qf * Qf, Pt * Pt + Qt * Qt])


def objective(d, x):
    nb, ng = d["nb"], d["ng"]
    p = d["base"] * x[2 * nb:2 * nb + ng]
    return torch.sum(d["c2"] * p * p + d["c1"] * p + d["c0"])


def dense_jacobian(grid, x):
    d = tensors(grid)
    xt = torch.as_tensor(x, dtype=torch.float64)
    return torch.autograd.functional.jacobian(lambda z: constraints(d, z), xt).numpy()


def dense_hessian(grid, x, sigma, lam):
    d = tensors(grid)
    xt = torch.as_tensor(x, dtype=torch.float64)
    lt = torch.as_tensor(lam, dtype=torch.float64)
    L = lambda z: sigma * objective(d, z) + torch.dot(lt, constraints(d, z))
    return torch.autograd.functional.hessian(L, xt).numpy()


def values(grid, x):
    d = tensors(grid)
    xt = torch.as_tensor(x, dtype=torch.float64)
    return constraints(d, xt).numpy(), float(objective(d, xt))
