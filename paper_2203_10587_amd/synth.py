"""Seeded synthetic power grids and interior-point iterates.

This module draws inputs only: bus/branch/generator data and the iterate
(x, lambda, sigma) at which the ACOPF model is evaluated.  It holds none of the
evaluation arithmetic (no admittances, flows or derivatives), so both the
HIP path and the CPU oracle can be fed from it without sharing method code.

The paper (OPFLOW section) states the ACOPF only in compact form and runs its
experiments on the ACTIVSg200/ACTIVSg2000 cases (TCOPFLOW, SCOPFLOW and
SOPFLOW sections), which are not available here.  The grids below are
synthetic stand-ins with the same structure: sparse, planar-like meshes of a
few thousand buses, mean degree about 2.6, a fifth of the branches being
transformers, generators on a quarter of the buses and loads on 70 %.

Conventions (all per unit on a 100 MVA base, angles in radians):
  x      = [theta (nb), v (nb), Pg (ng), Qg (ng)]
  lambda = [balance-P (nb), balance-Q (nb), flow-from (nl), flow-to (nl)]
Random streams come from numpy's PCG64 seeded through SeedSequence; a batch
instance k draws from SeedSequence(seed).spawn(K)[k] so it is the same alone
or inside any batch.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, replace
from typing import List, Optional, Sequence, Tuple

import numpy as np

BASE_MVA = 100.0


@dataclass
class Grid:
    """Structure-of-arrays network description (0-based bus ids)."""

    nbus: int
    br_from: np.ndarray   # int32 [nl]
    br_to: np.ndarray     # int32 [nl]
    br_r: np.ndarray      # f64 [nl] series resistance
    br_x: np.ndarray      # f64 [nl] series reactance
    br_b: np.ndarray      # f64 [nl] total line charging
    br_tap: np.ndarray    # f64 [nl] off-nominal tap ratio (1 for lines)
    br_shift: np.ndarray  # f64 [nl] phase shift, radians
    br_rate: np.ndarray   # f64 [nl] apparent-power limit
    bus_pd: np.ndarray    # f64 [nb]
    bus_qd: np.ndarray
    bus_gs: np.ndarray    # shunt conductance (power at v = 1)
    bus_bs: np.ndarray    # shunt susceptance
    gen_bus: np.ndarray   # int32 [ng]
    gen_c2: np.ndarray    # $/MW^2h
    gen_c1: np.ndarray    # $/MWh
    gen_c0: np.ndarray    # $/h
    gen_pmin: np.ndarray  # bounds, only used to draw iterates
    gen_pmax: np.ndarray
    gen_qmin: np.ndarray
    gen_qmax: np.ndarray
    base_mva: float = BASE_MVA

    @property
    def nbranch(self) -> int:
        return int(self.br_from.shape[0])

    @property
    def ngen(self) -> int:
        return int(self.gen_bus.shape[0])

    @property
    def n(self) -> int:
        return 2 * self.nbus + 2 * self.ngen

    @property
    def m(self) -> int:
        return 2 * self.nbus + 2 * self.nbranch


@dataclass
class Iterate:
    x: np.ndarray       # f64 [n]
    lam: np.ndarray     # f64 [m]
    sigma: float = 1.0


# --------------------------------------------------------------------------
# helpers


def _rng(seed) -> np.random.Generator:
    if isinstance(seed, np.random.SeedSequence):
        return np.random.Generator(np.random.PCG64(seed))
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))


def _children(seed, k: int) -> List[np.random.SeedSequence]:
    ss = seed if isinstance(seed, np.random.SeedSequence) else np.random.SeedSequence(seed)
    return ss.spawn(k)


def remove_branch(g: Grid, l: int) -> Grid:
    """The N-1 network: branch l taken out entirely (its flow rows vanish)."""
    keep = np.ones(g.nbranch, dtype=bool)
    keep[l] = False
    return replace(
        g,
        br_from=g.br_from[keep].copy(), br_to=g.br_to[keep].copy(),
        br_r=g.br_r[keep].copy(), br_x=g.br_x[keep].copy(), br_b=g.br_b[keep].copy(),
        br_tap=g.br_tap[keep].copy(), br_shift=g.br_shift[keep].copy(),
        br_rate=g.br_rate[keep].copy(),
    )


def scale_loads(g: Grid, s: float) -> Grid:
    return replace(g, bus_pd=g.bus_pd * s, bus_qd=g.bus_qd * s)


def _gen_bounds(pd_total: float, ng: int):
    # Pmin = 0, Pmax = 2 * total load / ng, |Q| <= Pmax / 2.
    pmax = 2.0 * pd_total / max(ng, 1)
    return 0.0, pmax, -pmax / 2.0, pmax / 2.0


def draw_iterate(g: Grid, rng: np.random.Generator, sigma: float = 1.0) -> Iterate:
    """v~U(.95,1.05), theta~U(-.2,.2), Pg/Qg uniform in bounds, lambda~N(0,1)."""
    nb, ng = g.nbus, g.ngen
    v = rng.uniform(0.95, 1.05, nb)
    th = rng.uniform(-0.2, 0.2, nb)
    pg = rng.uniform(g.gen_pmin, g.gen_pmax) if ng else np.zeros(0)
    qg = rng.uniform(g.gen_qmin, g.gen_qmax) if ng else np.zeros(0)
    lam = rng.standard_normal(g.m)
    x = np.concatenate([th, v, pg, qg]).astype(np.float64)
    return Iterate(x=x, lam=lam.astype(np.float64), sigma=float(sigma))


def draw_iterate_cartesian(g: Grid, rng: np.random.Generator, sigma: float = 1.0) -> Iterate:
    """Iterate of the cartesian representation x = [e; f; Pg; Qg]:
    e~U(.9,1.1), f~U(-.2,.2), Pg/Qg uniform in bounds, lambda~N(0,1) over
    the m + nbus rows (balance, flow, then magnitude rows)."""
    nb, ng = g.nbus, g.ngen
    e = rng.uniform(0.9, 1.1, nb)
    f = rng.uniform(-0.2, 0.2, nb)
    pg = rng.uniform(g.gen_pmin, g.gen_pmax) if ng else np.zeros(0)
    qg = rng.uniform(g.gen_qmin, g.gen_qmax) if ng else np.zeros(0)
    lam = rng.standard_normal(g.m + nb)
    x = np.concatenate([e, f, pg, qg]).astype(np.float64)
    return Iterate(x=x, lam=lam.astype(np.float64), sigma=float(sigma))


def _branch_params(nl: int, rng: np.random.Generator, n_xfmr: int = 0):
    r = rng.uniform(0.005, 0.05, nl)
    x = rng.uniform(0.05, 0.3, nl)
    b = rng.uniform(0.0, 0.2, nl)
    rate = rng.uniform(1.5, 3.0, nl)
    tap = np.ones(nl)
    shift = np.zeros(nl)
    if n_xfmr:
        idx = rng.choice(nl, n_xfmr, replace=False)
        tap[idx] = rng.uniform(0.95, 1.05, n_xfmr)
    return r, x, b, rate, tap, shift


def _finish(nb, f, t, r, x, b, rate, tap, shift, pd, qd, gen_bus, c2, c1) -> Grid:
    ng = len(gen_bus)
    pmin, pmax, qmin, qmax = _gen_bounds(float(np.sum(pd)), ng)
    return Grid(
        nbus=int(nb),
        br_from=np.asarray(f, dtype=np.int32), br_to=np.asarray(t, dtype=np.int32),
        br_r=np.asarray(r, float), br_x=np.asarray(x, float), br_b=np.asarray(b, float),
        br_tap=np.asarray(tap, float), br_shift=np.asarray(shift, float),
        br_rate=np.asarray(rate, float),
        bus_pd=np.asarray(pd, float), bus_qd=np.asarray(qd, float),
        bus_gs=np.zeros(nb), bus_bs=np.zeros(nb),
        gen_bus=np.asarray(gen_bus, dtype=np.int32),
        gen_c2=np.asarray(c2, float), gen_c1=np.asarray(c1, float), gen_c0=np.zeros(ng),
        gen_pmin=np.full(ng, pmin), gen_pmax=np.full(ng, pmax),
        gen_qmin=np.full(ng, qmin), gen_qmax=np.full(ng, qmax),
    )


# --------------------------------------------------------------------------
# the 9-bus ring


def ring9(seed=0) -> Tuple[Grid, Iterate]:
    """Ring of 9 buses plus 3 random chords (12 branches); generators on
    buses 0..2, loads on buses 3..8."""
    topo, par, it = (_rng(s) for s in _children(seed, 3))
    nb = 9
    edges = [(l, (l + 1) % nb) for l in range(nb)]
    used = {frozenset(e) for e in edges}
    free = [(i, j) for i in range(nb) for j in range(i + 1, nb) if frozenset((i, j)) not in used]
    pick = topo.choice(len(free), 3, replace=False)
    edges += [free[p] for p in pick]
    f = [min(e) for e in edges]
    t = [max(e) for e in edges]
    r, x, b, rate, tap, shift = _branch_params(len(edges), par)
    pd = np.zeros(nb)
    pd[3:] = par.uniform(0.5, 1.5, 6)
    qd = 0.3 * pd
    c2 = par.uniform(0.01, 0.1, 3)
    c1 = par.uniform(10.0, 40.0, 3)
    g = _finish(nb, f, t, r, x, b, rate, tap, shift, pd, qd, [0, 1, 2], c2, c1)
    return g, draw_iterate(g, it)


# --------------------------------------------------------------------------
# random geometric grids


def rgg_edges(nb: int, nl: int, rng: np.random.Generator, k: int = 12) -> np.ndarray:
    """Connected planar-like edge set: Euclidean MST of the k-nearest-neighbour
    graph, then the shortest unused candidate edges up to nl.  Bus ids follow a
    serpentine coarse-cell order, as regional numbering does.  Returns an
    (nl, 2) int array with from < to, sorted by (from, to)."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import minimum_spanning_tree
    from scipy.spatial import cKDTree

    if nl < nb - 1:
        raise ValueError("a connected grid needs nl >= nb - 1")
    pts = rng.random((nb, 2))
    ncell = max(1, int(math.sqrt(nb / 16.0)))
    cx = np.minimum((pts[:, 0] * ncell).astype(np.int64), ncell - 1)
    cy = np.minimum((pts[:, 1] * ncell).astype(np.int64), ncell - 1)
    cxs = np.where(cy % 2 == 0, cx, ncell - 1 - cx)
    order = np.lexsort((pts[:, 0], cxs, cy))
    pts = pts[order]
    while True:
        kk = min(k, nb - 1)
        dist, idx = cKDTree(pts).query(pts, k=kk + 1)
        i = np.repeat(np.arange(nb), kk)
        j = idx[:, 1:].reshape(-1)
        d = dist[:, 1:].reshape(-1)
        a, bb = np.minimum(i, j), np.maximum(i, j)
        key = a.astype(np.int64) * nb + bb
        key, first = np.unique(key, return_index=True)
        a, bb, d = a[first], bb[first], d[first]
        mst = minimum_spanning_tree(coo_matrix((d, (a, bb)), shape=(nb, nb))).tocoo()
        if mst.nnz == nb - 1 or kk == nb - 1:
            break
        k *= 2
    if mst.nnz != nb - 1:
        raise RuntimeError("candidate graph is not connected")
    tree_key = np.minimum(mst.row, mst.col).astype(np.int64) * nb + np.maximum(mst.row, mst.col)
    in_tree = np.isin(key, tree_key)
    extra = np.flatnonzero(~in_tree)
    extra = extra[np.argsort(d[extra], kind="stable")][: nl - (nb - 1)]
    if len(extra) < nl - (nb - 1):
        raise RuntimeError("not enough candidate edges for the requested branch count")
    keys = np.sort(np.concatenate([tree_key, key[extra]]))
    return np.stack([keys // nb, keys % nb], axis=1).astype(np.int64)


def rgg_grid(nb: int, nl: Optional[int] = None, seed=0, gen_frac: float = 0.25,
             load_frac: float = 0.70, xfmr_frac: float = 0.20,
             load_scale: float = 1.0) -> Grid:
    """Random geometric grid with the configured generator/load/transformer
    fractions, impedances r~U(.005,.05), x~U(.05,.3), b~U(0,.2), limits
    U(1.5,3), taps U(.95,1.05) on transformers, quadratic costs
    c2~U(.01,.1), c1~U(10,40), loads Pd~U(.5,1.5), Qd = .3 Pd."""
    nl = int(round(1.3 * nb)) if nl is None else int(nl)
    topo, par = (_rng(s) for s in _children(seed, 2))
    e = rgg_edges(nb, nl, topo)
    r, x, b, rate, tap, shift = _branch_params(nl, par, int(round(xfmr_frac * nl)))
    ng = int(round(gen_frac * nb))
    nload = int(round(load_frac * nb))
    gen_bus = np.sort(par.choice(nb, ng, replace=False))
    load_bus = par.choice(nb, nload, replace=False)
    pd = np.zeros(nb)
    pd[load_bus] = par.uniform(0.5, 1.5, nload) * load_scale
    qd = 0.3 * pd
    c2 = par.uniform(0.01, 0.1, ng)
    c1 = par.uniform(10.0, 40.0, ng)
    return _finish(nb, e[:, 0], e[:, 1], r, x, b, rate, tap, shift, pd, qd, gen_bus, c2, c1)


def bridges(nb: int, f: np.ndarray, t: np.ndarray) -> np.ndarray:
    """Boolean mask of bridge branches (removal disconnects the graph),
    by an iterative depth-first low-link search."""
    nl = len(f)
    adj = [[] for _ in range(nb)]
    for l in range(nl):
        adj[int(f[l])].append((int(t[l]), l))
        adj[int(t[l])].append((int(f[l]), l))
    disc = [-1] * nb
    low = [0] * nb
    is_bridge = np.zeros(nl, dtype=bool)
    timer = 0
    for root in range(nb):
        if disc[root] >= 0:
            continue
        disc[root] = low[root] = timer
        timer += 1
        stack = [(root, -1, iter(adj[root]))]
        while stack:
            u, pl, it = stack[-1]
            advanced = False
            for w, l in it:
                if l == pl:
                    continue
                if disc[w] < 0:
                    disc[w] = low[w] = timer
                    timer += 1
                    stack.append((w, l, iter(adj[w])))
                    advanced = True
                    break
                low[u] = min(low[u], disc[w])
            if not advanced:
                stack.pop()
                if stack:
                    p = stack[-1][0]
                    low[p] = min(low[p], low[u])
                    if low[u] > disc[p]:
                        is_bridge[pl] = True
    return is_bridge


# --------------------------------------------------------------------------
# the five workloads


def grid_10k(seed=0, nb: int = 10_000, nl: int = 13_000):
    """10,000-bus random geometric grid, 13,000 branches, one instance."""
    s_grid, s_it = _children(seed, 2)
    g = rgg_grid(nb, nl, s_grid)
    return g, draw_iterate(g, _rng(s_it))


@dataclass
class OutageSet:
    base: Grid
    outages: np.ndarray          # int32 [K] removed branch per instance
    iterates: List[Iterate]      # per instance, sized for the N-1 network


def n1_security_set(seed=0, nb: int = 2000, nl: int = 3000, count: int = 1000) -> OutageSet:
    """N-1 security set: `count` distinct non-bridge single-branch outages of a
    2,000-bus / 3,000-branch base grid, each with its own iterate."""
    s_grid, s_pick, s_it = _children(seed, 3)
    g = rgg_grid(nb, nl, s_grid)
    cand = np.flatnonzero(~bridges(g.nbus, g.br_from, g.br_to))
    if len(cand) < count:
        raise RuntimeError(f"only {len(cand)} non-bridge branches for {count} outages")
    outs = np.sort(_rng(s_pick).choice(cand, count, replace=False)).astype(np.int32)
    kids = _children(s_it, count)
    its = []
    m_out = 2 * g.nbus + 2 * (g.nbranch - 1)
    for k in range(count):
        rng = _rng(kids[k])
        it = draw_iterate(g, rng)
        # the N-1 network has two fewer flow rows; draw its multipliers afresh
        it.lam = rng.standard_normal(m_out)
        its.append(it)
    return OutageSet(base=g, outages=outs, iterates=its)


def n1_instance(os_: OutageSet, k: int) -> Tuple[Grid, Iterate]:
    return remove_branch(os_.base, int(os_.outages[k])), os_.iterates[k]


def uneven_scenario_sizes(seed=0, count: int = 512, lo: int = 200, hi: int = 25_000) -> np.ndarray:
    rng = _rng(_children(seed, 2)[0])
    return np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), count))).astype(np.int64)


def uneven_scenarios(seed=0, count: int = 512, lo: int = 200, hi: int = 25_000,
            only: Optional[Sequence[int]] = None) -> List[Tuple[int, Grid, Iterate]]:
    """Uneven scenarios: bus counts log-uniform in [lo, hi], branches 1.3x,
    loads scaled per instance by exp(N(0, 0.1^2)).  `only` restricts which
    instance indices are generated (each is independent of the others)."""
    sizes = uneven_scenario_sizes(seed, count, lo, hi)
    kids = _children(_children(seed, 2)[1], count)
    out = []
    for k in (range(count) if only is None else only):
        s_grid, s_scale, s_it = _children(kids[k], 3)
        s = float(np.exp(_rng(s_scale).normal(0.0, 0.1)))
        g = rgg_grid(int(sizes[k]), None, s_grid, load_scale=s)
        out.append((int(k), g, draw_iterate(g, _rng(s_it))))
    return out


SERVE_SIZES = (1_000, 10_000, 30_000, 70_000)


def served_grids(seed=0, sizes: Sequence[int] = SERVE_SIZES) -> List[Grid]:
    """The four resident grids of the served workload."""
    kids = _children(seed, len(sizes))
    return [rgg_grid(int(nb), None, kids[i]) for i, nb in enumerate(sizes)]


# --------------------------------------------------------------------------
# small irregular grids for tests


def random_grid(nb: int, nl: int, ng: int, seed=0, *, shunts: bool = True,
                parallel: int = 1, shifters: bool = True, multigen: bool = True,
                star: bool = False) -> Grid:
    """Irregular test grid: a random spanning tree plus random extra branches,
    `parallel` duplicated branches, nonzero shunts, phase-shifting
    transformers with taps in both directions, several generators per bus and
    random branch orientation.  `star` makes bus 0 adjacent to every bus."""
    rng = _rng(seed)
    edges = []
    if star:
        edges = [(0, j) for j in range(1, nb)]
    else:
        perm = rng.permutation(nb)
        for k in range(1, nb):
            edges.append((int(perm[k]), int(perm[rng.integers(0, k)])))
    have = {frozenset(e) for e in edges}
    tries = 0
    while len(edges) < nl - parallel and tries < 100 * nl:
        tries += 1
        i, j = (int(v) for v in rng.integers(0, nb, 2))
        if i == j or frozenset((i, j)) in have:
            continue
        have.add(frozenset((i, j)))
        edges.append((i, j))
    for _ in range(parallel):
        i, j = edges[int(rng.integers(0, len(edges)))]
        edges.append((j, i) if rng.random() < 0.5 else (i, j))
    edges = [edges[p] for p in rng.permutation(len(edges))]
    edges = [(j, i) if rng.random() < 0.5 else (i, j) for (i, j) in edges]
    nl = len(edges)
    f = np.array([e[0] for e in edges])
    t = np.array([e[1] for e in edges])
    r, x, b, rate, tap, shift = _branch_params(nl, rng, nl // 4)
    if shifters:
        sel = rng.choice(nl, max(1, nl // 5), replace=False)
        shift[sel] = rng.uniform(-0.3, 0.3, len(sel))
        tap[sel] = rng.uniform(0.9, 1.1, len(sel))
    if multigen:
        gen_bus = np.sort(rng.integers(0, nb, ng))
    else:
        gen_bus = np.sort(rng.choice(nb, ng, replace=False))
    pd = rng.uniform(0.0, 1.5, nb)
    qd = rng.uniform(-0.2, 0.5, nb)
    c2 = rng.uniform(0.01, 0.1, ng)
    c1 = rng.uniform(10.0, 40.0, ng)
    g = _finish(nb, f, t, r, x, b, rate, tap, shift, pd, qd, gen_bus, c2, c1)
    if shunts:
        g.bus_gs = rng.uniform(-0.05, 0.1, nb) * (rng.random(nb) < 0.5)
        g.bus_bs = rng.uniform(-0.2, 0.3, nb) * (rng.random(nb) < 0.5)
    g.gen_c0 = rng.uniform(0.0, 100.0, ng)
    return g
