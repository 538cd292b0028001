"""The coupled problem of a batch: per-instance blocks plus coupling rows.

A batch evaluates K independent instances into packed buffers; a coupling
(acopf_couple_create) adds rows Pg(child) - Pg(parent) for each link (paper:
SCOPFLOW, TCOPFLOW and SOPFLOW sections, the coupling constraints that join
subproblems into one block-structured problem).  A solver that treats the
whole thing as one NLP (the monolithic path) needs its global sparsity:

    x = packed x,
    c = [c_0; ...; c_{K-1}; coupling rows]   (packed c, then the rows),
    J = [blockdiag(J_k); J_couple],           values: packed J values, then
                                              acopf_couple_eval's values,
    H = blockdiag(H_k)                        (the rows are linear).

`global_pattern` returns those CSR patterns (host, int64); its value order
is exactly the concatenation above, so the device buffers need no
reordering.
"""
from __future__ import annotations

from typing import Tuple

import numpy as np

from . import acopf as A


def global_pattern(batch: "A.Batch", cp: "A.Couple" = None) -> Tuple[np.ndarray, ...]:
    """(jac_rowptr, jac_col, hess_rowptr, hess_col) of the coupled problem."""
    jrp, jcl, hrp, hcl = [np.zeros(1, np.int64)], [], [np.zeros(1, np.int64)], []
    jbase = hbase = 0
    for k, net in enumerate(batch.nets):
        jp, jc, hp, hc = A.acopf_pattern(net)
        xo = int(batch.x_off[k])
        jrp.append(jp[1:].astype(np.int64) + jbase)
        jcl.append(jc.astype(np.int64) + xo)
        hrp.append(hp[1:].astype(np.int64) + hbase)
        hcl.append(hc.astype(np.int64) + xo)
        jbase += int(jp[-1])
        hbase += int(hp[-1])
    if cp is not None and cp.rows:
        rp, col = A.acopf_couple_pattern(cp)
        jrp.append(rp[1:] + jbase)
        jcl.append(col)
    return (np.concatenate(jrp), np.concatenate(jcl) if jcl else np.zeros(0, np.int64),
            np.concatenate(hrp), np.concatenate(hcl) if hcl else np.zeros(0, np.int64))
