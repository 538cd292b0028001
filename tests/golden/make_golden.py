"""Writes ring9_seed0.json: the oracle's outputs on the seeded 9-bus ring.

Calls only the CPU oracle and the seeded input generator.  The paper prints no
worked example for the model evaluation, so this file is a frozen regression
pin of the oracle itself (it catches later unintended changes), not an
external truth; the external pins are the closed forms, invariants, finite
differences and the independent autograd model in tests/test_oracle.py.

    python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
from paper_2203_10587_amd import synth as S  # noqa: E402


def main():
    g, it = S.ring9(0)
    mdl = O.prepare(g)
    out = O.evaluate(mdl, it.x, it.sigma, it.lam)
    doc = {
        "what": "oracle outputs, 9-bus ring seed 0 (frozen regression pin)",
        "x": it.x.tolist(), "lam": it.lam.tolist(), "sigma": it.sigma,
        "f": out["f"], "grad_f": out["grad_f"].tolist(), "c": out["c"].tolist(),
        "jac_val": out["jac_val"].tolist(), "hess_val": out["hess_val"].tolist(),
        "jac_rowptr": mdl.jac_rowptr.tolist(), "jac_col": mdl.jac_col.tolist(),
        "hess_rowptr": mdl.hess_rowptr.tolist(), "hess_col": mdl.hess_col.tolist(),
    }
    with open(os.path.join(HERE, "ring9_seed0.json"), "w") as fh:
        json.dump(doc, fh, indent=0)


if __name__ == "__main__":
    main()
