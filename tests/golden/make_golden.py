"""Write the oracle regression fixture tests/golden/oracle_n300.json.

Calls only the oracle (and the seeded input generators): a 300-point
Gaussian case with three levels.  The fixture records the oracle's integer
results (tree permutation, H^2 skeletons, HSS ranks and pivots, PCG
iterations) and a few floating-point summaries, so that a later change to the
oracle's arithmetic shows up in test_oracle_pins.py::test_golden_fixture and
has to be justified.  These are the oracle's own values, not the paper's: the
paper prints no worked example.

    python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "..", ".."))

import numpy as np  # noqa: E402

import workloads  # noqa: E402
from oracle.h2 import H2  # noqa: E402
from oracle.pcg import pcg  # noqa: E402
from oracle.spdhss import SPDHSS  # noqa: E402

W = workloads.SMALL.with_(name="gaussian-l0.5-N300-golden", n=300, leaf=40, max_rank=20, seed_base=11)


def compute() -> dict:
    X = W.points()
    h = H2(X, W.kernel, W.ell, W.shift, W.leaf, W.h2_tol, eta=W.eta, shells=4, per_shell=64)
    T = h.tree
    s = SPDHSS(h, W.omega()[T.perm], W.hss_tol, W.max_rank, "chol")
    b = W.rhs()[T.perm]
    x, it, res = pcg(h.matvec, s.solve, b, W.pcg_tol, 200)
    y = h.matvec(np.ones((W.n, 1)))
    return {
        "workload": W.name,
        "perm": T.perm.tolist(),
        "h2_skeletons": {str(v): h.skel[v].tolist() for v in range(1, T.nnodes)},
        "hss_ranks": {str(v): int(s.rank[v]) for v in range(1, T.nnodes)},
        "hss_pivots": {str(v): np.asarray(s.piv[v]).tolist() for v in range(1, T.nnodes)},
        "pcg_iterations": it.tolist(),
        "matvec_ones_norm": float(np.linalg.norm(y)),
        "solution_norm": float(np.linalg.norm(x)),
    }


if __name__ == "__main__":
    with open(os.path.join(HERE, "oracle_n300.json"), "w") as f:
        json.dump(compute(), f, indent=0, sort_keys=True)
    print("wrote", os.path.join(HERE, "oracle_n300.json"))
