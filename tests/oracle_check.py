"""Checks of a library solve against the oracle (test helper; CPU side).

For one workload instance the oracle builds its own H^2 matrix and SPD HSS
preconditioner (same points, kernel, options and Omega) and runs its PCG; the
library's solution is then judged by the oracle's operator: its relative
residual ||b - A_oracle x|| / ||b|| (an independent product), and, for FP64
solves whose oracle run ends with a true residual at the tolerance, the
iteration counts (equal within one, the rounding of the threshold test)."""
import numpy as np

from oracle.h2 import H2 as OH2
from oracle.pcg import pcg as opcg
from oracle.spdhss import SPDHSS as OHSS


def check_against_oracle(w, x, iters, fp64: bool, maxit: int = 3000):
    X = w.points()
    h = OH2(X, w.kernel, w.ell, w.shift, w.leaf, w.h2_tol, eta=w.eta)
    T = h.tree
    b = w.rhs()
    r = b[T.perm] - h.matvec(np.asarray(x)[T.perm])
    res = np.linalg.norm(r, axis=0) / np.linalg.norm(b, axis=0)
    out = {"oracle_operator_relres": res}
    if fp64:
        s = OHSS(h, w.omega()[T.perm], w.hss_tol, w.max_rank, "chol")
        _, ito, reso = opcg(h.matvec, s.solve, b[T.perm], w.pcg_tol, maxit)
        out["oracle_iters"], out["oracle_relres"] = ito, reso
        strict = reso <= w.pcg_tol
        out["iters_match"] = bool((np.abs(np.asarray(iters) - ito)[strict] <= 1).all())
    return out
