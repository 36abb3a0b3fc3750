"""Write the oracle's results at the full size of the N = 100,000 Matern-3/2
workload (l = 0.1, sigma = 1e-4, leaf 200, eps_H = 1e-8, tau = 1e-2,
r = 100, p = 10, one right-hand side) to tests/golden/oracle_matern32-l0.1-N100k.npz.

Calls only the oracle and the seeded input generators.  The fixture records:
* the tree permutation, the points per proxy sphere and the H^2 ranks of every node,
  and a SHA-256 digest of each node's skeleton (original indices, int64 little
  endian) -- integer results, compared exactly;
* the HSS ranks of every node and a SHA-256 digest of each node's pivot list;
* the PCG iterate after 20 iterations (x0 = 0) and its norm;
* the iterations PCG needs to reach 1e-8 and the true relative residual then;
* the oracle's wall-clock phase times on this host (context only).

These are the oracle's own values (the paper prints no worked example at this
size).  The run takes hours on an 8-core host and about 40 GB of memory:

    python tests/golden/make_fullsize.py
"""
import hashlib
import json
import os
import platform
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "..", ".."))

import numpy as np  # noqa: E402

import workloads  # noqa: E402
from oracle.h2 import H2  # noqa: E402
from oracle.pcg import pcg  # noqa: E402
from oracle.spdhss import SPDHSS  # noqa: E402

W = workloads.MEDIUM
OUT = os.path.join(HERE, f"oracle_{W.name.rsplit('-', 1)[0]}.npz")
FIXED_ITERS = 20


def digest(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(np.asarray(a, dtype="<i8")).tobytes()).hexdigest()


def main():
    t0 = time.time()
    X = W.points()
    h = H2(X, W.kernel, W.ell, W.shift, W.leaf, W.h2_tol, eta=W.eta)
    T = h.tree
    t1 = time.time()
    print(f"H2 built in {t1 - t0:.0f} s", flush=True)
    s = SPDHSS(h, W.omega()[T.perm], W.hss_tol, W.max_rank, "chol")
    t2 = time.time()
    print(f"SPD HSS built in {t2 - t1:.0f} s", flush=True)
    b = W.rhs()[T.perm]
    x20_t, it20, _ = pcg(h.matvec, s.solve, b, 0.0, FIXED_ITERS)
    x20 = np.empty_like(x20_t)
    x20[T.perm] = x20_t
    t3 = time.time()
    print(f"{FIXED_ITERS} PCG iterations in {t3 - t2:.0f} s", flush=True)
    _, its, res = pcg(h.matvec, s.solve, b, W.pcg_tol, 20000)
    t4 = time.time()
    print(f"PCG to {W.pcg_tol}: {its.tolist()} iterations, residual {res.tolist()}, {t4 - t3:.0f} s", flush=True)
    nn = T.nnodes
    meta = {
        "workload": W.name, "n": W.n, "fixed_iterations": FIXED_ITERS,
        "pcg_iterations": [int(i) for i in its], "pcg_true_relres": [float(r) for r in res],
        "seconds": {"h2": t1 - t0, "spdhss": t2 - t1, "pcg_fixed": t3 - t2, "pcg_converge": t4 - t3},
        "host": {"cpu": platform.processor() or platform.machine(), "nproc": os.cpu_count()},
        "skeleton_sha256": [digest(h.skel[v]) if v in h.skel else digest([]) for v in range(nn)],
        "pivot_sha256": [digest(s.piv[v]) if v in s.piv else digest([]) for v in range(nn)],
    }
    np.savez_compressed(
        OUT,
        perm=T.perm.astype(np.int32),
        proxy_n=np.array([h.proxy_n.get(v, 0) for v in range(nn)], dtype=np.int32),
        h2_rank=np.array([h.rank(v) if v in h.skel else 0 for v in range(nn)], dtype=np.int32),
        hss_rank=np.array([s.rank.get(v, 0) for v in range(nn)], dtype=np.int32),
        x_fixed=x20,
        meta=np.frombuffer(json.dumps(meta).encode(), dtype=np.uint8),
    )
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
