"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only draws random numbers and names workload shapes.  It holds
none of the method's arithmetic, so both the oracle and the HIP path may use
it without sharing any computation.

Point sets follow the workload descriptions used for the experiments: points
uniform in the unit cube, or uniform on the unit sphere surface (normalised
standard-normal triples).  The paper itself uses constant-density balls and
spheres (Section 6); 'ball' gives the former (a uniform direction times a
radius U^(1/3)), and the unit cube/sphere recipes stand in for them in the
benchmark configurations.

Array conventions
-----------------
* points: float64, shape (N, 3), C-contiguous, in ORIGINAL order.
* rhs / omega: float64, shape (N, ncols), Fortran (column-major) order, rows
  indexed by ORIGINAL point index.
"""
from __future__ import annotations

import dataclasses
import numpy as np

KERNELS = ("gaussian", "matern32", "exponential", "imq", "rpy")


def points(kind: str, n: int, seed: int) -> np.ndarray:
    """Seeded point set: 'cube' = iid U[0,1)^3, 'sphere' = unit-sphere surface,
    'ball' = uniform (constant density) in the unit ball, 'ball1' = uniform in
    the ball of radius (3n / (4 pi))^(1/3), one point per unit volume."""
    rng = np.random.default_rng(seed)
    if kind == "cube":
        x = rng.random((n, 3))
    elif kind == "sphere":
        g = rng.standard_normal((n, 3))
        x = g / np.linalg.norm(g, axis=1, keepdims=True)
    elif kind in ("ball", "ball1"):
        g = rng.standard_normal((n, 3))
        r = rng.random(n) ** (1.0 / 3.0)
        x = g / np.linalg.norm(g, axis=1, keepdims=True) * r[:, None]
        if kind == "ball1":  # constant density 1: radius (3n / (4 pi))^(1/3)
            x = x * (3.0 * n / (4.0 * np.pi)) ** (1.0 / 3.0)
    else:
        raise ValueError(f"unknown point set {kind!r}")
    return np.ascontiguousarray(x, dtype=np.float64)


def gaussian_matrix(n: int, ncols: int, seed: int) -> np.ndarray:
    """iid N(0,1) matrix, column-major; used for right-hand sides and Omega."""
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.standard_normal((n, ncols)))


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic problem: points, kernel, shift and solver tolerances."""
    name: str
    n: int
    point_set: str
    kernel: str
    ell: float
    shift: float
    leaf: int
    h2_tol: float
    hss_tol: float
    max_rank: int
    oversample: int
    nrhs: int
    pcg_tol: float
    eta: float = 1.0
    seed_base: int = 0
    rhs_seed: int | None = None  # right-hand sides of a request on another request's matrix
    tree: str = "kd"  # partition tree: "kd" or "box" (2^d-ary box bisection)

    @property
    def s(self) -> int:
        return self.max_rank + self.oversample

    def points(self) -> np.ndarray:
        return points(self.point_set, self.n, 1000 + self.seed_base)

    @property
    def rows(self) -> int:
        """Rows of the matrix: 3 per point for the tensor kernel (row 3p + c is
        component c of point p), else one."""
        return 3 * self.n if self.kernel == "rpy" else self.n

    def rhs(self) -> np.ndarray:
        return gaussian_matrix(self.rows, self.nrhs,
                               2000 + (self.seed_base if self.rhs_seed is None else self.rhs_seed))

    def omega(self) -> np.ndarray:
        return gaussian_matrix(self.rows, self.s, 3000 + self.seed_base)

    def with_(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


# Small case: Gaussian exp(-r^2/0.5^2) + 1e-2 I on 2,000 cube points.
SMALL = Workload(name="gaussian-l0.5-N2000-cube", n=2000, point_set="cube",
                 kernel="gaussian", ell=0.5, shift=1e-2, leaf=64, h2_tol=1e-8,
                 hss_tol=1e-2, max_rank=100, oversample=10, nrhs=1,
                 pcg_tol=1e-8, seed_base=0)

# Matern-3/2, l = 0.1, + 1e-4 I on 100,000 cube points.
MEDIUM = Workload(name="matern32-l0.1-N100k-cube", n=100_000, point_set="cube",
                  kernel="matern32", ell=0.1, shift=1e-4, leaf=200,
                  h2_tol=1e-8, hss_tol=1e-2, max_rank=100, oversample=10,
                  nrhs=1, pcg_tol=1e-8, seed_base=1)

# Gaussian l = 0.2 + 1e-3 I on 1,000,000 cube points, 16 right-hand sides.
LARGE = Workload(name="gaussian-l0.2-N1M-cube", n=1_000_000, point_set="cube",
                 kernel="gaussian", ell=0.2, shift=1e-3, leaf=400, h2_tol=1e-6,
                 hss_tol=1e-1, max_rank=100, oversample=10, nrhs=16,
                 pcg_tol=1e-8, seed_base=3)

# The N = 1M Gaussian workload as it is benchmarked: eps_H = 1e-8 instead of
# 1e-6 (at 1e-6 the H^2 matrix is not positive definite at this size, the
# input condition of Algorithm 5.3), and the HSS preconditioner with
# tau = 1e-2 and rank cap r = 200 (the paper's larger fixed rank) instead of
# tau = 1e-1 (with which PCG has not reached 1e-8 after 17,500 iterations).
HEADLINE = LARGE.with_(name="gaussian-l0.2-N1M-cube-eps1e-8-tau1e-2-r200", h2_tol=1e-8, hss_tol=1e-2,
                       max_rank=200)

# The same problem on the paper's 2^d-ary box-bisection tree (Section 6:
# bisect every dimension until no box holds more than 400 points): 4,096 boxes
# of 190 to 301 points at depth 12, the kd-tree's depth.
HEADLINE_BOX = HEADLINE.with_(name="gaussian-l0.2-N1M-cube-eps1e-8-tau1e-2-r200-boxtree", tree="box")

# The medium workload with a hundredfold larger shift (+ 1e-2 I): a better
# conditioned system on which FP32 rounding of the stored blocks stays far below
# the smallest eigenvalue (used to compare the mixed-precision forms).
MEDIUM_S2 = MEDIUM.with_(name="matern32-l0.1-s1e-2-N100k-cube", shift=1e-2)

# The RPY tensor kernel of the paper's Section 6: particles of radius a = 0.29
# (volume fraction about 0.1) in the ball of unit point density, no shift;
# 3 rows per particle.
RPY_SMALL = Workload(name="rpy-a0.29-N1200-ball1", n=1200, point_set="ball1", kernel="rpy", ell=0.29,
                     shift=0.0, leaf=96, h2_tol=1e-8, hss_tol=1e-2, max_rank=60, oversample=10, nrhs=1,
                     pcg_tol=1e-8, seed_base=20)
RPY_LARGE = Workload(name="rpy-a0.29-N100k-ball1", n=100_000, point_set="ball1", kernel="rpy", ell=0.29,
                     shift=0.0, leaf=400, h2_tol=1e-8, hss_tol=1e-2, max_rank=100, oversample=10, nrhs=16,
                     pcg_tol=1e-8, seed_base=21)

BY_NAME = {w.name: w for w in (SMALL, MEDIUM, LARGE, MEDIUM_S2, HEADLINE, HEADLINE_BOX, RPY_LARGE)}


# Batched case: independent instances of uneven sizes.  N is log-uniform in
# [5,000, 50,000]; instances alternate between the unit cube and the unit
# sphere; the kernel is drawn uniformly from Gaussian l = 0.3, exponential
# l = 0.2 and inverse multiquadric c = 0.1, each + 1e-3 I; leaf 128, HSS
# tolerance 1e-2, 4 right-hand sides.  Instance j draws its points, right-hand
# sides and Omega with seeds offset by BATCH_SEED + j.
BATCH_KERNELS = (("gaussian", 0.3), ("exponential", 0.2), ("imq", 0.1))
BATCH_SEED = 100 * 1002


def batch_instances(count: int = 64, seed: int = 4002, n_lo: int = 5000, n_hi: int = 50000) -> list:
    rng = np.random.default_rng(seed)
    out = []
    for j in range(count):
        n = int(round(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi)))))
        kern, ell = BATCH_KERNELS[int(rng.integers(len(BATCH_KERNELS)))]
        ps = "cube" if j % 2 == 0 else "sphere"
        out.append(Workload(name=f"batch{j}-{kern}-N{n}-{ps}", n=n, point_set=ps, kernel=kern, ell=ell,
                            shift=1e-3, leaf=128, h2_tol=1e-8, hss_tol=1e-2, max_rank=100, oversample=10,
                            nrhs=4, pcg_tol=1e-8, seed_base=BATCH_SEED + j))
    return out


# Served case: a seeded trace of solve requests with Poisson arrivals (rate
# per second), N log-uniform in [n_lo, n_hi], cube points, a kernel drawn from
# Gaussian / Matern-3/2 / exponential with l uniform in [0.05, 0.5], + 1e-3 I,
# leaf 400, 1 to 32 right-hand sides.  Request j draws its data with seeds
# offset by SERVE_SEED + j.
SERVE_KERNELS = ("gaussian", "matern32", "exponential")
SERVE_SEED = 100 * 1004


def serve_requests(count: int = 64, rate: float = 20.0, seed: int = 4004, n_lo: int = 10_000,
                   n_hi: int = 1_000_000, repeat: float = 0.0) -> list:
    """[(arrival seconds, Workload, key)] sorted by arrival.  With probability
    `repeat` a request (after the first) solves new right-hand sides on the
    matrix of an earlier non-repeated request, drawn uniformly; `key` names
    the matrix (the index of its first request, plus one)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    firsts = []
    for j in range(count):
        t += float(rng.exponential(1.0 / rate))
        n = int(round(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi)))))
        kern = SERVE_KERNELS[int(rng.integers(len(SERVE_KERNELS)))]
        ell = float(rng.uniform(0.05, 0.5))
        nrhs = int(rng.integers(1, 33))
        again = bool(rng.random() < repeat) if repeat > 0 else False
        if again and firsts:
            k = firsts[int(rng.integers(len(firsts)))]
            base = out[k][1]
            w = dataclasses.replace(base, name=f"req{j}-on-req{k}-r{nrhs}", nrhs=nrhs,
                                    rhs_seed=SERVE_SEED + 100_000 + j)
            out.append((t, w, k + 1))
            continue
        firsts.append(j)
        out.append((t, Workload(name=f"req{j}-{kern}-l{ell:.3f}-N{n}-r{nrhs}", n=n, point_set="cube",
                                kernel=kern, ell=ell, shift=1e-3, leaf=400, h2_tol=1e-8, hss_tol=1e-2,
                                max_rank=100, oversample=10, nrhs=nrhs, pcg_tol=1e-8,
                                seed_base=SERVE_SEED + j), j + 1))
    return out
