"""HIP path vs the CPU oracle, stage by stage, on seeded workloads (GPU).

Tolerances: 1e-10 relative for FP64 quantities; exact equality for the tree,
lists, skeleton sets, pivots and ranks (integer results)."""
import sys

import math

import numpy as np
import pytest

import workloads
from oracle.h2 import H2 as OH2
from oracle.pcg import pcg as opcg
from oracle.spdhss import SPDHSS as OHSS

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-10
# Phi_v U_v^H2 contains the interpolation matrix W = [I; (R11^{-1} R12)^T] of the
# proxy ID entry by entry.  With relative truncation at eps_H the triangular
# R11 has condition number up to about 1/eps_H, so last-bit differences in the
# proxy matrix can grow to u/eps_H in W (and Phi U).  Products that apply W to
# data (matvec, samples, bases, couplings) stay at TOL.
U_ROUND = 2.0 ** -53


def phiu_tol(eps_h):
    return max(TOL, 10 * U_ROUND / eps_h)


# An HSS basis is the first r columns of Q of a pivoted QR of the m x s
# samples Psi, i.e. (with equal pivots) the Q factor of the r pivot columns.
# By the perturbation bound of the QR factorization (Stewart 1977; Sun 1991:
# |dQ| <= sqrt(2) kappa(A) |dA| / |A| to first order), it moves by about
# sqrt(2) |R_00| / |R_{r-1,r-1}| times the relative difference of its input.
# That input is held to TOL by the stages before it (samples, products), and
# Householder QR itself adds m u; threshold forms keep |R_00| / |R_rr| below
# 1/tau, the fixed-rank form (tau = 0) can reach 1e5 (the r = 200 case).
def basis_tol(o, v, m):
    d, r = o.Rdiag[v], o.rank[v]
    return max(TOL, math.sqrt(2.0) * max(TOL, m * U_ROUND) * float(d[0]) / float(d[r - 1]))

CASES = {
    # small Gaussian case: 2,000 cube points, 32 leaves of 62/63
    "gauss2000": dict(w=workloads.SMALL, shells=8, per_shell=128),
    # ragged Matern case spanning several tiles: 3,001 points, leaves of 46/47
    "matern3001": dict(w=workloads.SMALL.with_(name="matern32-l0.15-N3001", n=3001, kernel="matern32",
                                               ell=0.15, shift=1e-3, leaf=50, max_rank=40, seed_base=7),
                       shells=6, per_shell=96),
    # exponential kernel on the unit sphere, threshold form with a small cap
    "exp1500": dict(w=workloads.SMALL.with_(name="exp-l0.2-N1500-sphere", n=1500, point_set="sphere",
                                            kernel="exponential", ell=0.2, shift=1e-2, leaf=40,
                                            max_rank=30, hss_tol=1e-3, seed_base=8),
                    shells=6, per_shell=96),
    # deep tree (12 levels, 2,048 leaves of 9/10 points): exercises the level
    # recursions far beyond the shallow cases
    "deep20000": dict(w=workloads.SMALL.with_(name="gaussian-l0.2-N20000-deep", n=20000, ell=0.2, shift=1e-1,
                                              leaf=10, max_rank=30, hss_tol=1e-1, seed_base=10),
                      shells=4, per_shell=64, pcg_maxit=60),
    # constant-density ball (the paper's point set), Matern kernel
    "ball1800": dict(w=workloads.SMALL.with_(name="matern32-l0.2-N1800-ball", n=1800, point_set="ball",
                                             kernel="matern32", ell=0.2, shift=1e-2, leaf=48, max_rank=40,
                                             seed_base=11),
                     shells=6, per_shell=96),
    # the paper's larger fixed rank r = 200 (s = 210 samples: the global-memory
    # CPQR with Q formation), exponential kernel, leaves of 256
    "r200": dict(w=workloads.SMALL.with_(name="exp-l0.1-N4096-r200", n=4096, kernel="exponential", ell=0.1,
                                         shift=1e-2, leaf=256, max_rank=200, hss_tol=0.0, seed_base=31),
                 shells=4, per_shell=64),
    # the RPY tensor (3 rows per particle, no shift): 2,000 particles of radius
    # 0.29 at unit density in a ball, 6,000 rows in leaves of 90 rows
    "rpy2000": dict(w=workloads.RPY_SMALL.with_(name="rpy-a0.29-N2000-ball1", n=2000, leaf=90),
                    shells=8, per_shell=128),
    # the 2^d-ary box-bisection tree (Section 6): 4,000 cube points, 64 boxes
    # of 48-80 points (6 binary levels), Gaussian kernel
    "box4000": dict(w=workloads.SMALL.with_(name="gaussian-l0.3-N4000-box", n=4000, ell=0.3, leaf=128,
                                            max_rank=40, seed_base=12, tree="box"),
                    shells=6, per_shell=96),
    # box-bisection tree on the ball: ragged leaves at the surface (11 to 103
    # points), Matern kernel
    "boxball3000": dict(w=workloads.SMALL.with_(name="matern32-l0.2-N3000-ball-box", n=3000, point_set="ball",
                                                kernel="matern32", ell=0.2, shift=1e-2, leaf=128, max_rank=40,
                                                seed_base=13, tree="box"),
                        shells=6, per_shell=96),
    # the RPY tensor on the box-bisection tree: 1,000 particles (3,000 rows),
    # leaves of 12 to 96 rows, a particle's three rows in one leaf
    "rpybox1000": dict(w=workloads.RPY_SMALL.with_(name="rpy-a0.29-N1000-ball1-box", n=1000, leaf=150,
                                                   seed_base=14, tree="box"),
                       shells=8, per_shell=128),
    # inverse multiquadric, fixed-rank form (tol = 0)
    "imq1200": dict(w=workloads.SMALL.with_(name="imq-c0.1-N1200", n=1200, kernel="imq", ell=0.1,
                                            shift=1e-3, leaf=30, max_rank=20, hss_tol=0.0, seed_base=9),
                    shells=4, per_shell=64),
}


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    d = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (d if d > 0 else 1.0)


class Pair:
    def __init__(self, name):
        from paper_2011_07632_amd import binding as B
        c = CASES[name]
        w = c["w"]
        print(f"\n[parity] case {name}: N={w.n} kernel={w.kernel}", flush=True)
        self.w, self.B, self.name = w, B, name
        X = w.points()
        self.X = X
        self.o_h2 = OH2(X, w.kernel, w.ell, w.shift, w.leaf, w.h2_tol, eta=w.eta,
                        shells=c["shells"], per_shell=c["per_shell"], tree_kind=w.tree)
        self.T = self.o_h2.tree
        om = w.omega()
        self.o_hss = OHSS(self.o_h2, om[self.T.perm], w.hss_tol, w.max_rank, "chol")
        self.g_h2 = B.h2_build(torch.from_numpy(X).cuda(), w.kernel, w.ell, w.shift, leaf=w.leaf,
                               tol=w.h2_tol, eta=w.eta, proxy_shells=c["shells"],
                               proxy_per_shell=c["per_shell"], tree=w.tree)
        self.g_hss = B.spdhss_build(self.g_h2, w.hss_tol, w.max_rank, w.oversample,
                                    omega=B.cols_like(w.rows, w.s, "cuda").copy_(torch.from_numpy(om)))
        self.g_ulv = B.ulv_factor(self.g_hss)


_pairs = {}


@pytest.fixture(scope="module", params=list(CASES))
def P(request):
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    if request.param not in _pairs:
        _pairs[request.param] = Pair(request.param)
    return _pairs[request.param]


def test_tree_and_lists_exact(P):
    T = P.T
    assert P.g_h2.perm().tolist() == T.perm.tolist()
    assert P.g_h2.node_start()[:-1].tolist() == T.start.tolist()
    near, coup = P.g_h2.lists()
    for v in range(T.nnodes):
        assert near[v] == T.near[v], v
        assert coup[v] == T.coup[v], v


def test_h2_skeletons_exact(P):
    T = P.T
    k = P.g_h2.ranks()
    sk = P.g_h2.skeletons()
    pc = P.g_h2.proxy_counts()
    for v in range(1, T.nnodes):
        assert pc[v] == P.o_h2.proxy_n.get(v, 0), v
        assert k[v] == P.o_h2.rank(v), v
        assert sk[v].tolist() == P.o_h2.skel[v].tolist(), v


# 1-4 columns take the symmetric-pair streaming product (1, 2 and 4-column
# kernels), 5 and 16 the symmetric-pair MFMA product
@pytest.mark.parametrize("nrhs", [1, 2, 3, 5, 16])
def test_h2_matvec(P, nrhs):
    rng = np.random.default_rng(1)
    x = rng.standard_normal((P.w.rows, nrhs))
    xg = P.B.cols_like(P.w.rows, nrhs, "cuda").copy_(torch.from_numpy(x))
    y = P.B.h2_matvec(P.g_h2, xg).cpu().numpy()
    yo = np.empty_like(x)
    yo[P.T.perm] = P.o_h2.matvec(x[P.T.perm])
    assert rel(y, yo) <= TOL


def test_hss_ranks_pivots_exact(P):
    T = P.T
    r = P.g_hss.ranks()
    for v in range(1, T.nnodes):
        assert r[v] == P.o_hss.rank[v], v
        assert P.g_hss.pivots(v).tolist() == P.o_hss.piv[v].tolist(), v


def test_hss_generators(P):
    T, o = P.T, P.o_hss
    for v in range(1, T.nnodes):
        if o.rank[v] == 0:
            continue
        Vo = o.V[v] if T.is_leaf(v) else o.Vbar[v]
        assert np.abs(P.g_hss.basis(v) - Vo).max() <= basis_tol(o, v, Vo.shape[0]), v
        if not T.is_leaf(v):
            assert rel(P.g_hss.transfer(v), o.R[v]) <= TOL, v
        if P.o_h2.rank(v) > 0:
            assert rel(P.g_hss.phiu(v), o.PhiU[v]) <= phiu_tol(P.w.h2_tol), v
    for (i, j), Bo in o.Bc.items():
        if o.rank[i] and o.rank[j]:
            assert rel(P.g_hss.coupling(i, j), Bo) <= TOL, (i, j)


def test_leaf_factors(P):
    for v in P.T.leaves()[:8]:
        assert rel(P.g_hss.factor(v), P.o_hss.S[v]) <= TOL


def test_ulv_apply(P):
    b = workloads.gaussian_matrix(P.w.rows, 4, 77)
    bg = P.B.cols_like(P.w.rows, 4, "cuda").copy_(torch.from_numpy(b))
    x = P.B.ulv_apply(P.g_ulv, bg).cpu().numpy()
    xo = np.empty_like(b)
    xo[P.T.perm] = P.o_hss.solve(b[P.T.perm])
    assert rel(x, xo) <= TOL


def test_pcg_fixed_iterations(P):
    b = P.w.rhs()
    bg = P.B.cols_like(P.w.rows, b.shape[1], "cuda").copy_(torch.from_numpy(b))
    for k in (1, 5):
        x, it, _ = P.B.pcg_solve(P.g_h2, P.g_ulv, bg, rtol=0.0, maxit=k, raise_on_nonconvergence=False)
        xo_t, ito, _ = opcg(P.o_h2.matvec, P.o_hss.solve, b[P.T.perm], 0.0, k)
        xo = np.empty_like(b)
        xo[P.T.perm] = xo_t
        assert it.tolist() == ito.tolist()
        assert rel(x.cpu().numpy(), xo) <= TOL


def test_pcg_fixed_iterations_16_columns(P):
    """16 right-hand sides (the N = 1M workload's width): the MFMA symmetric-pair
    product, the MFMA apply and the per-column recurrences against the oracle
    at fixed iteration counts."""
    b = workloads.gaussian_matrix(P.w.rows, 16, 2016)
    bg = P.B.cols_like(P.w.rows, 16, "cuda").copy_(torch.from_numpy(b))
    x, it, _ = P.B.pcg_solve(P.g_h2, P.g_ulv, bg, rtol=0.0, maxit=4, raise_on_nonconvergence=False)
    xo_t, ito, _ = opcg(P.o_h2.matvec, P.o_hss.solve, b[P.T.perm], 0.0, 4)
    xo = np.empty_like(b)
    xo[P.T.perm] = xo_t
    assert it.tolist() == ito.tolist()
    assert rel(x.cpu().numpy(), xo) <= TOL


def test_pcg_converges_like_oracle(P):
    """Same stopping behaviour as the oracle: equal iteration counts (within one
    for rounding at the threshold) and, when the oracle converges, a true
    residual at the tolerance."""
    b = P.w.rhs()
    bg = P.B.cols_like(P.w.rows, b.shape[1], "cuda").copy_(torch.from_numpy(b))
    maxit = CASES[P.name].get("pcg_maxit", 500)
    x, it, res = P.B.pcg_solve(P.g_h2, P.g_ulv, bg, rtol=P.w.pcg_tol, maxit=maxit,
                               raise_on_nonconvergence=False)
    _, ito, reso = opcg(P.o_h2.matvec, P.o_hss.solve, b[P.T.perm], P.w.pcg_tol, maxit)
    # the oracle stops on the recursive residual (the paper's PCG); the library
    # then also requires the true residual to meet rtol and otherwise continues
    # from it, so where the oracle's true residual is above rtol the library
    # may take more iterations
    strict = reso <= P.w.pcg_tol
    assert np.abs(it - ito)[strict].max(initial=0) <= 1
    assert (it >= ito - 1).all()
    if (ito < maxit).all():
        assert (res <= 2 * P.w.pcg_tol).all()
    print(f"[parity] iterations gpu={it.tolist()} oracle={ito.tolist()} relres={res.tolist()} "
          f"oracle relres={reso.tolist()}", flush=True)
