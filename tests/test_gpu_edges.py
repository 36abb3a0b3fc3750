"""Degenerate and edge cases of the HIP path against the oracle and closed
forms (GPU): a single leaf (the HSS matrix is the dense block), the
block-Jacobi limit r_max = 0, more than 4 right-hand sides (the MFMA product
and apply), a negative shift (indefinite leaf blocks), and argument errors
reported through the C ABI."""
import numpy as np
import pytest

import workloads
from oracle import kernels as okern
from oracle.h2 import H2 as OH2
from oracle.pcg import pcg as opcg
from oracle.spdhss import SPDHSS as OHSS

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2011_07632_amd import binding
    return binding


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b))


def cols(B, a):
    return B.cols_like(a.shape[0], a.shape[1], "cuda").copy_(torch.from_numpy(np.ascontiguousarray(a)))


def test_single_leaf_is_dense(B):
    w = workloads.SMALL.with_(name="gaussian-l0.5-N50", n=50)
    X = w.points()
    A = okern.evaluate(w.kernel, w.ell, X, X) + w.shift * np.eye(w.n)
    h2 = B.h2_build(torch.from_numpy(X).cuda(), w.kernel, w.ell, w.shift, leaf=64, tol=w.h2_tol)
    assert h2.levels == 1
    x = workloads.gaussian_matrix(w.n, 2, 5)
    assert rel(B.h2_matvec(h2, cols(B, x)).cpu().numpy(), A @ x) <= 1e-13
    ulv = B.ulv_factor(B.spdhss_build(h2, w.hss_tol, w.max_rank, w.oversample,
                                      omega=cols(B, w.omega())))
    assert rel(B.ulv_apply(ulv, cols(B, x)).cpu().numpy(), np.linalg.solve(A, x)) <= 1e-10
    _, it, res = B.pcg_solve(h2, ulv, cols(B, x), rtol=1e-10, maxit=10)
    assert it.tolist() == [1, 1]
    assert float(res.max()) <= 1e-10


def test_block_jacobi_limit(B):
    """r_max = 0: the HSS matrix is blockdiag(A_ii); its solve is per-leaf."""
    w = workloads.SMALL.with_(name="gaussian-l0.5-N1500-bj", n=1500, max_rank=0, seed_base=3)
    X = w.points()
    h2 = B.h2_build(torch.from_numpy(X).cuda(), w.kernel, w.ell, w.shift, leaf=w.leaf, tol=w.h2_tol)
    hss = B.spdhss_build(h2, w.hss_tol, 0, w.oversample, omega=cols(B, w.omega()))
    assert (hss.ranks() == 0).all()
    ulv = B.ulv_factor(hss)
    b = workloads.gaussian_matrix(w.n, 1, 9)
    x = B.ulv_apply(ulv, cols(B, b)).cpu().numpy()
    perm, start = h2.perm(), h2.node_start()
    L = h2.levels
    xo = np.empty_like(b)
    for v in range((1 << (L - 1)) - 1, (1 << L) - 1):
        idx = perm[start[v]:start[v + 1]]
        Aii = okern.evaluate(w.kernel, w.ell, X[idx], X[idx]) + w.shift * np.eye(len(idx))
        xo[idx] = np.linalg.solve(Aii, b[idx])
    assert rel(x, xo) <= 1e-10
    o_h2 = OH2(X, w.kernel, w.ell, w.shift, w.leaf, w.h2_tol, eta=w.eta)
    o_hss = OHSS(o_h2, w.omega()[o_h2.tree.perm], w.hss_tol, 0, "chol")
    _, it, _ = B.pcg_solve(h2, ulv, cols(B, b), rtol=w.pcg_tol, maxit=500, raise_on_nonconvergence=False)
    _, ito, _ = opcg(o_h2.matvec, o_hss.solve, b[o_h2.tree.perm], w.pcg_tol, 500)
    assert abs(int(it[0]) - int(ito[0])) <= 1


def test_more_than_four_columns(B):
    """6 right-hand sides: the product and the apply take the MFMA kernels."""
    w = workloads.SMALL
    X = w.points()
    h2 = B.h2_build(torch.from_numpy(X).cuda(), w.kernel, w.ell, w.shift, leaf=w.leaf, tol=w.h2_tol)
    ulv = B.ulv_factor(B.spdhss_build(h2, w.hss_tol, w.max_rank, w.oversample, omega=cols(B, w.omega())))
    o_h2 = OH2(X, w.kernel, w.ell, w.shift, w.leaf, w.h2_tol, eta=w.eta)
    perm = o_h2.tree.perm
    o_hss = OHSS(o_h2, w.omega()[perm], w.hss_tol, w.max_rank, "chol")
    b = workloads.gaussian_matrix(w.n, 6, 21)
    xo = np.empty_like(b)
    xo[perm] = o_hss.solve(b[perm])
    assert rel(B.ulv_apply(ulv, cols(B, b)).cpu().numpy(), xo) <= 1e-10
    x, it, _ = B.pcg_solve(h2, ulv, cols(B, b), rtol=0.0, maxit=3, raise_on_nonconvergence=False)
    xo_t, ito, _ = opcg(o_h2.matvec, o_hss.solve, b[perm], 0.0, 3)
    xo = np.empty_like(b)
    xo[perm] = xo_t
    assert it.tolist() == ito.tolist()
    assert rel(x.cpu().numpy(), xo) <= 1e-10


def test_negative_shift_reports_not_spd(B):
    """sigma = -0.05 makes every leaf block K_ii + sigma I of the Gaussian
    kernel indefinite (its smallest eigenvalue is about -0.05): the build stops
    at a leaf Cholesky with SPD_E_NOT_SPD and names the node.  The H^2
    product itself is defined for any shift and matches the oracle's."""
    w = workloads.SMALL.with_(name="gaussian-l0.5-N1200-indefinite", n=1200, shift=-0.05)
    X = w.points()
    h2 = B.h2_build(torch.from_numpy(X).cuda(), w.kernel, w.ell, w.shift, leaf=w.leaf, tol=w.h2_tol)
    o_h2 = OH2(X, w.kernel, w.ell, w.shift, w.leaf, w.h2_tol, eta=w.eta)
    perm = o_h2.tree.perm
    x = workloads.gaussian_matrix(w.n, 2, 31)
    yo = np.empty_like(x)
    yo[perm] = o_h2.matvec(x[perm])
    assert rel(B.h2_matvec(h2, cols(B, x)).cpu().numpy(), yo) <= 1e-10
    with pytest.raises(B.SpdError) as e:
        B.spdhss_build(h2, w.hss_tol, w.max_rank, w.oversample, omega=cols(B, w.omega()))
    assert e.value.code == B.SPD_E_NOT_SPD and "node" in str(e.value)


def test_argument_errors(B):
    X = torch.from_numpy(workloads.SMALL.with_(n=200).points()).cuda()
    with pytest.raises(B.SpdError):
        B.h2_build(X[:0], "gaussian", 0.5, 1e-2)
    with pytest.raises(B.SpdError):
        B.h2_build(X, "gaussian", 0.5, 1e-2, leaf=0)
    with pytest.raises(B.SpdError):
        B.h2_build(X, "gaussian", 0.5, 1e-2, tol=1.5)
    with pytest.raises(B.SpdError):
        B.h2_build(X, "gaussian", -0.5, 1e-2)
    h2 = B.h2_build(X, "gaussian", 0.5, 1e-2, leaf=32)
    with pytest.raises(B.SpdError):  # more than 256 samples
        B.spdhss_build(h2, 1e-2, max_rank=250, oversample=10)
    hss = B.spdhss_build(h2, 1e-2, max_rank=20, oversample=10)
    ulv = B.ulv_factor(hss)
    b = B.cols_like(200, 1, "cuda").fill_(1.0)
    with pytest.raises(B.SpdError):
        B.pcg_solve(h2, ulv, b, rtol=-1.0, maxit=10)


@pytest.mark.parametrize("n", [1, 2, 3])
def test_tiny_problems(B, n):
    """N = 1, 2, 3 points: one leaf, the matrix is dense K + sigma I; the
    product, the HSS solve and PCG must reproduce it exactly up to rounding."""
    w = workloads.SMALL.with_(name=f"gaussian-l0.5-N{n}", n=n)
    X = w.points()
    A = okern.evaluate(w.kernel, w.ell, X, X) + w.shift * np.eye(n)
    h2 = B.h2_build(torch.from_numpy(X).cuda(), w.kernel, w.ell, w.shift, leaf=64, tol=w.h2_tol)
    assert h2.levels == 1
    x = workloads.gaussian_matrix(n, 2, 5)
    assert rel(B.h2_matvec(h2, cols(B, x)).cpu().numpy(), A @ x) <= 1e-14
    ulv = B.ulv_factor(B.spdhss_build(h2, w.hss_tol, 2, 1, omega=cols(B, workloads.gaussian_matrix(n, 3, 6))))
    assert rel(B.ulv_apply(ulv, cols(B, x)).cpu().numpy(), np.linalg.solve(A, x)) <= 1e-12
    sol, it, res = B.pcg_solve(h2, ulv, cols(B, x), rtol=1e-12, maxit=10)
    assert rel(sol.cpu().numpy(), np.linalg.solve(A, x)) <= 1e-12
    assert it.tolist() == [1, 1]


def test_padded_leading_dimension(B):
    """Right-hand sides with ld > N (columns of a taller buffer): the default
    outputs take the same layout, and product, apply and PCG give the same
    results bit for bit as with ld = N."""
    w = workloads.SMALL.with_(n=700)
    X = torch.from_numpy(w.points()).cuda()
    h2 = B.h2_build(X, w.kernel, w.ell, w.shift, leaf=64, tol=w.h2_tol)
    ulv = B.ulv_factor(B.spdhss_build(h2, w.hss_tol, 20, 10))
    x = workloads.gaussian_matrix(w.n, 3, 71)
    ld = w.n + 7
    print(f"[edges] padded ld = {ld}, N = {w.n}, 3 columns", flush=True)
    big = torch.full((3, ld), float("nan"), dtype=torch.float64, device="cuda")
    xp = big.t()[:w.n]
    xp.copy_(torch.from_numpy(x))
    xc = cols(B, x)
    for f in (lambda v: B.h2_matvec(h2, v), lambda v: B.ulv_apply(ulv, v),
              lambda v: B.pcg_solve(h2, ulv, v, rtol=1e-8, maxit=200, raise_on_nonconvergence=False)[0]):
        yp, yc = f(xp), f(xc)
        assert yp.stride() == (1, ld) and yc.stride() == (1, w.n)
        assert torch.equal(yp, yc)
    with pytest.raises(ValueError):  # an output whose layout differs from the input's
        B.pcg_solve(h2, ulv, xp, out=B.cols_like(w.n, 3, "cuda"))


def test_largest_leaf_and_sample_count(B):
    """The library's largest leaf (512 points) and sample count (s = 256 with
    fixed rank 246, so the compression runs in the global-memory pivoted QR):
    ranks and pivots equal the oracle's, and the product and the HSS solve
    agree with it to 1e-10."""
    w = workloads.SMALL.with_(name="matern32-l0.3-N1024-leaf512", n=1024, kernel="matern32", ell=0.3,
                              shift=1e-3, leaf=512, max_rank=246, oversample=10, hss_tol=0.0, seed_base=12)
    print(f"[edges] {w.name}: s = {w.s}", flush=True)
    X = w.points()
    h2 = B.h2_build(torch.from_numpy(X).cuda(), w.kernel, w.ell, w.shift, leaf=w.leaf, tol=w.h2_tol,
                    proxy_shells=4, proxy_per_shell=64)
    hss = B.spdhss_build(h2, w.hss_tol, w.max_rank, w.oversample, omega=cols(B, w.omega()))
    o_h2 = OH2(X, w.kernel, w.ell, w.shift, w.leaf, w.h2_tol, shells=4, per_shell=64)
    o_hss = OHSS(o_h2, w.omega()[o_h2.tree.perm], w.hss_tol, w.max_rank, "chol")
    T = o_h2.tree
    assert [T.size(v) for v in T.leaves()] == [512, 512]
    r = hss.ranks()
    for v in T.leaves():
        assert r[v] == o_hss.rank[v] == 246
        assert hss.pivots(v).tolist() == o_hss.piv[v].tolist()
    x = workloads.gaussian_matrix(w.n, 2, 13)
    yo = np.empty_like(x)
    yo[T.perm] = o_h2.matvec(x[T.perm])
    assert rel(B.h2_matvec(h2, cols(B, x)).cpu().numpy(), yo) <= 1e-10
    xo = np.empty_like(x)
    xo[T.perm] = o_hss.solve(x[T.perm])
    assert rel(B.ulv_apply(B.ulv_factor(hss), cols(B, x)).cpu().numpy(), xo) <= 1e-10
