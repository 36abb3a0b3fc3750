"""Run-to-run determinism on the GPU: the same inputs give bit-identical
results (no floating-point atomics; every sum has a fixed order)."""
import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2011_07632_amd import binding
    return binding


def cols(B, a):
    return B.cols_like(a.shape[0], a.shape[1], "cuda").copy_(torch.from_numpy(np.ascontiguousarray(a)))


def solve_once(B, w, b):
    X = torch.from_numpy(w.points()).cuda()
    h2 = B.h2_build(X, w.kernel, w.ell, w.shift, leaf=w.leaf, tol=w.h2_tol)
    hss = B.spdhss_build(h2, w.hss_tol, w.max_rank, w.oversample, omega=cols(B, w.omega()))
    ulv = B.ulv_factor(hss)
    y = B.h2_matvec(h2, cols(B, b)).cpu().numpy()
    z = B.ulv_apply(ulv, cols(B, b)).cpu().numpy()
    x, it, res = B.pcg_solve(h2, ulv, cols(B, b), rtol=w.pcg_tol, maxit=500)
    return y, z, x.cpu().numpy(), it.tolist(), hss.ranks().tolist()


@pytest.mark.parametrize("nrhs", [1, 3, 6])
def test_two_runs_are_bit_identical(B, nrhs):
    w = workloads.SMALL.with_(name="matern32-l0.2-N2500", n=2500, kernel="matern32", ell=0.2, shift=1e-3,
                              leaf=48, max_rank=40, seed_base=21)
    b = workloads.gaussian_matrix(w.n, nrhs, 22)
    r1 = solve_once(B, w, b)
    r2 = solve_once(B, w, b)
    for a1, a2 in zip(r1, r2):
        if isinstance(a1, np.ndarray):
            assert np.array_equal(a1, a2)
        else:
            assert a1 == a2
