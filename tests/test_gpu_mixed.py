"""Mixed precision against the FP64 oracle (GPU): FP32 solve operators (FP64
vectors and sums), the FP32-block H^2 product (FP64 accumulation), and PCG
with either.  The FP32 bar is 1e-4 relative on the same quantity; PCG must
still reach the FP64 tolerance on the true residual (FP64 product)."""
import numpy as np
import pytest

import workloads
from oracle.h2 import H2 as OH2
from oracle.pcg import pcg as opcg
from oracle.spdhss import SPDHSS as OHSS

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

W = workloads.SMALL


@pytest.fixture(scope="module")
def S():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2011_07632_amd import binding as B
    X = W.points()
    h2 = B.h2_build(torch.from_numpy(X).cuda(), W.kernel, W.ell, W.shift, leaf=W.leaf, tol=W.h2_tol)
    om = B.cols_like(W.n, W.s, "cuda").copy_(torch.from_numpy(W.omega()))
    hss = B.spdhss_build(h2, W.hss_tol, W.max_rank, W.oversample, omega=om)
    o_h2 = OH2(X, W.kernel, W.ell, W.shift, W.leaf, W.h2_tol, eta=W.eta)
    o_hss = OHSS(o_h2, W.omega()[o_h2.tree.perm], W.hss_tol, W.max_rank, "chol")
    return dict(B=B, h2=h2, hss=hss, u64=B.ulv_factor(hss), u32=B.ulv_factor(hss, precision="f32"),
                o_h2=o_h2, o_hss=o_hss)


def cols(B, a):
    return B.cols_like(a.shape[0], a.shape[1], "cuda").copy_(torch.from_numpy(np.ascontiguousarray(a)))


# 1-4 columns: the dot-form products with FP32 operators; 5-16: the
# symmetric-pair kernel's row sums with FP32 A operands
@pytest.mark.parametrize("nrhs", [1, 3, 5, 16])
def test_f32_apply_against_oracle(S, nrhs):
    B, perm = S["B"], S["o_h2"].tree.perm
    b = workloads.gaussian_matrix(W.n, nrhs, 31)
    xo = np.empty_like(b)
    xo[perm] = S["o_hss"].solve(b[perm])
    x32 = B.ulv_apply(S["u32"], cols(B, b)).cpu().numpy()
    x64 = B.ulv_apply(S["u64"], cols(B, b)).cpu().numpy()
    e32 = np.linalg.norm(x32 - xo) / np.linalg.norm(xo)
    e64 = np.linalg.norm(x64 - xo) / np.linalg.norm(xo)
    print(f"[mixed] apply error vs oracle: f32 {e32:.2e}, f64 {e64:.2e}", flush=True)
    assert e64 <= 1e-10
    assert e32 <= 1e-4
    assert e32 > e64  # the FP32 operators are in use


def test_f32_pcg_reaches_fp64_tolerance(S):
    B = S["B"]
    b = W.rhs()
    _, it32, res32 = B.pcg_solve(S["h2"], S["u32"], cols(B, b), rtol=W.pcg_tol, maxit=500)
    _, it64, res64 = B.pcg_solve(S["h2"], S["u64"], cols(B, b), rtol=W.pcg_tol, maxit=500)
    _, ito, _ = opcg(S["o_h2"].matvec, S["o_hss"].solve, b[S["o_h2"].tree.perm], W.pcg_tol, 500)
    print(f"[mixed] iterations f32 {it32.tolist()} f64 {it64.tolist()} oracle {ito.tolist()}; "
          f"relres f32 {res32.tolist()}", flush=True)
    assert float(res32.max()) <= 2 * W.pcg_tol
    assert abs(int(it32[0]) - int(ito[0])) <= 3


def test_more_than_sixteen_columns_use_fp64_operators(S):
    B, perm = S["B"], S["o_h2"].tree.perm
    b = workloads.gaussian_matrix(W.n, 17, 41)
    xo = np.empty_like(b)
    xo[perm] = S["o_hss"].solve(b[perm])
    x32 = B.ulv_apply(S["u32"], cols(B, b)).cpu().numpy()
    assert np.linalg.norm(x32 - xo) / np.linalg.norm(xo) <= 1e-10


@pytest.mark.parametrize("nrhs", [1, 2, 4, 5, 16])
def test_f32_product_against_oracle(S, nrhs):
    B, perm = S["B"], S["o_h2"].tree.perm
    x = workloads.gaussian_matrix(W.n, nrhs, 51)
    yo = np.empty_like(x)
    yo[perm] = S["o_h2"].matvec(x[perm])
    y32 = B.h2_matvec(S["h2"], cols(B, x), precision="f32").cpu().numpy()
    y64 = B.h2_matvec(S["h2"], cols(B, x)).cpu().numpy()
    e32 = np.linalg.norm(y32 - yo) / np.linalg.norm(yo)
    e64 = np.linalg.norm(y64 - yo) / np.linalg.norm(yo)
    print(f"[mixed] product error vs oracle ({nrhs} columns): f32 {e32:.2e}, f64 {e64:.2e}", flush=True)
    assert e64 <= 1e-10
    assert e32 <= 1e-6  # FP32 rounding of the blocks (relative 6e-8 per entry), well inside 1e-4
    assert e32 > e64


@pytest.mark.parametrize("pre,ncols", [("f64", 3), ("f32", 3), ("f32", 16)])
def test_f32_operator_pcg_reaches_fp64_tolerance(S, pre, ncols):
    B = S["B"]
    b = workloads.gaussian_matrix(W.n, ncols, 61)
    M = S["u64"] if pre == "f64" else S["u32"]
    x, it, res = B.pcg_solve(S["h2"], M, cols(B, b), rtol=W.pcg_tol, maxit=500, op_precision="f32")
    _, it64, _ = B.pcg_solve(S["h2"], M, cols(B, b), rtol=W.pcg_tol, maxit=500)
    # the reported residual is the FP64 one; check it independently with the FP64 product
    r = cols(B, b) - B.h2_matvec(S["h2"], x)
    rel = (torch.linalg.norm(r, dim=0) / torch.linalg.norm(cols(B, b), dim=0)).cpu().numpy()
    print(f"[mixed] FP32 operator, {pre} preconditioner: iterations {it.tolist()} (FP64 operator "
          f"{it64.tolist()}), relres {res.tolist()}", flush=True)
    assert float(res.max()) <= 2 * W.pcg_tol and float(rel.max()) <= 2 * W.pcg_tol
    assert np.allclose(rel, res, rtol=1e-3, atol=0)
    assert (np.abs(it - it64) <= np.maximum(3, 0.2 * it64)).all()


def test_f32_product_argument_errors(S):
    B = S["B"]
    with pytest.raises(B.SpdError):
        B.h2_matvec(S["h2"], cols(B, workloads.gaussian_matrix(W.n, 17, 1)), precision="f32")
    import ctypes as C
    x = cols(B, workloads.gaussian_matrix(W.n, 1, 1))
    y = torch.empty_like(x)
    assert B.lib.h2_matvec_ex(S["h2"]._h, x.data_ptr(), y.data_ptr(), 1, W.n, 7, None) != 0


def test_unknown_precision_rejected(S):
    import ctypes as C
    B = S["B"]
    out = C.c_void_p()
    assert B.lib.ulv_factor_ex(S["hss"]._h, 7, None, C.byref(out)) != 0
