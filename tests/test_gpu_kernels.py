"""Each batched HIP kernel against the CPU oracle's building blocks (GPU)."""
import numpy as np
import pytest
import scipy.linalg as sla

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2011_07632_amd import binding
    return binding


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def colmajor_batch(mats):
    """list of (rows x cols) arrays -> (batch, cols, rows) contiguous array"""
    return np.stack([m.T for m in mats])


@pytest.mark.parametrize("m,n,k", [(70, 8, 33), (129, 24, 65), (245, 110, 245), (5, 3, 1)])
@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_gemm(B, m, n, k, ta, tb):
    rng = np.random.default_rng(m * n + ta * 2 + tb)
    bt = 3
    As = [rng.standard_normal((k, m) if ta else (m, k)) for _ in range(bt)]
    Bs = [rng.standard_normal((n, k) if tb else (k, n)) for _ in range(bt)]
    Cs = [rng.standard_normal((m, n)) for _ in range(bt)]
    dA, dB, dC = dev(colmajor_batch(As)), dev(colmajor_batch(Bs)), dev(colmajor_batch(Cs))
    B.test_gemm(dA, dB, dC, ta, tb, alpha=0.5, beta=-2.0)
    out = dC.cpu().numpy()
    for b in range(bt):
        a = As[b].T if ta else As[b]
        bb = Bs[b].T if tb else Bs[b]
        ref = 0.5 * a @ bb - 2.0 * Cs[b]
        np.testing.assert_allclose(out[b].T, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


# Products with at most 4 right-hand columns take the streaming kernel: row
# tiles of 64, 128 and 256 (several tiles past 256), inner dimensions shorter
# than the number of waves and with ragged last steps, 16-wave workgroups for
# small batches and 4-wave workgroups for batches of 2048 or more.
@pytest.mark.parametrize("m,n,k,bt", [(1, 1, 1, 3), (64, 1, 3, 3), (65, 2, 17, 3), (128, 4, 100, 3),
                                      (129, 1, 257, 3), (256, 3, 64, 3), (300, 1, 95, 3),
                                      (600, 2, 33, 2), (100, 1, 203, 2100), (200, 4, 41, 2100),
                                      (40, 2, 7, 2100)])
@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 1)])
def test_gemm_skinny(B, m, n, k, bt, ta, tb):
    rng = np.random.default_rng(m * 7 + n * 3 + k + bt + ta)
    As = [rng.standard_normal((k, m) if ta else (m, k)) for _ in range(bt)]
    Bs = [rng.standard_normal((n, k) if tb else (k, n)) for _ in range(bt)]
    Cs = [rng.standard_normal((m, n)) for _ in range(bt)]
    dA, dB, dC = dev(colmajor_batch(As)), dev(colmajor_batch(Bs)), dev(colmajor_batch(Cs))
    B.test_gemm(dA, dB, dC, ta, tb, alpha=1.5, beta=0.25)
    out = dC.cpu().numpy()
    for b in range(bt):
        a = As[b].T if ta else As[b]
        bb = Bs[b].T if tb else Bs[b]
        ref = 1.5 * a @ bb + 0.25 * Cs[b]
        np.testing.assert_allclose(out[b].T, ref, rtol=0, atol=1e-12 * max(np.abs(ref).max(), 1.0))


@pytest.mark.parametrize("n", [1, 31, 63, 245, 300])
def test_cholesky(B, n):
    rng = np.random.default_rng(n)
    mats = []
    for _ in range(3):
        G = rng.standard_normal((n, n))
        mats.append(G @ G.T + n * np.eye(n))
    d = dev(colmajor_batch(mats))
    fail = torch.zeros(3, dtype=torch.int32, device="cuda")
    B.test_chol(d, fail)
    assert fail.cpu().numpy().tolist() == [0, 0, 0]
    out = d.cpu().numpy()
    for b in range(3):
        ref = np.linalg.cholesky(mats[b])
        np.testing.assert_allclose(out[b].T, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_cholesky_reports_indefinite(B):
    rng = np.random.default_rng(5)
    n = 70
    G = rng.standard_normal((n, n))
    good = G @ G.T + n * np.eye(n)
    bad = good.copy()
    bad[40, 40] = -1e3
    d = dev(colmajor_batch([good, bad]))
    fail = torch.zeros(2, dtype=torch.int32, device="cuda")
    B.test_chol(d, fail)
    assert fail.cpu().numpy().tolist() == [0, 1]


@pytest.mark.parametrize("n,nrhs", [(1, 3), (63, 110), (245, 16), (300, 40)])
@pytest.mark.parametrize("trans,upper", [(0, 0), (1, 0), (1, 1)])
def test_trsm(B, n, nrhs, trans, upper):
    rng = np.random.default_rng(n + nrhs)
    Ls, Bs = [], []
    for _ in range(2):
        Lm = np.tril(rng.standard_normal((n, n))) + n * np.eye(n)
        if upper:
            Lm = Lm.T
        Ls.append(Lm)
        Bs.append(rng.standard_normal((n, nrhs)))
    dL, dB = dev(colmajor_batch(Ls)), dev(colmajor_batch(Bs))
    B.test_trsm(dL, dB, trans, upper)
    out = dB.cpu().numpy()
    for b in range(2):
        if upper:
            ref = sla.solve_triangular(Ls[b], Bs[b], lower=False)
        else:
            ref = sla.solve_triangular(Ls[b], Bs[b], lower=True, trans="T" if trans else "N")
        np.testing.assert_allclose(out[b].T, ref, rtol=0, atol=1e-11 * np.abs(ref).max())


@pytest.mark.parametrize("m,n,which", [(245, 110, 0), (63, 110, 0), (200, 110, 0), (300, 110, 0),
                                       (1024, 245, 1), (512, 300, 1),
                                       # above 2048 rows: the wide form with the Householder vector in
                                       # LDS (the sketched proxy ID), and above 8000 rows read from the
                                       # pivot column
                                       (3000, 400, 1), (2100, 1200, 1), (9000, 300, 1)])
def test_cpqr(B, m, n, which):
    from oracle.linalg import CPQR
    rng = np.random.default_rng(m + n)
    mats = [rng.standard_normal((m, n)) @ np.diag(np.exp(-0.05 * np.arange(n))) @
            np.linalg.qr(rng.standard_normal((n, n)))[0] for _ in range(2)]
    maxrank = min(m, n, 100 if which == 0 else 4096)
    tol = 1e-3
    bt = len(mats)
    dA = dev(colmajor_batch(mats))
    Q = torch.zeros((bt, max(maxrank, 1), m), dtype=torch.float64, device="cuda")
    piv = torch.zeros((bt, n if which else max(maxrank, 1)), dtype=torch.int32, device="cuda")
    rank = torch.zeros(bt, dtype=torch.int32, device="cuda")
    diag = torch.zeros((bt, max(maxrank, 1)), dtype=torch.float64, device="cuda")
    B.test_cpqr(dA, Q if which == 0 else None, piv, rank, diag, maxrank, tol, which)
    for b in range(bt):
        f = CPQR(mats[b], tol, maxrank)
        r = int(rank[b])
        assert r == f.rank
        assert piv[b, :r].cpu().numpy().tolist() == f.piv.tolist()
        np.testing.assert_allclose(diag[b, :r].cpu().numpy(), f.diag, rtol=1e-10)
        if which == 0:
            Qg = Q[b, :r].cpu().numpy().T
            np.testing.assert_allclose(Qg, f.q(), rtol=0, atol=1e-10)


# The symmetric-pair product on a block-cyclic symmetric matrix: every block
# A_it is read once for S_ij x_j and S_ji x_i = A_it^T x_i.  Up to 4 columns
# take the streaming kernel, 5-16 the FP64 MFMA kernel; rows span partial
# waves (37), several waves (100), exactly one tile (256), a ragged second tile
# (300) and the 1 MiB split of long rows (m = 512, 4 terms).  In the MFMA
# kernel a wave skips the 16-row quads of its 64-row strip past the last row:
# m = 16 and 20 keep one and two quads, 37 three; m = 150 gives four strips of
# which the third keeps two quads and the fourth none.
@pytest.mark.parametrize("nblk,m,nterm", [(3, 37, 1), (7, 100, 3), (5, 256, 2), (9, 300, 4), (9, 512, 4),
                                          (4, 16, 0), (7, 20, 3), (5, 150, 2)])
@pytest.mark.parametrize("n", [1, 3, 5, 16])
def test_symmetric_pair_product(B, nblk, m, nterm, n):
    rng = np.random.default_rng(nblk * 1000 + m + 7 * nterm + n)
    A = rng.standard_normal((nblk * max(nterm, 1), m, m))  # block (i, t): A[i * nterm + t] (row-major view)
    X = rng.standard_normal((n, nblk * m))
    Y = np.full((n, nblk * m), np.nan)
    dA, dX, dY = dev(A), dev(X), dev(Y)
    B.test_symm(dA, dX, dY, nblk, m, nterm)
    out = dY.cpu().numpy()
    ref = np.zeros((nblk * m, n))
    xc = X.T
    for i in range(nblk):
        for t in range(nterm):
            j = (i + 1 + t) % nblk
            blk = A[i * nterm + t].T  # the stored column-major m x m block
            ref[i * m:(i + 1) * m] += blk @ xc[j * m:(j + 1) * m]
            ref[j * m:(j + 1) * m] += blk.T @ xc[i * m:(i + 1) * m]
    scale = max(np.abs(ref).max(), 1.0)
    np.testing.assert_allclose(out.T, ref, rtol=0, atol=1e-13 * scale * m * max(nterm, 1))
