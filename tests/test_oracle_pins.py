"""Pins for the CPU oracle: each check fixes the oracle against something other
than itself (dense brute force, closed forms, library routines, identities of
the paper).  CPU only."""
import math

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

import workloads
from oracle import kernels
from oracle.h2 import H2
from oracle.linalg import CPQR
from oracle.pcg import pcg, matvec_error
from oracle.spdhss import SPDHSS
from oracle.tree import Tree


def small_h2(n=600, leaf=32, kind="gaussian", ell=0.5, shift=1e-2, tol=1e-8,
             shells=4, per_shell=64, seed=7, pset="cube"):
    X = workloads.points(pset, n, seed)
    return H2(X, kind, ell, shift, leaf, tol, shells=shells, per_shell=per_shell)


@pytest.fixture(scope="module")
def h2s():
    return small_h2()


@pytest.fixture(scope="module")
def hss(h2s):
    om = workloads.gaussian_matrix(h2s.tree.N, 40, 11)[h2s.tree.perm]
    return SPDHSS(h2s, om, 1e-2, 30, "chol")


@pytest.fixture(scope="module")
def hss_eig(h2s):
    om = workloads.gaussian_matrix(h2s.tree.N, 40, 11)[h2s.tree.perm]
    return SPDHSS(h2s, om, 1e-2, 30, "eig")


def dense_of(h2):
    return h2.dense()


# ---------------------------------------------------------------- kernels --
def test_kernel_closed_forms():
    o = np.zeros((1, 3))
    ell = 0.3
    for k in ("gaussian", "matern32", "exponential"):
        assert kernels.evaluate(k, ell, o, o)[0, 0] == 1.0
    assert kernels.evaluate("imq", 0.1, o, o)[0, 0] == pytest.approx(10.0, rel=1e-15)
    e1 = np.array([[1.0, 0.0, 0.0]])
    # Gaussian and exponential at r = ell give 1/e; Matern-3/2 at r = ell/sqrt(3) gives 2/e
    assert kernels.evaluate("gaussian", ell, o, ell * e1)[0, 0] == pytest.approx(math.exp(-1), rel=1e-15)
    assert kernels.evaluate("exponential", ell, o, ell * e1)[0, 0] == pytest.approx(math.exp(-1), rel=1e-15)
    assert kernels.evaluate("matern32", ell, o, ell / math.sqrt(3) * e1)[0, 0] == pytest.approx(2 * math.exp(-1), rel=1e-14)
    assert kernels.evaluate("imq", 0.1, o, 0.1 * e1)[0, 0] == pytest.approx(1 / (0.1 * math.sqrt(2)), rel=1e-15)
    # symmetry in its arguments, distance through all three coordinates
    X = workloads.points("cube", 5, 1)
    Y = workloads.points("cube", 4, 2)
    for k in kernels.KINDS:
        if k in kernels.TENSOR:  # tensor entries: their own pins in test_oracle_rpy.py
            continue
        np.testing.assert_allclose(kernels.evaluate(k, ell, X, Y), kernels.evaluate(k, ell, Y, X).T, rtol=0, atol=0)


# ------------------------------------------------------------------- tree --
@pytest.mark.parametrize("n,leaf", [(1, 4), (5, 8), (17, 4), (600, 32), (1000, 7)])
def test_tree_properties(n, leaf):
    X = workloads.points("cube", n, 3)
    T = Tree(X, leaf)
    assert sorted(T.perm.tolist()) == list(range(n))
    assert (1 << T.D) >= n / leaf and (T.D == 0 or (1 << (T.D - 1)) < n / leaf)
    for k in range(1, T.L + 1):
        sizes = [T.size(v) for v in T.nodes_at(k)]
        assert max(sizes) - min(sizes) <= 1
        assert sum(sizes) == n
    for v in range((1 << T.D) - 1):
        c1, c2 = T.children(v)
        P = X[T.perm[T.rng(v)]]
        ext = P.max(0) - P.min(0)
        ax = int(np.argmax(ext))
        left, right = X[T.perm[T.rng(c1)], ax], X[T.perm[T.rng(c2)], ax]
        if len(left) and len(right):
            assert left.max() <= right.min()
        assert T.size(c1) == T.size(v) // 2


def _lattice(m, seed, jitter):
    """An m x m x m lattice of integer points (spacing 1) in a seeded random
    order, each point moved by at most jitter along every axis."""
    rng = np.random.default_rng(seed)
    ijk = np.stack(np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij"), -1).reshape(-1, 3)
    ijk = ijk[rng.permutation(len(ijk))]
    return ijk, ijk + rng.uniform(-jitter, jitter, ijk.shape)


def _morton(ijk, bits):
    """Z-order code with x the most significant bit of every triple."""
    code = np.zeros(len(ijk), dtype=np.int64)
    for b in range(bits - 1, -1, -1):
        for a in range(3):
            code = (code << 1) | ((ijk[:, a] >> b) & 1)
    return code


@pytest.mark.parametrize("jitter", [0.0, 0.2])
@pytest.mark.parametrize("leaf,depth,group", [(1, 9, 0), (7, 9, 0), (8, 6, 1), (63, 6, 1), (64, 3, 2), (512, 0, 3)])
def test_box_tree_on_a_lattice_is_the_octree(leaf, depth, group, jitter):
    """On an 8 x 8 x 8 lattice the 2^d-ary box bisection is the octree of
    the lattice cells: the leaves at depth 3k, in heap order, are the
    2^(3-k)-cubes of points in Z-order (Morton order, x first), whatever the
    input order and a jitter below a quarter of the spacing."""
    ijk, X = _lattice(8, 5, jitter)
    T = Tree(X, leaf, kind="box")
    assert T.D == depth
    leaves = T.leaves()
    for a, v in enumerate(leaves):
        members = T.perm[T.rng(v)]
        assert len(members) == 8 ** group
        assert (_morton(ijk[members] >> group, 3 - group) == a).all()


@pytest.mark.parametrize("point_set,n,leaf", [("cube", 3000, 100), ("ball", 4000, 200), ("sphere", 2500, 100)])
def test_box_tree_properties(point_set, n, leaf):
    X = workloads.points(point_set, n, 4)
    T = Tree(X, leaf, kind="box")
    assert T.D % 3 == 0
    assert sorted(T.perm.tolist()) == list(range(n))
    sizes = [T.size(v) for v in T.leaves()]
    assert min(sizes) >= 1 and max(sizes) <= leaf and sum(sizes) == n
    up = T.nodes_at(4) if T.D >= 3 else []  # depth D - 3: some node exceeds leaf
    assert T.D == 0 or max(T.size(v) for v in up) > leaf
    for v in range((1 << T.D) - 1):
        ax = T.depth(v) % 3
        c1, c2 = T.children(v)
        x = X[T.perm[T.rng(v)], ax]
        mid = 0.5 * (x.min() + x.max())
        assert (X[T.perm[T.rng(c1)], ax] < mid).all() and (X[T.perm[T.rng(c2)], ax] >= mid).all()


def test_box_tree_rejects_a_node_without_extent():
    X = workloads.points("cube", 400, 6)
    X[:, 2] = 0.5  # a plane: the z bisection has nothing to split
    with pytest.raises(ValueError, match="no extent"):
        Tree(X, 50, kind="box")
    # a perfect tree cannot hold a box that runs out of points above depth D:
    # sparse boxes at the surface of a ball with small leaves
    with pytest.raises(ValueError, match="a node of 1 points"):
        Tree(workloads.points("ball", 4000, 4), 64, kind="box")
    with pytest.raises(ValueError, match="unknown tree"):
        Tree(X, 50, kind="oct")


def test_lists_tile_the_matrix_exactly(h2s):
    """Every leaf pair is covered exactly once by a near leaf block or by one
    coupling block at some level (the H^2 block partition)."""
    T = h2s.tree
    leaves = T.leaves()
    pos = {v: a for a, v in enumerate(leaves)}
    cnt = np.zeros((len(leaves), len(leaves)), dtype=int)

    def leaf_desc(v):
        while not T.is_leaf(v):
            v = T.children(v)[0]
        first = v
        return first

    def leaves_under(v):
        d = T.depth(v)
        span = 1 << (T.D - d)
        f = pos[leaf_desc(v)]
        return range(f, f + span)

    for i in leaves:
        for j in T.near[i]:
            cnt[pos[i], pos[j]] += 1
    for v in range(1, T.nnodes):
        for j in T.coup[v]:
            for a in leaves_under(v):
                for b in leaves_under(j):
                    cnt[a, b] += 1
    assert (cnt == 1).all()
    for v in range(T.nnodes):
        for j in T.near[v]:
            assert v in T.near[j] and not T.admissible(v, j)
        for j in T.coup[v]:
            assert v in T.coup[j] and T.admissible(v, j)
            assert not T.admissible(T.parent(v), T.parent(j))


# ------------------------------------------------------------------- CPQR --
def test_cpqr_matches_lapack_pivoting():
    rng = np.random.default_rng(0)
    for m, n in [(30, 20), (20, 30), (64, 64)]:
        M = rng.standard_normal((m, n)) * np.exp(-0.3 * rng.permutation(n))[None, :]
        f = CPQR(M, 0.0, min(m, n))
        Q = f.q()
        _, Rl, pl = sla.qr(M, pivoting=True, mode="economic")
        assert f.piv.tolist() == pl[: f.rank].tolist()
        np.testing.assert_allclose(np.abs(np.diag(f.R)), np.abs(np.diag(Rl))[: f.rank], rtol=1e-10)
        np.testing.assert_allclose(Q.T @ Q, np.eye(f.rank), atol=1e-13)
        np.testing.assert_allclose(Q @ f.R, M[:, f.perm], atol=1e-12 * np.abs(M).max())
        assert (np.diag(f.R) >= 0).all()


def test_cpqr_truncation_rule():
    rng = np.random.default_rng(1)
    U = np.linalg.qr(rng.standard_normal((40, 40)))[0]
    s = 10.0 ** -np.arange(40)
    M = (U * s) @ np.linalg.qr(rng.standard_normal((40, 40)))[0]
    f = CPQR(M, 1e-5, 100)
    d = f.diag
    assert (d[1:] > 1e-5 * d[0]).all()
    g = CPQR(M, 0.0, 40)
    assert g.diag[f.rank] <= 1e-5 * g.diag[0]
    assert CPQR(M, 0.0, 7).rank == 7


# --------------------------------------------------------------------- H2 --
def test_h2_matches_dense_kernel_matrix():
    h = small_h2(n=800, leaf=50, shells=8, per_shell=128, tol=1e-8)
    A, Ah = h.exact_dense(), h.dense()
    err = np.linalg.norm(A - Ah) / np.linalg.norm(A)
    assert err <= 10 * h.tol


@pytest.mark.parametrize("kind,pset,n,leaf,ell", [("gaussian", "cube", 1500, 64, 0.3), ("matern32", "ball", 1200, 100, 0.2),
                                                   ("rpy", "ball1", 500, 120, 0.29)])
def test_h2_on_the_box_tree_matches_dense(kind, pset, n, leaf, ell):
    """The H^2 construction on the 2^d-ary box-bisection tree (ragged leaves;
    for the RPY tensor the three rows of a particle stay in one box) still
    reproduces sigma*I + K to the order of its tolerance."""
    X = workloads.points(pset, n, 9)
    h = H2(X, kind, ell, 0.0 if kind == "rpy" else 1e-2, leaf, 1e-8, shells=8, per_shell=128, tree_kind="box")
    assert h.tree.kind == "box" and h.tree.D % 3 == 0
    A, Ah = h.exact_dense(), h.dense()
    assert np.linalg.norm(A - Ah) / np.linalg.norm(A) <= 10 * h.tol
    if kind == "rpy":  # rows 3p, 3p+1, 3p+2 share a leaf
        T = h.tree
        for v in T.leaves():
            parts = T.perm[T.rng(v)] // 3
            for q in np.unique(parts):
                assert np.count_nonzero(parts == q) == 3


def test_h2_matvec_matches_assembled(h2s):
    Ah = dense_of(h2s)
    x = np.random.default_rng(2).standard_normal((h2s.tree.N, 3))
    y = h2s.matvec(x)
    assert np.linalg.norm(y - Ah @ x) / np.linalg.norm(Ah @ x) < 1e-13
    # near blocks and coupling blocks are exact kernel entries
    T = h2s.tree
    for (i, j), B in list(h2s.B.items())[:20]:
        np.testing.assert_allclose(B, kernels.evaluate(h2s.kind, h2s.ell, h2s.X[h2s.skel[i]], h2s.X[h2s.skel[j]]), rtol=0, atol=0)


def test_sampling_is_masked_product(h2s):
    """Y^(k) = (A - diag({A_ii}_{lvl(k)})) Omega, eq. (Yk)."""
    T = h2s.tree
    Ah = dense_of(h2s)
    Om = np.random.default_rng(3).standard_normal((T.N, 5))
    for k in range(1, T.L):
        M = Ah.copy()
        for v in T.nodes_at(k):
            M[T.rng(v), T.rng(v)] = 0.0
        Y = h2s.matvec(Om, above=k)
        assert np.linalg.norm(Y - M @ Om) <= 1e-13 * np.linalg.norm(M @ Om)


# ---------------------------------------------------------------- SPD HSS --
def test_sketch_matches_dense_lambda(hss, h2s):
    """Psi_i equals Lambda_{ii^c} Omega_{i^c} built from dense Phi (Section 5.2.1)."""
    T = h2s.tree
    Ah = dense_of(h2s)
    Om = hss.Omega
    for k in range(1, T.L):
        for i in T.nodes_at(k)[:6]:
            rows = T.rng(i)
            off = Ah[rows, :].copy()
            off[:, rows] = 0.0
            if k == 1:
                ref = sla.solve_triangular(hss.S[i], off @ Om, lower=True)
            else:
                c1, c2 = T.children(i)
                P1, P2 = hss.Phi_full(c1), hss.Phi_full(c2)
                D = sla.block_diag(P1, P2)
                ref = sla.solve_triangular(hss.F[i], D @ (off @ Om), lower=True)
            assert np.linalg.norm(hss.Psi[i] - ref) <= 1e-12 * np.linalg.norm(ref)


def test_couplings_match_dense_phi(hss, h2s):
    """B_ij = Phi_i A_ij Phi_j^T (eq. bij_hss), Type-1 and Type-3 alike."""
    T = h2s.tree
    Ah = dense_of(h2s)
    Phi = {v: hss.Phi_full(v) for v in range(1, T.nnodes)}
    n = 0
    for (i, j), B in hss.Bc.items():
        ref = Phi[i] @ Ah[T.rng(i), T.rng(j)] @ Phi[j].T
        assert np.linalg.norm(B - ref) <= 1e-12 * max(np.linalg.norm(ref), 1e-300)
        n += 1
    assert n > 0


def test_phi_inverts_basis(hss):
    """Phi_i U_i = V_i^T S_i^{-1} S_i V_i = I for every node."""
    T = hss.tree
    for v in range(1, T.nnodes):
        P = hss.Phi_full(v) @ hss.U_full(v)
        np.testing.assert_allclose(P, np.eye(hss.rank[v]), atol=1e-11)


def test_cholesky_and_eig_forms_agree(hss, hss_eig):
    T = hss.tree
    for v in range(1, T.nnodes):
        assert hss.rank[v] == hss_eig.rank[v]
        assert hss.piv[v].tolist() == hss_eig.piv[v].tolist()
    for v in hss.R:
        np.testing.assert_allclose(hss.R[v], hss_eig.R[v], atol=1e-12 * np.abs(hss.R[v]).max())
    for key, B in hss.Bc.items():
        np.testing.assert_allclose(B, hss_eig.Bc[key], atol=1e-12 * max(np.abs(B).max(), 1.0))
    A1, A2 = hss.dense(), hss_eig.dense()
    assert np.linalg.norm(A1 - A2) <= 1e-12 * np.linalg.norm(A1)


def test_formal_recursion_reproduces_hss(hss, h2s):
    """eq. (recursion) with projections P_i = U_i Phi_i = S_i V_i V_i^T S_i^{-1},
    and the Section 3.2 identity A^(k) = diag(P_i) A^(k-1) diag(P_i)^T +
    diag(S_i (I - V_i V_i^T) S_i^T)."""
    T = h2s.tree
    Ak = dense_of(h2s)
    for k in range(1, T.L):
        P = np.zeros_like(Ak)
        Dg = np.zeros_like(Ak)
        for v in T.nodes_at(k):
            r = T.rng(v)
            P[r, r] = hss.U_full(v) @ hss.Phi_full(v)
            Dg[r, r] = Ak[r, r]
        nxt = Dg + P @ (Ak - Dg) @ P.T
        # S (I - V V^T) S^T = A_ii - P A_ii P^T for the block factor S_i of A^(k-1)_ii
        alt = P @ Ak @ P.T + (Dg - P @ Dg @ P.T)
        assert np.linalg.norm(nxt - alt) <= 1e-12 * np.linalg.norm(nxt)
        Ak = nxt
    Ahss = hss.dense()
    assert np.linalg.norm(Ak - Ahss) <= 1e-11 * np.linalg.norm(Ahss)


@pytest.mark.parametrize("kind,ell,shift", [("gaussian", 0.5, 1e-4), ("matern32", 0.2, 1e-4),
                                            ("exponential", 0.3, 1e-3), ("imq", 0.1, 1e-4)])
def test_hss_is_spd(kind, ell, shift):
    h = small_h2(n=400, leaf=25, kind=kind, ell=ell, shift=shift, shells=6, per_shell=96)
    assert np.linalg.eigvalsh(h.dense()).min() > 0
    om = workloads.gaussian_matrix(400, 20, 5)[h.tree.perm]
    s = SPDHSS(h, om, 1e-1, 10, "chol")
    assert np.linalg.eigvalsh(s.dense()).min() > 0


def test_exact_limit_full_rank():
    """tol = 0 with as many samples as rows keeps every basis complete, so the
    HSS matrix equals the H^2 matrix and one PCG step solves."""
    h = small_h2(n=120, leaf=15, shells=4, per_shell=64)
    om = workloads.gaussian_matrix(120, 80, 9)[h.tree.perm]
    s = SPDHSS(h, om, 0.0, 200, "chol")
    Ah = h.dense()
    assert np.linalg.norm(s.dense() - Ah) <= 1e-10 * np.linalg.norm(Ah)
    b = workloads.gaussian_matrix(120, 1, 4)
    _, it, res = pcg(h.matvec, s.solve, b, 1e-8, 50)
    assert it[0] <= 2 and res[0] <= 1e-8


def test_largest_leaf_and_sample_count():
    """At the library's largest leaf (512 points) and sample count (s = 256,
    fixed rank 246): each leaf rank is min(r_max, rows, s), the diagonal
    blocks are kept exactly, and the HSS matrix is SPD (Section 3.2), as its
    dense eigenvalues show."""
    h = small_h2(n=1024, leaf=512, kind="matern32", ell=0.3, shift=1e-3, seed=77)
    T = h.tree
    assert [T.size(v) for v in T.leaves()] == [512, 512]
    om = workloads.gaussian_matrix(1024, 256, 5)[T.perm]
    s = SPDHSS(h, om, 0.0, 246, "chol")
    assert all(s.rank[v] == 246 for v in T.leaves())
    D, A = s.dense(), h.dense()
    for v in T.leaves():
        assert np.array_equal(D[T.rng(v), T.rng(v)], A[T.rng(v), T.rng(v)])
    assert np.linalg.eigvalsh(0.5 * (D + D.T)).min() > 0
    assert np.linalg.norm(D - A) <= 1e-4 * np.linalg.norm(A)


def test_block_jacobi_limit():
    """max_rank = 0 leaves A_hss = blockdiag(A_ii); PCG then follows
    block-Jacobi PCG step for step (compared with SciPy's CG)."""
    h = small_h2(n=300, leaf=20, kind="matern32", ell=0.2, shift=1e-2)
    om = workloads.gaussian_matrix(300, 10, 9)[h.tree.perm]
    s = SPDHSS(h, om, 1e-2, 0, "chol")
    T = h.tree
    Ah = h.dense()
    BJ = np.zeros_like(Ah)
    for v in T.leaves():
        BJ[T.rng(v), T.rng(v)] = Ah[T.rng(v), T.rng(v)]
    np.testing.assert_allclose(s.dense(), BJ, atol=0)
    b = workloads.gaussian_matrix(300, 1, 4)[:, 0]
    bj_inv = np.linalg.inv(BJ)
    for k in (3, 8):
        x, it, _ = pcg(h.matvec, s.solve, b, 0.0, k)
        xs, _ = spla.cg(spla.aslinearoperator(Ah), b, rtol=1e-300, atol=0.0, maxiter=k,
                        M=spla.aslinearoperator(bj_inv))
        assert np.linalg.norm(x - xs) <= 1e-9 * np.linalg.norm(xs)


def test_spdhss_beats_block_jacobi():
    """Qualitative claim of Section 6: PCG with the SPD HSS preconditioner
    converges in fewer iterations than with block Jacobi (the r_max = 0 limit
    of the same construction), both reaching the tolerance."""
    h = small_h2(n=800, leaf=40, kind="matern32", ell=0.2, shift=1e-3, shells=6, per_shell=96)
    om = workloads.gaussian_matrix(800, 40, 12)[h.tree.perm]
    hss = SPDHSS(h, om, 1e-2, 30, "chol")
    bj = SPDHSS(h, om[:, :10], 1e-2, 0, "chol")
    b = workloads.gaussian_matrix(800, 1, 13)[:, 0]
    _, it_h, res_h = pcg(h.matvec, hss.solve, b, 1e-8, 2000)
    _, it_b, res_b = pcg(h.matvec, bj.solve, b, 1e-8, 2000)
    assert res_h[0] <= 1.5e-8 and res_b[0] <= 1.5e-8
    assert it_h[0] < it_b[0]


def test_single_leaf_is_dense_cholesky():
    h = small_h2(n=30, leaf=64)
    assert h.tree.L == 1
    om = workloads.gaussian_matrix(30, 10, 9)
    s = SPDHSS(h, om, 1e-2, 5, "chol")
    b = workloads.gaussian_matrix(30, 2, 4)
    A = h.exact_dense()
    np.testing.assert_allclose(s.solve(b), sla.cho_solve(sla.cho_factor(A, lower=True), b), rtol=1e-12)


def test_nested_solve_matches_dense(hss):
    A = hss.dense()
    b = workloads.gaussian_matrix(A.shape[0], 3, 8)
    x = hss.solve(b)
    ref = np.linalg.solve(A, b)
    assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref)


def test_pcg_matches_scipy_cg(h2s, hss):
    Ah = dense_of(h2s)
    b = workloads.gaussian_matrix(h2s.tree.N, 1, 6)[:, 0]
    for k in (2, 6):
        x, it, _ = pcg(h2s.matvec, None, b, 0.0, k)
        xs, _ = spla.cg(spla.aslinearoperator(Ah), b, rtol=1e-300, atol=0.0, maxiter=k)
        assert it[0] == k
        assert np.linalg.norm(x - xs) <= 1e-10 * np.linalg.norm(xs)
        xp, _, _ = pcg(h2s.matvec, hss.solve, b, 0.0, k)
        Minv = spla.LinearOperator(Ah.shape, matvec=hss.solve)
        xsp, _ = spla.cg(spla.aslinearoperator(Ah), b, rtol=1e-300, atol=0.0, maxiter=k, M=Minv)
        assert np.linalg.norm(xp - xsp) <= 1e-10 * np.linalg.norm(xsp)
    x, it, res = pcg(h2s.matvec, hss.solve, b, 1e-8, 500)
    assert res[0] <= 1e-8 * 1.5


def test_matvec_error_closed_forms():
    """Section 6.1's metric (mean relative 2-norm error over Gaussian vectors)
    on products whose error is known exactly: a product scaled by (1 + d)
    errs by |d| on every vector; one that scales vector j by (1 + d_j) errs by
    the mean of |d_j|; the exact product errs by 0."""
    rng = np.random.default_rng(5)
    A = rng.standard_normal((40, 40))
    ref = lambda X: A @ X  # noqa: E731
    assert matvec_error(ref, ref, 40, nvec=10, seed=1) == 0.0
    assert matvec_error(ref, lambda X: 1.25 * (A @ X), 40, nvec=10, seed=1) == pytest.approx(0.25, rel=1e-14)
    d = np.linspace(-0.3, 0.5, 10)
    err = matvec_error(ref, lambda X: (A @ X) * (1.0 + d)[None, :], 40, nvec=10, seed=1)
    assert err == pytest.approx(np.abs(d).mean(), rel=1e-14)


def test_matvec_error_on_order_of_tau():
    """Sanity range only (parity unpinned): with the threshold form the HSS
    matvec error vs the H^2 product is of the order of tau (Table 4 reports
    0.05-0.06 at 1e-1 and 0.003-0.005 at 1e-2 on its own point sets)."""
    h = small_h2(n=1000, leaf=40, kind="matern32", ell=0.25, shift=1e-2, shells=6, per_shell=96)
    om = workloads.gaussian_matrix(1000, 110, 9)[h.tree.perm]
    errs = {}
    for tau in (1e-1, 1e-2):
        s = SPDHSS(h, om, tau, 100, "chol")
        A = s.dense()
        errs[tau] = matvec_error(h.matvec, lambda X: A @ X, 1000)
    assert 1e-3 < errs[1e-1] < 0.3
    assert 1e-5 < errs[1e-2] < errs[1e-1]


def test_golden_fixture():
    """The oracle reproduces its recorded results (tests/golden/oracle_n300.json,
    written by tests/golden/make_golden.py): integers exactly, norms to 1e-12.
    A change here means the oracle's arithmetic changed."""
    import importlib.util
    import json
    import os
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    spec = importlib.util.spec_from_file_location("make_golden", os.path.join(here, "make_golden.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    with open(os.path.join(here, "oracle_n300.json")) as f:
        want = json.load(f)
    got = json.loads(json.dumps(mod.compute()))
    for key in ("perm", "h2_skeletons", "hss_ranks", "hss_pivots", "pcg_iterations"):
        assert got[key] == want[key], key
    for key in ("matvec_ones_norm", "solution_norm"):
        assert abs(got[key] - want[key]) <= 1e-12 * abs(want[key]), key
