"""Pins of the RPY tensor kernel and of the oracle's H^2 / SPD-HSS on it (CPU).

The tensor of Section 6 (particle radius a, normalized so that the self term
is I / a) is pinned to properties the formula does not state directly:
symmetry, continuity where its two branches meet (|r| = 2a), the Oseen limit
far away, the isotropic self term, and positive definiteness of the 3N x 3N
matrix for any particle configuration, overlapping ones included (the RPY
construction's defining property).  The H^2 form is then checked against the
dense matrix, and the SPD HSS preconditioner against SPD-ness and PCG."""
import numpy as np
import pytest

import workloads
from oracle import kernels
from oracle.h2 import H2
from oracle.pcg import pcg
from oracle.spdhss import SPDHSS


def tensor(a, r):
    """The 3 x 3 tensor at separation r (one particle pair)."""
    X = np.zeros((3, 3))
    Y = np.tile(-np.asarray(r, dtype=np.float64), (3, 1))  # x - y = r
    c = np.arange(3)
    return kernels.evaluate("rpy", a, X, Y, c, c)


@pytest.mark.parametrize("r", [[0.1, 0.0, 0.0], [0.3, -0.2, 0.5], [2.0, 1.0, -3.0]])
def test_symmetric_and_even(r):
    T = tensor(0.29, r)
    assert np.allclose(T, T.T, rtol=0, atol=1e-15)
    assert np.allclose(T, tensor(0.29, -np.asarray(r)), rtol=0, atol=1e-15)


def test_self_term_and_isotropy():
    a = 0.42
    assert np.array_equal(tensor(a, [0.0, 0.0, 0.0]), np.eye(3) / a)
    # rotating r rotates the tensor: T(Q r) = Q T(r) Q^T
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    for rr in ([0.5, 0.1, 0.2], [1.5, -0.7, 0.4]):
        r = np.asarray(rr)
        assert np.allclose(tensor(a, Q @ r), Q @ tensor(a, r) @ Q.T, rtol=0, atol=1e-13)


@pytest.mark.parametrize("a", [0.29, 0.42])
def test_branches_meet_at_two_radii(a):
    u = np.array([0.6, -0.48, 0.64])  # unit vector
    inside = tensor(a, 2 * a * (1 - 1e-12) * u)
    outside = tensor(a, 2 * a * u)
    assert np.allclose(inside, outside, rtol=1e-9, atol=0)
    # the common value: 7/(16a) I + 3/(16a) u u^T
    assert np.allclose(outside, 7 / (16 * a) * np.eye(3) + 3 / (16 * a) * np.outer(u, u), rtol=1e-14, atol=0)


def test_oseen_limit_far_away():
    a = 0.29
    u = np.array([2.0, -1.0, 2.0]) / 3.0
    for dist in (10.0, 100.0, 1000.0):
        T = tensor(a, dist * u)
        oseen = 0.75 / dist * (np.eye(3) + np.outer(u, u))
        # the next term is O(a^2 / dist^3)
        assert np.abs(T - oseen).max() <= 1.5 * a * a / dist ** 3 * 1.0001


@pytest.mark.parametrize("a,seed", [(0.29, 1), (0.42, 2), (1.5, 3)])
def test_matrix_is_spd_with_overlaps(a, seed):
    # 80 particles in a small box: many pairs overlap (|r| < 2a)
    rng = np.random.default_rng(seed)
    X = rng.random((80, 3)) * 2.0
    P = np.repeat(X, 3, axis=0)
    c = np.tile(np.arange(3), 80)
    A = kernels.evaluate("rpy", a, P, P, c, c)
    assert np.allclose(A, A.T, rtol=0, atol=1e-14)
    lam = np.linalg.eigvalsh(A)
    assert lam.min() > 0.0
    d = np.sqrt(((X[:, None, :] - X[None, :, :]) ** 2).sum(-1))
    assert (d[np.triu_indices(80, 1)] < 2 * a).sum() > 10  # the overlapping branch is exercised


def test_h2_matches_dense_rpy():
    # 2,000 particles of radius 0.29 at unit density (6,000 rows): the upper
    # levels compress, the realized error stays at the ID tolerance
    w = workloads.RPY_SMALL.with_(n=2000, leaf=90)
    h = H2(w.points(), w.kernel, w.ell, w.shift, w.leaf, w.h2_tol, eta=w.eta)
    assert h.tree.N == 3 * w.n
    A, E = h.dense(), h.exact_dense()
    err = np.linalg.norm(A - E) / np.linalg.norm(E)
    T = h.tree
    compressed = [v for v in range(1, T.nnodes) if 0 < h.rank(v) < len(h.candidates(v))]
    assert compressed
    assert err <= 10 * w.h2_tol
    # rows are point components: the diagonal of the dense matrix is 1/a
    assert np.allclose(np.diag(E), 1 / w.ell, rtol=0, atol=1e-14)


def test_spdhss_and_pcg_on_rpy():
    w = workloads.RPY_SMALL
    h = H2(w.points(), w.kernel, w.ell, w.shift, w.leaf, w.h2_tol, eta=w.eta)
    s = SPDHSS(h, w.omega()[h.tree.perm], w.hss_tol, w.max_rank, "chol")
    M = s.dense()
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > 0.0
    b = w.rhs()[h.tree.perm]
    x, it, res = pcg(h.matvec, s.solve, b, w.pcg_tol, 300)
    E = h.exact_dense()
    assert np.linalg.norm(E @ x - b) / np.linalg.norm(b) <= 2 * w.pcg_tol
    assert it[0] < 100
