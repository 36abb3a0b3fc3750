"""The seeded input generators (CPU): shapes, determinism and the
distributions they claim."""
import numpy as np
import pytest

import workloads


@pytest.mark.parametrize("kind", ["cube", "sphere", "ball"])
def test_points_are_seeded_and_shaped(kind):
    a = workloads.points(kind, 1000, 5)
    b = workloads.points(kind, 1000, 5)
    assert a.shape == (1000, 3) and a.dtype == np.float64 and a.flags.c_contiguous
    assert np.array_equal(a, b)
    assert not np.array_equal(a, workloads.points(kind, 1000, 6))


def test_point_set_supports():
    c = workloads.points("cube", 20000, 1)
    assert c.min() >= 0.0 and c.max() < 1.0
    s = np.linalg.norm(workloads.points("sphere", 20000, 1), axis=1)
    assert np.allclose(s, 1.0, rtol=0, atol=1e-14)
    r = np.linalg.norm(workloads.points("ball", 20000, 1), axis=1)
    assert r.max() <= 1.0


def test_ball_has_constant_density():
    """Uniform in the unit ball: P(|x| <= t) = t^3, and the directions are
    isotropic (mean near 0)."""
    x = workloads.points("ball", 200000, 3)
    r = np.linalg.norm(x, axis=1)
    for t in (0.25, 0.5, 0.75, 0.9):
        frac = float(np.mean(r <= t))
        assert abs(frac - t ** 3) <= 5 * np.sqrt(t ** 3 * (1 - t ** 3) / len(r)) + 1e-12
    assert np.abs(x.mean(axis=0)).max() <= 0.01


def test_gaussian_matrix_is_column_major():
    g = workloads.gaussian_matrix(100, 3, 9)
    assert g.shape == (100, 3) and g.flags.f_contiguous
    assert np.array_equal(g, workloads.gaussian_matrix(100, 3, 9))


def test_batch_recipe():
    inst = workloads.batch_instances()
    assert len(inst) == 64
    ns = np.array([w.n for w in inst])
    assert ns.min() >= 5000 and ns.max() <= 50000
    # log-uniform: the median sits near the geometric mean of the range
    assert abs(np.log(np.median(ns)) - 0.5 * (np.log(5000) + np.log(50000))) < 0.35
    assert [w.point_set for w in inst] == ["cube", "sphere"] * 32
    assert {(w.kernel, w.ell) for w in inst} == set(workloads.BATCH_KERNELS)
    for w in inst:
        assert (w.shift, w.leaf, w.hss_tol, w.max_rank, w.oversample, w.nrhs, w.pcg_tol) == \
            (1e-3, 128, 1e-2, 100, 10, 4, 1e-8)
    assert len({w.seed_base for w in inst}) == 64  # every instance draws its own data
    assert [w.name for w in workloads.batch_instances()] == [w.name for w in inst]  # seeded


def test_serve_recipe():
    reqs = workloads.serve_requests()
    assert len(reqs) == 64
    t = np.array([a for a, _, _ in reqs])
    assert np.all(np.diff(t) > 0)
    # Poisson arrivals at 20/s: 64 exponential gaps with mean 0.05 s
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert 0.03 < gaps.mean() < 0.07 and gaps.std() / gaps.mean() > 0.6
    ws = [w for _, w, _ in reqs]
    assert [k for _, _, k in reqs] == list(range(1, 65))  # no repeats: every request its own matrix
    assert all(10_000 <= w.n <= 1_000_000 and w.point_set == "cube" for w in ws)  # the served range
    assert {w.kernel for w in ws} == set(workloads.SERVE_KERNELS)
    assert all(0.05 <= w.ell <= 0.5 and 1 <= w.nrhs <= 32 for w in ws)
    assert all((w.shift, w.leaf, w.pcg_tol) == (1e-3, 400, 1e-8) for w in ws)


def test_serve_recipe_with_repeats():
    # the served trace over the full size range, a quarter of the requests on
    # an earlier request's matrix with new right-hand sides
    reqs = workloads.serve_requests(count=256, n_hi=1_000_000, repeat=0.25)
    ws = {k: w for _, w, k in reqs if w.rhs_seed is None}
    reps = [(w, k) for _, w, k in reqs if w.rhs_seed is not None]
    assert 30 < len(reps) < 100
    assert all(10_000 <= w.n <= 1_000_000 for _, w, _ in reqs)
    assert max(w.n for _, w, _ in reqs) > 300_000
    for w, k in reps:
        base = ws[k]  # the matrix of the request it names
        assert (w.n, w.kernel, w.ell, w.seed_base, w.point_set) == (base.n, base.kernel, base.ell, base.seed_base,
                                                                    base.point_set)
        assert np.array_equal(w.points()[:5], base.points()[:5])
        assert not np.array_equal(w.rhs()[:5, 0], base.rhs()[:5, 0]) or w.nrhs != base.nrhs
    # without repeats the trace is the one above
    assert [w.name for _, w, _ in workloads.serve_requests()] == \
        [w.name for _, w, _ in workloads.serve_requests(repeat=0.0)]
