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
