"""The bound that lets the device evaluate the three FE maps over one
common denominator without clamping its factors: ln prod_{i,j} D_ij, with
D_ij = 1 + exp(2 xi (w_i - nu_ij)), is convex in w, so over the simplex of
weights it peaks at a vertex.  Checked against random points of the simplex
and the vertices' value at the paper's xi = 100 (below the 600 the device
path allows) with the null points of eq. 21 at kappa = 0.5 (the band edges of
the sharp-limit maps: 1/32, 27/352, 6/11 | 5/16, 31/48, 26/33, 21/22 |
5/32, 31/96, 2/3)."""
import numpy as np
import pytest

NU = [np.array([1 / 32, 27 / 352, 6 / 11]), np.array([5 / 16, 31 / 48, 26 / 33, 21 / 22]),
      np.array([5 / 32, 31 / 96, 2 / 3])]


def log_den(w, xi):
    """ln of the product of the three maps' denominators at weights w (n, 3)."""
    return sum(np.logaddexp(0.0, 2 * xi * (w[:, i:i + 1] - NU[i][None, :])).sum(1) for i in range(3))


def vertex_bound(xi):
    return max(log_den(np.eye(3)[i:i + 1], xi)[0] for i in range(3))


@pytest.mark.parametrize("xi", [10.0, 100.0, 120.0, 300.0])
def test_simplex_maximum_is_at_a_vertex(xi):
    rng = np.random.default_rng(5)
    w = rng.dirichlet(np.full(3, 0.3), size=200000)
    w = np.vstack([w, np.eye(3) * (1 - 1e-12) + 1e-12 / 3])
    assert log_den(w, xi).max() <= vertex_bound(xi) + 1e-9


def test_paper_steepness_is_inside_the_unclamped_range():
    assert vertex_bound(100.0) == pytest.approx(469.318, abs=1e-3)
    assert vertex_bound(120.0) < 600.0 < vertex_bound(130.0)
