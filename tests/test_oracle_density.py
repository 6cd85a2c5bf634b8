"""Pins of the oracle's two alternative density providers (the estimators
Sec. 5 tried before the octree): the fixed-radius count (naive
estimator) and the k-nearest-neighbour estimate, over one iteration's NEE
vertices.

- a hand-placed configuration gives exact counts, k-th distances, the
  fallback to the fixed-radius estimate and the point's own contribution;
- for a Poisson point process of intensity lambda on a plane, queried at
  points that are not data points, the fixed-radius estimate is unbiased
  (E = lambda) and the k-nearest-neighbour estimate has the closed-form
  mean lambda k / (k - 1) (pi lambda d_k^2 is Gamma(k, 1) distributed);
- at the data points themselves the fixed-radius estimate gains the point
  itself, E = lambda + 1 / (pi R^2);
- rendered with either provider, the white furnace stays near its closed
  form (both estimators are biased; the bound is loose).
"""
import numpy as np
import pytest

from neb_inputs import furnace_sphere


def test_hand_placed_points(oracle):
    dirs = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1], [-1, 0, 0], [0, -1, 0], [0, 0, -1], [1, 1, 0]], float)
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    dist = np.array([0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7])
    pts = dirs * dist[:, None] + np.array([0.3, -0.2, 0.5])
    q = np.array([[0.3, -0.2, 0.5]])
    R = 0.55
    assert oracle.point_density(pts, q, 4, R)[0] == pytest.approx(5 / (np.pi * R * R), rel=1e-14)
    assert oracle.point_density(pts, q, 5, R, k=3)[0] == pytest.approx(3 / (np.pi * 0.3 ** 2), rel=1e-12)
    assert oracle.point_density(pts, q, 5, R, k=5)[0] == pytest.approx(5 / (np.pi * 0.5 ** 2), rel=1e-12)
    # fewer than k within R: the fixed-radius estimate
    assert oracle.point_density(pts, q, 5, R, k=6)[0] == pytest.approx(5 / (np.pi * R * R), rel=1e-14)
    # the ball is open: a point exactly at R does not count (axis points about
    # the origin lie at exactly representable distances)
    axis = dirs[:6] * dist[:6, None]
    assert oracle.point_density(axis, np.zeros((1, 3)), 4, 0.5)[0] == pytest.approx(4 / (np.pi * 0.25), rel=1e-14)
    # a query at a data point counts that point (at distance 0): the nearest
    # other point of pts[0] is pts[1], at |0.1 e_x - 0.2 e_y| = 0.2236
    q2 = pts[:1]
    assert oracle.point_density(pts, q2, 4, 0.15)[0] == pytest.approx(1 / (np.pi * 0.15 ** 2), rel=1e-14)
    assert oracle.point_density(pts, q2, 4, 0.23)[0] == pytest.approx(2 / (np.pi * 0.23 ** 2), rel=1e-14)
    assert oracle.point_density(pts, q2, 5, 0.3, k=2)[0] == pytest.approx(2 / (np.pi * 0.05), rel=1e-12)
    # empty set
    assert oracle.point_density(np.zeros((0, 3)), q, 5, R, k=4)[0] == 0.0


def _poisson_plane(rng, lam, side):
    n = rng.poisson(lam * side * side)
    p = np.zeros((n, 3))
    p[:, 0] = rng.uniform(0, side, n)
    p[:, 2] = rng.uniform(0, side, n)
    p[:, 1] = 0.25
    return p


def test_poisson_closed_forms(oracle):
    rng = np.random.default_rng(21)
    lam, side, R = 2000.0, 3.0, 0.1
    pts = _poisson_plane(rng, lam, side)
    # queries that are not data points, away from the border by more than R
    nq = 3000
    q = np.zeros((nq, 3))
    q[:, 0] = rng.uniform(0.2, side - 0.2, nq)
    q[:, 2] = rng.uniform(0.2, side - 0.2, nq)
    q[:, 1] = 0.25
    naive = oracle.point_density(pts, q, 4, R)
    assert naive.mean() / lam - 1 == pytest.approx(0.0, abs=0.03)
    for k in (4, 8, 16):
        knn = oracle.point_density(pts, q, 5, R, k=k)
        assert knn.mean() / (lam * k / (k - 1)) - 1 == pytest.approx(0.0, abs=0.04), k
    # at the data points the point itself adds 1 / (pi R^2)
    inner = pts[(pts[:, 0] > 0.2) & (pts[:, 0] < side - 0.2) & (pts[:, 2] > 0.2) & (pts[:, 2] < side - 0.2)]
    at = oracle.point_density(pts, inner[:3000], 4, R)
    assert at.mean() / (lam + 1 / (np.pi * R * R)) - 1 == pytest.approx(0.0, abs=0.03)


@pytest.mark.parametrize("mode", [4, 5])
def test_furnace_with_alternative_providers(oracle, mode):
    sc = furnace_sphere(subdiv=4, width=16, height=16, max_path_len=5)
    ref = sum(0.5 ** j for j in range(sc.max_path_len))
    r = oracle.render(sc, n_iter=32, density_mode=mode, enable_photons=True, density_radius=0.2, knn_k=8)
    assert r["tech"]["P"].sum() > 0.03 * r["sum"].sum()
    assert abs(r["mean"].mean() / ref - 1) < 0.1
