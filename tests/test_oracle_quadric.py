"""Pins for the quadric part (Eq. (1)-(4)): the conic box against brute-force
projection of ellipsoid surface points, exact recovery of a known ellipsoid
from its closed-form boxes in three or more views, and the degenerate cases."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from paper_2503_02223_amd import scenes


def _ellipsoid(rng):
    mu = rng.uniform(-0.5, 0.5, 3)
    R = Rotation.random(random_state=int(rng.integers(1 << 30))).as_matrix()
    axes = rng.uniform(0.1, 0.4, 3)
    return mu, R, axes


def test_conic_box_matches_projected_surface(oracle):
    rng = np.random.default_rng(0)
    cams = scenes.ring_cameras(4, radius=2.5)
    for _ in range(5):
        mu, R, axes = _ellipsoid(rng)
        Q = oracle.dual_quadric_from_ellipsoid(mu, R, axes)
        th, ph = np.meshgrid(np.linspace(0, np.pi, 400), np.linspace(0, 2 * np.pi, 800))
        unit = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)]).reshape(3, -1)
        pts = mu[:, None] + R @ (axes[:, None] * unit)
        for cam in cams:
            P = oracle.camera_matrix(cam)
            box = oracle.conic_box(oracle.project_dual_quadric(Q, P))
            h = P @ np.vstack([pts, np.ones(pts.shape[1])])
            uv = h[:2] / h[2]
            bf = np.array([uv[0].min(), uv[1].min(), uv[0].max(), uv[1].max()])
            np.testing.assert_allclose(box, bf, atol=0.05)
            assert box[0] <= bf[0] + 1e-9 and box[1] <= bf[1] + 1e-9
            assert box[2] >= bf[2] - 1e-9 and box[3] >= bf[3] - 1e-9


@pytest.mark.parametrize("n_views", [3, 5, 8])
def test_fit_recovers_ellipsoid_from_closed_form_boxes(oracle, n_views):
    rng = np.random.default_rng(n_views)
    cams = scenes.ring_cameras(n_views, radius=2.5)
    Ps = [oracle.camera_matrix(c) for c in cams]
    objs = [_ellipsoid(rng) for _ in range(4)]
    boxes, bo, bv = [], [], []
    for k, (mu, R, axes) in enumerate(objs):
        Q = oracle.dual_quadric_from_ellipsoid(mu, R, axes)
        for v, P in enumerate(Ps):
            boxes.append(oracle.conic_box(oracle.project_dual_quadric(Q, P)))
            bo.append(k)
            bv.append(v)
    fit = oracle.fit_dual_quadric(np.array(boxes), np.array(bo), np.array(bv), Ps, len(objs))
    assert (fit["status"] == 0).all()
    for k, (mu, R, axes) in enumerate(objs):
        Q = oracle.dual_quadric_from_ellipsoid(mu, R, axes)
        Q = Q / -Q[3, 3]
        np.testing.assert_allclose(fit["Q"][k], Q, atol=1e-8 * np.abs(Q).max())
        np.testing.assert_allclose(fit["mu"][k], mu, atol=1e-8)
        np.testing.assert_allclose(np.sort(fit["axes"][k]), np.sort(axes), rtol=1e-7)
        M = fit["R"][k] @ np.diag(fit["axes"][k] ** 2) @ fit["R"][k].T
        np.testing.assert_allclose(M, R @ np.diag(axes ** 2) @ R.T, atol=1e-9)
        assert np.linalg.det(fit["R"][k]) == pytest.approx(1.0)


def test_two_views_are_degenerate(oracle):
    rng = np.random.default_rng(3)
    cams = scenes.ring_cameras(8, radius=2.5)[:2]
    Ps = [oracle.camera_matrix(c) for c in cams]
    mu, R, axes = _ellipsoid(rng)
    Q = oracle.dual_quadric_from_ellipsoid(mu, R, axes)
    boxes = [oracle.conic_box(oracle.project_dual_quadric(Q, P)) for P in Ps]
    fit = oracle.fit_dual_quadric(np.array(boxes), np.array([0, 0]), np.array([0, 1]), Ps, 2)
    assert fit["status"][0] == oracle.QUADRIC_DEGENERATE
    assert fit["status"][1] == oracle.QUADRIC_DEGENERATE   # no boxes at all


def test_border_edges_are_dropped(oracle):
    cams = scenes.ring_cameras(3, radius=2.5)
    Ps = [oracle.camera_matrix(c) for c in cams]
    rows = oracle.quadric_rows(np.array([[0.5, 10, 100, 200], [5, 5, 639.5, 470]]), Ps,
                               np.array([0, 1]), img_wh=[(640, 480)] * 3)
    assert rows.shape == (3 + 3, 10)
