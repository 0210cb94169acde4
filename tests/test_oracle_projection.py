"""Pins for the oracle's EWA projection (the Gaussian = quadric shape of Eq. (2)).

Independent references: a closed form on the optical axis, a finite-difference
Jacobian of the pinhole map, and scipy's quaternion-to-rotation routine."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from paper_2503_02223_amd import scenes


def _one(mu, ls, q, eta=0.0, rgb=(1, 1, 1)):
    return scenes.pack(np.asarray(mu, float).reshape(3, 1), np.asarray(ls, float).reshape(3, 1),
                       np.asarray(q, float).reshape(4, 1), np.array([eta]), np.asarray(rgb, float).reshape(3, 1))


@pytest.mark.parametrize("z,s", [(3.0, 0.05), (1.0, 0.01), (7.5, 0.2)])
def test_on_axis_isotropic_closed_form(oracle, z, s):
    cam = scenes.camera(fx=110, fy=110, cx=64, cy=48)
    rng = np.random.default_rng(1)
    q = rng.normal(size=4)  # isotropic: rotation must not matter
    p = _one([0, 0, z], [np.log(s)] * 3, q)
    pr = oracle.project(p, cam)
    assert pr["visible"][0]
    assert pr["mx"][0] == pytest.approx(64.0, abs=1e-12)
    assert pr["my"][0] == pytest.approx(48.0, abs=1e-12)
    var = (110 * s / z) ** 2 + 0.3
    assert pr["s00"][0] == pytest.approx(var, rel=1e-12)
    assert pr["s11"][0] == pytest.approx(var, rel=1e-12)
    assert abs(pr["s01"][0]) < 1e-12 * var
    assert pr["A"][0] == pytest.approx(1 / var, rel=1e-12)
    assert pr["ex"][0] == pytest.approx(3 * np.sqrt(var), rel=1e-12)


def _pix(cam, p):
    return np.array([cam["fx"] * p[0] / p[2] + cam["cx"], cam["fy"] * p[1] / p[2] + cam["cy"]])


def test_off_axis_covariance_matches_fd_jacobian_and_scipy_rotation(oracle):
    rng = np.random.default_rng(7)
    cam = scenes.look_at([0.3, -0.2, -3.0], [0.1, 0.2, 0.5], fx=300, fy=280, cx=160, cy=120,
                         width=320, height=240)
    for _ in range(20):
        mu = rng.uniform(-1, 1, 3) + np.array([0, 0, 0.5])
        ls = rng.normal(-2, 0.5, 3)
        q = rng.normal(size=4)
        pr = oracle.project(_one(mu, ls, q), cam)
        W = cam["R"]
        pc = W @ mu + cam["t"]
        h = 1e-6
        Jfd = np.stack([(_pix(cam, pc + h * e) - _pix(cam, pc - h * e)) / (2 * h) for e in np.eye(3)], axis=1)
        qn = q / np.linalg.norm(q)
        Rq = Rotation.from_quat([qn[1], qn[2], qn[3], qn[0]]).as_matrix()
        S3 = Rq @ np.diag(np.exp(2 * ls)) @ Rq.T
        S2 = Jfd @ W @ S3 @ W.T @ Jfd.T + 0.3 * np.eye(2)
        got = np.array([[pr["s00"][0], pr["s01"][0]], [pr["s01"][0], pr["s11"][0]]])
        np.testing.assert_allclose(got, S2, rtol=1e-7, atol=1e-9 * np.abs(S2).max())
        np.testing.assert_allclose(_pix(cam, pc), [pr["mx"][0], pr["my"][0]], rtol=1e-12)
        inv = np.linalg.inv(S2)
        np.testing.assert_allclose([pr["A"][0], pr["B"][0], pr["C"][0]], [inv[0, 0], inv[0, 1], inv[1, 1]],
                                   rtol=1e-6)
        assert pr["z"][0] == pytest.approx(pc[2], rel=1e-12)


def test_culling_near_plane_and_behind(oracle):
    cam = scenes.camera()
    p = np.concatenate([_one([0, 0, 0.1], [-3] * 3, [1, 0, 0, 0]), _one([0, 0, -2], [-3] * 3, [1, 0, 0, 0]),
                        _one([0, 0, 0.25], [-3] * 3, [1, 0, 0, 0])], axis=1)
    pr = oracle.project(p, cam)
    assert list(pr["visible"]) == [False, False, True]


@pytest.mark.parametrize("ratio", [(0.9, 0.1), (-1.2, 0.3), (0.2, -0.95), (1.5, 1.4)])
def test_jacobian_frustum_limit(oracle, ratio):
    """Outside 1.3x the half field of view the Jacobian is that of the pinhole
    map at the point moved onto the limit (x/z, y/z clamped, z kept); the 2D
    mean stays the unclamped projection."""
    cam = scenes.camera(fx=110, fy=100, cx=64, cy=48, width=128, height=96)
    lx, ly = 1.3 * 0.5 * 128 / 110, 1.3 * 0.5 * 96 / 100
    z = 2.5
    pc = np.array([ratio[0] * z, ratio[1] * z, z])
    rng = np.random.default_rng(5)
    ls, q = rng.normal(-1.5, 0.3, 3), rng.normal(size=4)
    pr = oracle.project(_one(pc, ls, q), cam)
    clamped = np.array([np.clip(ratio[0], -lx, lx) * z, np.clip(ratio[1], -ly, ly) * z, z])
    h = 1e-6
    Jfd = np.stack([(_pix(cam, clamped + h * e) - _pix(cam, clamped - h * e)) / (2 * h) for e in np.eye(3)], axis=1)
    qn = q / np.linalg.norm(q)
    Rq = Rotation.from_quat([qn[1], qn[2], qn[3], qn[0]]).as_matrix()
    S2 = Jfd @ Rq @ np.diag(np.exp(2 * ls)) @ Rq.T @ Jfd.T + 0.3 * np.eye(2)
    got = np.array([[pr["s00"][0], pr["s01"][0]], [pr["s01"][0], pr["s11"][0]]])
    np.testing.assert_allclose(got, S2, rtol=1e-7, atol=1e-9 * np.abs(S2).max())
    np.testing.assert_allclose([pr["mx"][0], pr["my"][0]], _pix(cam, pc), rtol=1e-12)
