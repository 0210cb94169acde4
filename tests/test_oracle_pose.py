"""Pins for the camera-pose gradient oracle: central finite differences of the
oracle's render with respect to left perturbations of the camera (rotation
vector w and translation tau), on small scenes, with pixels near a discrete
decision given zero upstream weight (as for the parameter adjoint)."""
import numpy as np
import pytest

from oracle import pose as OP
from paper_2503_02223_amd import scenes


def _setup(oracle, seed, n=24, W=24, H=20, f=30.0):
    sc = scenes.tiny_scene(seed=seed, n=n, width=W, height=H, f=f)
    cam = sc["cams"][0]
    base = oracle.render(sc["params"], sc["ids"], cam, K=sc["K"])
    w = scenes.random_image_grads(300 + seed, (3, H, W), K=sc["K"])
    keep = (base["margin"] > 1e-3) & (base["margin_clamp"] > 1e-3) & (base["depth_gap"] > 1e-4)
    for k in w:
        w[k] = w[k] * keep
    return sc, cam, w


def _loss(oracle, sc, cam, w):
    o = oracle.render(sc["params"], sc["ids"], cam, K=sc["K"])
    return ((w["gC"] * o["C"]).sum() + (w["gD"] * o["D"]).sum() + (w["gT"] * o["Tf"]).sum()
            + (w["gP"] * o["P"]).sum())


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_pose_gradient_matches_central_differences(oracle, seed):
    sc, cam, w = _setup(oracle, seed)
    # a camera that is not the identity, so rotation and translation mix
    cam = OP.perturb_camera(cam, [0.05, -0.03, 0.02], [0.02, -0.01, 0.03])
    base = oracle.render(sc["params"], sc["ids"], cam, K=sc["K"])
    keep = (base["margin"] > 1e-3) & (base["margin_clamp"] > 1e-3) & (base["depth_gap"] > 1e-4)
    for k in w:
        w[k] = w[k] * keep
    grads, _ = oracle.render_backward(sc["params"], sc["ids"], cam, K=sc["K"], **w)
    d_w, d_tau = OP.pose_grad(sc["params"], grads, cam)
    h = 1e-6
    fd = np.zeros(6)
    for j in range(6):
        e = np.zeros(6)
        e[j] = h
        lp = _loss(oracle, sc, OP.perturb_camera(cam, e[:3], e[3:]), w)
        lm = _loss(oracle, sc, OP.perturb_camera(cam, -e[:3], -e[3:]), w)
        fd[j] = (lp - lm) / (2 * h)
    got = np.concatenate([d_w, d_tau])
    assert np.abs(fd).max() > 0
    np.testing.assert_allclose(got, fd, rtol=1e-4, atol=1e-6 * np.abs(fd).max())


def test_pose_gradient_invariant_under_quaternion_sign(oracle):
    """q and -q are the same rotation: same render, same pose gradient (the
    rotation term flips sign with q and with dL/dq together)."""
    sc, cam, w = _setup(oracle, 5)
    grads, _ = oracle.render_backward(sc["params"], sc["ids"], cam, K=sc["K"], **w)
    p2 = sc["params"].copy()
    p2[6:10] = -p2[6:10]          # q and -q are the same rotation: same render, same pose gradient
    g2, _ = oracle.render_backward(p2, sc["ids"], cam, K=sc["K"], **w)
    dw1, _ = OP.pose_grad(sc["params"], grads, cam)
    dw2, _ = OP.pose_grad(p2, g2, cam)
    np.testing.assert_allclose(dw2, dw1, rtol=1e-10, atol=1e-14)
