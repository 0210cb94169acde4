"""GPU parity of the camera-pose gradient (tracking): dqo_pose_backward
against the oracle's pose gradient (from its own adjoint through the
rigid-motion identity, itself pinned by finite differences), for one view
and for two views in one frame, in FP32 and FP64, and bitwise
reproducibility.  The pose gradient is a sum over all Gaussians, so the
tolerance is relative to the sum of the magnitudes of their contributions."""
import numpy as np
import pytest
import torch

from oracle import pose as OP
from paper_2503_02223_amd import binding as B
from paper_2503_02223_amd import scenes
from tests.gpu_util import to_dev, unambiguous

pytestmark = pytest.mark.gpu


def _upstream(seed, ref, H, W, K, keep):
    rng = np.random.default_rng(seed)
    g = dict(gC=rng.normal(size=(3, H, W)), gD=rng.normal(size=(H, W)), gT=rng.normal(size=(H, W)),
             gP=rng.normal(size=(K, H, W)))
    return {k: v * keep for k, v in g.items()}


def _oracle_pose(oracle, params, ids, cam, K, up):
    grads, _ = oracle.render_backward(params, ids, cam, K=K, **up)
    d_w, d_tau = OP.pose_grad(params, grads, cam)
    scale = np.zeros(6)
    for i in range(params.shape[1]):      # sum of |contribution| of every Gaussian
        a, b = OP.pose_grad(params[:, i:i + 1], grads[:, i:i + 1], cam)
        scale += np.abs(np.concatenate([a, b]))
    return np.concatenate([d_w, d_tau]), scale


def _cams(sc, views):
    cams = [OP.perturb_camera(sc["cams"][0], [0.04, -0.03, 0.02], [0.05, -0.02, 0.1])]
    if views == 2:
        cams.append(OP.perturb_camera(sc["cams"][0], [-0.03, 0.05, -0.01], [-0.08, 0.03, -0.05]))
    return cams


@pytest.mark.parametrize("views,dtype,rtol", [(1, torch.float32, 2e-3), (2, torch.float32, 2e-3),
                                              (1, torch.float64, 1e-9)])
def test_pose_gradient_parity(oracle, views, dtype, rtol):
    sc = scenes.single_view_scene(seed=11, n=2000)
    cams = _cams(sc, views)
    K, H, W = sc["K"], cams[0]["height"], cams[0]["width"]
    r = B.Rasterizer(cams, sc["params"].shape[1], K, dtype=dtype)
    p = to_dev(sc["params"], dtype)
    ids = torch.tensor(sc["ids"], device="cuda")
    img = r.forward(p, ids, probs=True)
    ups = []
    for v, cam in enumerate(cams):
        ref = oracle.render(sc["params"], sc["ids"], cam, K=K)
        ups.append(_upstream(40 + v, ref, H, W, K, unambiguous(ref, grads=True)))
    grads = dict(d_color=to_dev(np.stack([u["gC"] for u in ups]), dtype),
                 d_depth=to_dev(np.stack([u["gD"] for u in ups]), dtype),
                 d_t_final=to_dev(np.stack([u["gT"] for u in ups]), dtype),
                 d_probs=to_dev(np.stack([u["gP"] for u in ups]), dtype))
    r.frame.render_backward(img, grads)
    pg = r.frame.pose_backward(p).cpu().numpy()
    pg2 = r.frame.pose_backward(p).cpu().numpy()
    assert np.array_equal(pg, pg2)
    for v, cam in enumerate(cams):
        want, scale = _oracle_pose(oracle, sc["params"], sc["ids"], cam, K, ups[v])
        assert (np.abs(pg[v] - want) <= rtol * scale + 1e-12).all(), (v, pg[v], want, scale)
        assert np.abs(want).max() > 1e-3 * scale.max()   # not a sum that cancels to noise


def test_pose_descent_reduces_the_loss_on_the_device(oracle):
    """A few steps of gradient descent on the pose of a displaced camera,
    with the pose gradient from the device, reduce the object loss against
    the frame rendered from the true pose (a property at any size)."""
    sc = scenes.single_view_scene(seed=12, n=2000)
    true_cam = sc["cams"][0]
    tg = oracle.render(sc["params"], sc["ids"], true_cam, K=sc["K"])
    tid = oracle.id_map(tg["P"], tg["Tf"]).astype(np.int32)
    targets = dict(color=to_dev(tg["C"][None]), depth=to_dev(tg["D"][None]), id=torch.tensor(tid[None], device="cuda"))
    p = to_dev(sc["params"])
    ids = torch.tensor(sc["ids"], device="cuda")
    cam = OP.perturb_camera(true_cam, [0.0, 0.01, 0.0], [0.03, -0.02, 0.0])
    losses = []
    w, tau = np.zeros(3), np.zeros(3)
    for it in range(25):
        c = OP.perturb_camera(cam, w, tau)
        r = B.Rasterizer([c], p.shape[1], sc["K"])
        img = r.forward(p, ids, target=targets["id"])
        gi = dict(d_color=torch.empty_like(img["color"]), d_depth=torch.empty_like(img["depth"]),
                  d_p_target=torch.empty_like(img["depth"]))
        loss = torch.zeros(4, dtype=torch.float64, device="cuda")
        r.frame.object_loss(img, targets, gi, loss)
        r.frame.render_backward(img, gi)
        g = r.frame.pose_backward(p).cpu().numpy()[0]
        losses.append(float(loss[0]))
        # a left perturbation composes on the left: step in (w, tau) of the current camera
        cam = c
        w, tau = -0.001 * np.sign(g[:3]), -0.002 * np.sign(g[3:])
    assert min(losses[-5:]) < 0.8 * losses[0]


def test_pose_gradient_full_size_descent_direction():
    """At the tracking workload's size (200k Gaussians, 640x480) the device
    pose gradient is a descent direction of the device loss: a small step
    along -g lowers it and a step along +g raises it."""
    sc = scenes.slam_view_scene(seed=0, n=200_000)
    true_cam = sc["cams"][0]
    n, K = sc["params"].shape[1], sc["K"]
    p = to_dev(sc["params"])
    ids = torch.tensor(sc["ids"], device="cuda")
    r0 = B.Rasterizer([true_cam], n, K, ctx=B.Context(tile_w=8, tile_h=8))
    t0 = r0.forward(p, ids, probs=True, id_map=True)
    targets = dict(color=t0["color"].clone(), depth=t0["depth"].clone(), id=t0["id_map"].clone())
    cam = OP.perturb_camera(true_cam, [0.004, -0.003, 0.002], [0.02, -0.015, 0.01])

    def loss_and_grad(c, want_grad):
        r = B.Rasterizer([c], n, K, ctx=B.Context(tile_w=8, tile_h=8))
        img = r.forward(p, ids, target=targets["id"])
        gi = dict(d_color=torch.empty_like(img["color"]), d_depth=torch.empty_like(img["depth"]),
                  d_p_target=torch.empty_like(img["depth"]))
        loss = torch.zeros(4, dtype=torch.float64, device="cuda")
        r.frame.object_loss(img, targets, gi, loss)
        g = None
        if want_grad:
            r.frame.render_backward(img, gi)
            g = r.frame.pose_backward(p).cpu().numpy()[0]
        return float(loss[0]), g

    L0, g = loss_and_grad(cam, True)
    assert np.isfinite(g).all() and np.abs(g).max() > 0
    step = 2e-4 * g / np.linalg.norm(g)
    Lm, _ = loss_and_grad(OP.perturb_camera(cam, -step[:3], -step[3:]), False)
    Lp, _ = loss_and_grad(OP.perturb_camera(cam, step[:3], step[3:]), False)
    assert Lm < L0 < Lp, (Lm, L0, Lp)
