"""Oracle of the camera-pose gradient used for tracking (test infrastructure
only; numpy, FP64).

The paper tracks the camera with the same differentiable rasterizer (Sec.
IV: tracking and mapping run on the GPU).  The pose of view v is x_c = R x_w
+ t; it is perturbed on the left, in the camera frame: R' = exp([w]x) R,
t' = exp([w]x) t + tau, and the gradient is dL/d(w, tau) at w = tau = 0.

The gradient is obtained from the per-Gaussian gradients of the render
through the rigid-motion identity: moving the camera by (w, tau) renders
exactly what moving every Gaussian by the world-frame motion
x -> R^T (exp([w]x)(R x + t) + tau - t) renders with the camera fixed (the
means move with it; each rotation is multiplied on the left by
R^T exp([w]x) R = exp([R^T w]x)).  Hence, with g_i = R dL/dmu_i (the gradient
with respect to the camera-frame mean p_i = R mu_i + t),
  dL/dtau = sum_i g_i,
  dL/dw   = sum_i p_i x g_i + R sum_i dL/dphi_i,
where phi is a world-frame left rotation of Gaussian i's quaternion q = (s, u):
d(q_phi * q)/dphi = 1/2 [-u^T; s I - [u]x], so
dL/dphi = 1/2 (-u dL/ds + s dL/du + u x dL/du).
"""
from __future__ import annotations

import numpy as np


def pose_grad(params, dparams, cam):
    """dL/dw (3) and dL/dtau (3) of one view from the parameters (14, n) and
    the per-Gaussian gradients (14, n) of the loss rendered through `cam`."""
    p = np.asarray(params, np.float64)
    d = np.asarray(dparams, np.float64)
    R = np.asarray(cam["R"], np.float64).reshape(3, 3)
    t = np.asarray(cam["t"], np.float64).reshape(3)
    pc = R @ p[0:3] + t[:, None]
    g = R @ d[0:3]
    d_tau = g.sum(axis=1)
    d_w = np.cross(pc.T, g.T).sum(axis=0)
    s, u = p[6], p[7:10]
    ds, du = d[6], d[7:10]
    dphi = 0.5 * (-u * ds[None] + s[None] * du + np.cross(u.T, du.T).T)
    d_w = d_w + R @ dphi.sum(axis=1)
    return d_w, d_tau


def perturb_camera(cam, w, tau):
    """The camera with R' = exp([w]x) R and t' = exp([w]x) t + tau."""
    from scipy.spatial.transform import Rotation
    E = Rotation.from_rotvec(np.asarray(w, np.float64)).as_matrix()
    out = dict(cam)
    out["R"] = E @ np.asarray(cam["R"], np.float64).reshape(3, 3)
    out["t"] = E @ np.asarray(cam["t"], np.float64).reshape(3) + np.asarray(tau, np.float64)
    return out
