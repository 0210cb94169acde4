"""Oracle of the quadric pose refinement (test infrastructure only; numpy,
FP64).

Sec. III-E (object pose training loss), Eq. (9): the quadric of every object
is optimised so that its projected box matches the observed 2D boxes of the
frames that see it.  The projection is Eq. (4)'s dual conic C* = P Q* P^T
(read with the transpose on the right), Q* = Z diag(a^2, b^2, c^2, -1) Z^T
with Z = [[R, mu], [0, 1]] (Eq. (2)-(3)), and the box is the conic's
axis-aligned tangent box.

Readings: the loss of object k is J_k = sum over its boxes of (1 - IoU) (Eq. (9)
writes the sum of IoU, which is maximised); the predicted box is clipped to
the image [0, W] x [0, H] when the image size is given (observed boxes are
clipped by construction); a box whose conic is not an ellipse in front of the
camera (C*_33 >= 0, or no real tangent) counts 1 with no gradient; the
parameters are the centre mu, a quaternion q (w, x, y, z; normalised when
used) and log semi-axes; they are optimised by Adam (PyTorch's update, one
learning rate per group).

The gradient is not derived by hand here: it is the complex-step derivative
(Squire and Trapp, 1998) of the forward, which for code built from real-
analytic operations gives the derivative to rounding, with comparisons taken
on real parts.
"""
from __future__ import annotations

import numpy as np

N_PARAMS = 10          # mu (3), q (4), log-axes (3)
DEFAULTS = dict(iterations=100, lr_mu=0.01, lr_rot=0.01, lr_axes=0.01, beta1=0.9, beta2=0.999, eps=1e-15)


def quat_to_rot(q):
    """Rotation matrix of the quaternion q = (w, x, y, z) after normalisation
    (the usual unit-quaternion formula); works on complex input."""
    n = np.sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3])
    w, x, y, z = q[0] / n, q[1] / n, q[2] / n, q[3] / n
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def rot_to_quat(R):
    """A quaternion (w, x, y, z) of the rotation R (scipy's conversion)."""
    from scipy.spatial.transform import Rotation
    x, y, z, w = Rotation.from_matrix(np.asarray(R, np.float64)).as_quat()
    return np.array([w, x, y, z])


def pack(mu, R, axes):
    return np.concatenate([np.asarray(mu, np.float64), rot_to_quat(R), np.log(np.asarray(axes, np.float64))])


def unpack(theta):
    theta = np.asarray(theta)
    return theta[0:3], quat_to_rot(theta[3:7]), np.exp(theta[7:10])


def _re(x):
    return np.real(x)


def predicted_box(theta, P, wh=None):
    """Box (x0, y0, x1, y1) of the quadric theta seen by camera P (3x4), and
    whether it is defined.  Complex theta is carried through."""
    mu, R, ax = unpack(theta)
    P = np.asarray(P, np.float64)
    G = np.zeros((3, 4), dtype=np.result_type(theta, np.float64))
    G[:, :3] = P[:, :3] @ R
    G[:, 3] = P[:, :3] @ mu + P[:, 3]
    w = np.array([ax[0] ** 2, ax[1] ** 2, ax[2] ** 2, -1.0 + 0 * ax[0]])
    C = (G * w[None, :]) @ G.T                      # P Q* P^T with Q* = Z diag(w) Z^T, G = P Z
    if _re(C[2, 2]) >= 0:
        return None
    c = C / C[2, 2]
    dx2 = c[0, 2] * c[0, 2] - c[0, 0]
    dy2 = c[1, 2] * c[1, 2] - c[1, 1]
    if _re(dx2) <= 0 or _re(dy2) <= 0:
        return None
    dx, dy = np.sqrt(dx2), np.sqrt(dy2)
    b = [c[0, 2] - dx, c[1, 2] - dy, c[0, 2] + dx, c[1, 2] + dy]
    if wh is not None:
        lim = (wh[0], wh[1], wh[0], wh[1])
        for i in range(4):
            if _re(b[i]) < 0:
                b[i] = 0 * b[i]
            elif _re(b[i]) > lim[i]:
                b[i] = lim[i] + 0 * b[i]
    return b


def iou(b, o):
    """Intersection over union of boxes b and o (x0, y0, x1, y1); complex b is
    carried through, comparisons on real parts."""
    lo_x = b[0] if _re(b[0]) > o[0] else o[0] + 0 * b[0]
    hi_x = b[2] if _re(b[2]) < o[2] else o[2] + 0 * b[2]
    lo_y = b[1] if _re(b[1]) > o[1] else o[1] + 0 * b[1]
    hi_y = b[3] if _re(b[3]) < o[3] else o[3] + 0 * b[3]
    iw = hi_x - lo_x
    ih = hi_y - lo_y
    if _re(iw) <= 0 or _re(ih) <= 0:
        return 0 * b[0]
    inter = iw * ih
    union = (b[2] - b[0]) * (b[3] - b[1]) + (o[2] - o[0]) * (o[3] - o[1]) - inter
    return inter / union


def loss(theta, boxes, Ps, views, img_wh=None):
    """J of one object: sum over its observed boxes of 1 - IoU (Eq. (9))."""
    J = 0.0 * theta[0]
    for o, v in zip(np.asarray(boxes, np.float64), views):
        b = predicted_box(theta, Ps[v], None if img_wh is None else img_wh[v])
        J = J + 1.0 - (0.0 if b is None else iou(b, o))
    return J


def grad(theta, boxes, Ps, views, img_wh=None, h=1e-30):
    """dJ/dtheta by complex step: Im J(theta + i h e_j) / h for each j."""
    theta = np.asarray(theta, np.float64)
    g = np.zeros(N_PARAMS)
    for j in range(N_PARAMS):
        t = theta.astype(np.complex128)
        t[j] += 1j * h
        g[j] = np.imag(loss(t, boxes, Ps, views, img_wh)) / h
    return g


def kink_margin(theta, boxes, Ps, views, img_wh=None):
    """Smallest distance (px) of a predicted box edge to the observed edge it
    is compared with, or to the image border when clipping applies: where it
    is tiny the two sides of a comparison are a rounding apart."""
    m = np.inf
    for o, v in zip(np.asarray(boxes, np.float64), views):
        wh = None if img_wh is None else img_wh[v]
        b = predicted_box(theta, Ps[v], None)
        if b is None:
            continue
        b = np.real(np.asarray(b))
        m = min(m, np.abs(b - o).min())
        if wh is not None:
            m = min(m, np.abs(b[[0, 2]]).min(), np.abs(b[[1, 3]]).min(), np.abs(b[[0, 2]] - wh[0]).min(),
                    np.abs(b[[1, 3]] - wh[1]).min())
    return m


def refine(theta0, boxes, Ps, views, img_wh=None, **hp):
    """Adam on theta for `iterations` steps (PyTorch's update with bias
    correction; learning rate lr_mu for mu, lr_rot for q, lr_axes for the
    log-axes).  Returns the final theta, J before and after, the per-step J
    and the smallest kink margin met on the way."""
    c = {**DEFAULTS, **hp}
    theta = np.asarray(theta0, np.float64).copy()
    lr = np.array([c["lr_mu"]] * 3 + [c["lr_rot"]] * 4 + [c["lr_axes"]] * 3)
    m = np.zeros(N_PARAMS)
    v = np.zeros(N_PARAMS)
    hist = []
    margin = np.inf
    b1, b2 = c["beta1"], c["beta2"]
    for step in range(1, c["iterations"] + 1):
        hist.append(float(np.real(loss(theta, boxes, Ps, views, img_wh))))
        margin = min(margin, kink_margin(theta, boxes, Ps, views, img_wh))
        g = grad(theta, boxes, Ps, views, img_wh)
        m = b1 * m + (1 - b1) * g
        v = b2 * v + (1 - b2) * g * g
        theta = theta - lr * (m / (1 - b1 ** step)) / (np.sqrt(v / (1 - b2 ** step)) + c["eps"])
    J1 = float(np.real(loss(theta, boxes, Ps, views, img_wh)))
    return dict(theta=theta, J0=hist[0] if hist else J1, J=J1, hist=np.array(hist + [J1]), margin=margin)
