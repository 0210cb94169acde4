"""Oracle of the object-level association (test infrastructure only; numpy,
FP64).

Sec. III-B: existing objects are projected into a frame through their dual
quadrics (Eq. (4), C* = P Q* P^T) and the tangent box of each projection is
compared with the frame's detected boxes by IoU (coarse association); a
quadric distance QD = exp(-tau (||mu_a - mu_b|| + ||S_a - S_b||_F)) (Eq. (5))
between an observation's quadric and an object's filters wrong matches; and
for two detections where the smaller box B_j lies mostly inside the larger
B_i, the overlap ratio t = |B_i n B_j| / |B_j| (Eq. (6)) with t > 0.85 and a
QD test marks B_j as a piece of the object of B_i (occlusion).

Readings: S in Eq. (5) is the quadric's shape matrix R diag(a^2, b^2, c^2)
R^T (rotation-aware, in m^2); tau = 1 / m (unstated); the coarse match of a
detection is the object of largest IoU provided IoU >= iou_min = 0.3
(unstated; ties to the lower object index), else the detection starts a new
object (-1); a match whose QD falls below qd_min = 0.5 (unstated; Eq. (5)'s
inequality reads reversed) is rejected; the occlusion test is t > 0.85
(stated) and QD(O_i, O_j) > d with d = 0.1 (stated as QD < d; read with QD a
similarity, so the two pieces must be close); projected boxes are clipped to
the image; an undefined projection (camera inside or behind the quadric)
has IoU 0.
"""
from __future__ import annotations

import numpy as np

from oracle import refine as RF

IOU_MIN, TAU, QD_MIN, T_OCC, QD_OCC = 0.3, 1.0, 0.5, 0.85, 0.1


def projected_boxes(mu, R, axes, P, wh):
    """Clipped tangent boxes (n, 4) of the objects' quadrics in camera P and
    whether each is defined (n,)."""
    n = len(mu)
    out = np.zeros((n, 4))
    ok = np.zeros(n, bool)
    for k in range(n):
        b = RF.predicted_box(RF.pack(mu[k], R[k], axes[k]), P, wh)
        if b is not None:
            out[k] = np.real(np.asarray(b))
            ok[k] = True
    return out, ok


def iou_matrix(obj_boxes, obj_ok, det_boxes):
    """IoU[k][j] between object k's projected box and detection j."""
    M = np.zeros((len(obj_boxes), len(det_boxes)))
    for k in range(len(obj_boxes)):
        if not obj_ok[k]:
            continue
        for j in range(len(det_boxes)):
            M[k, j] = float(np.real(RF.iou(list(obj_boxes[k]), np.asarray(det_boxes[j], np.float64))))
    return M


def shape(R, axes):
    return np.asarray(R) @ np.diag(np.asarray(axes, np.float64) ** 2) @ np.asarray(R).T


def quadric_distance(mu_a, R_a, ax_a, mu_b, R_b, ax_b, tau=TAU):
    """Eq. (5): exp(-tau (||mu_a - mu_b||_2 + ||S_a - S_b||_F))."""
    d = np.linalg.norm(np.asarray(mu_a) - np.asarray(mu_b)) + np.linalg.norm(shape(R_a, ax_a) - shape(R_b, ax_b))
    return float(np.exp(-tau * d))


def coarse_match(iou, iou_min=IOU_MIN):
    """Per detection: the object of largest IoU (lowest index among equals)
    if that IoU >= iou_min, else -1."""
    n_obj, n_det = iou.shape
    m = np.full(n_det, -1, np.int32)
    for j in range(n_det):
        best, arg = -1.0, -1
        for k in range(n_obj):
            if iou[k, j] > best:
                best, arg = iou[k, j], k
        if arg >= 0 and best >= iou_min:
            m[j] = arg
    return m


def occlusion_ratio(det_boxes):
    """t[i][j] = |B_i n B_j| / |B_j| where |B_j| < |B_i|, else 0 (Eq. (6))."""
    b = np.asarray(det_boxes, np.float64)
    n = len(b)
    area = (b[:, 2] - b[:, 0]) * (b[:, 3] - b[:, 1])
    t = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            if i == j or not area[j] < area[i] or area[j] <= 0:
                continue
            iw = min(b[i, 2], b[j, 2]) - max(b[i, 0], b[j, 0])
            ih = min(b[i, 3], b[j, 3]) - max(b[i, 1], b[j, 1])
            if iw > 0 and ih > 0:
                t[i, j] = iw * ih / area[j]
    return t


def decide(match, qd_obs, occ, qd_det, label, qd_min=QD_MIN, t_occ=T_OCC, qd_occ=QD_OCC):
    """The decisions taken from the scores (Sec. III-B, Eq. (5)-(6)).

    fine[j]   = match[j] when QD(observation j, object match[j]) >= qd_min,
                else -1 (the wrong match is dropped: j seeds a new object);
    parent[j] = the detection i whose larger box holds j's (occ[i][j] >
                t_occ) with the same label and QD(observation i,
                observation j) > qd_occ: j is a piece of i's object and is
                popped; among several, the largest ratio, then the lowest
                index; -1 when there is none;
    root[j]   = the end of j's chain of parents (j when not absorbed);
    obj[j]    = fine[root[j]]: the object that j's observation updates, or
                -1 for a new object seeded by detection root[j].
    A parent's box is strictly larger (occ is 0 otherwise), so chains end."""
    match = np.asarray(match)
    n = len(match)
    fine = np.full(n, -1, np.int32)
    for j in range(n):
        k = match[j]
        if k >= 0 and qd_obs[j][k] >= qd_min:
            fine[j] = k
    parent = np.full(n, -1, np.int32)
    for j in range(n):
        best = -np.inf
        for i in range(n):
            if label[i] == label[j] and occ[i][j] > t_occ and qd_det[i][j] > qd_occ and occ[i][j] > best:
                best, parent[j] = occ[i][j], i
    root = np.arange(n, dtype=np.int32)
    for j in range(n):
        while parent[root[j]] >= 0:
            root[j] = parent[root[j]]
    obj = fine[root] if n else np.zeros(0, np.int32)
    return dict(fine=fine, parent=parent, root=root, obj=obj.astype(np.int32))
