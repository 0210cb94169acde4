"""Pins for the association oracle (Eq. (4)-(6)): the quadric distance in
closed form (identical quadrics, pure translation, rotation of a sphere),
the coarse match on a hand-made IoU matrix (threshold, ties, empty), the
occlusion ratio on hand boxes, and a scene whose detections are the
brute-force projected boxes of known ellipsoids, shuffled, plus a spurious
one."""
import numpy as np
from scipy.spatial.transform import Rotation

import oracle as O
from oracle import associate as A
from paper_2503_02223_amd import scenes


def test_quadric_distance_closed_forms():
    R = Rotation.from_rotvec([0.3, -0.2, 0.5]).as_matrix()
    mu, ax = np.array([0.1, 0.2, 0.3]), np.array([0.1, 0.2, 0.3])
    assert A.quadric_distance(mu, R, ax, mu, R, ax) == 1.0
    # translation only: exp(-tau d)
    np.testing.assert_allclose(A.quadric_distance(mu, R, ax, mu + [0.3, 0.4, 0.0], R, ax), np.exp(-0.5), rtol=1e-14)
    # a sphere is the same whatever its rotation
    s = np.array([0.2, 0.2, 0.2])
    np.testing.assert_allclose(A.quadric_distance(mu, np.eye(3), s, mu, R, s), 1.0, rtol=1e-14)
    # axis-aligned boxes of different size: ||diag(a^2) - diag(b^2)||_F
    d = np.linalg.norm([0.1 ** 2 - 0.2 ** 2, 0.2 ** 2 - 0.2 ** 2, 0.3 ** 2 - 0.1 ** 2])
    np.testing.assert_allclose(A.quadric_distance(mu, np.eye(3), ax, mu, np.eye(3), [0.2, 0.2, 0.1]),
                               np.exp(-d), rtol=1e-14)


def test_coarse_match_hand_matrix():
    iou = np.array([[0.9, 0.2, 0.0, 0.4],
                    [0.1, 0.2, 0.0, 0.4],
                    [0.0, 0.25, 0.0, 0.1]])
    np.testing.assert_array_equal(A.coarse_match(iou), [0, -1, -1, 0])   # 0.25 < 0.3; tie 0.4 -> object 0
    np.testing.assert_array_equal(A.coarse_match(iou, iou_min=0.2), [0, 2, -1, 0])
    assert A.coarse_match(np.zeros((0, 3))).tolist() == [-1, -1, -1]


def test_occlusion_ratio_hand_boxes():
    b = np.array([[0, 0, 10, 10],      # large
                  [8, 8, 12, 12],      # small, 1/4 inside the large one
                  [2, 2, 4, 4],        # tiny, fully inside both? only inside box 0
                  [20, 20, 30, 30]])   # same area as box 0, disjoint
    t = A.occlusion_ratio(b)
    np.testing.assert_allclose(t[0, 1], 4 / 16)
    np.testing.assert_allclose(t[0, 2], 1.0)
    assert t[1, 0] == 0 and t[2, 0] == 0          # only the smaller box is the denominator
    assert t[0, 3] == 0 and t[3, 0] == 0          # equal areas: neither is the smaller
    assert t[1, 2] == 0                           # disjoint
    assert (np.diag(t) == 0).all()


def _surface_box(mu, R, axes, P, n=400):
    u = np.linspace(0, np.pi, n)[:, None]
    v = np.linspace(0, 2 * np.pi, 2 * n)[None, :]
    s = np.stack([np.sin(u) * np.cos(v), np.sin(u) * np.sin(v), np.cos(u) + 0 * v]).reshape(3, -1)
    X = R @ (np.asarray(axes)[:, None] * s) + np.asarray(mu)[:, None]
    x = P @ np.vstack([X, np.ones(X.shape[1])])
    return np.array([(x[0] / x[2]).min(), (x[1] / x[2]).min(), (x[0] / x[2]).max(), (x[1] / x[2]).max()])


def test_detections_of_known_ellipsoids_match_their_objects():
    rng = np.random.default_rng(0)
    cam = scenes.ring_cameras(1, radius=2.0, width=640, height=480, f=600.0, angles=[0.4])[0]
    P = O.camera_matrix(cam)
    mus = [np.array([-0.5, 0.0, 0.0]), np.array([0.2, 0.1, 0.3]), np.array([0.6, -0.2, -0.3])]
    Rs = [Rotation.random(random_state=k).as_matrix() for k in range(3)]
    axs = [rng.uniform(0.08, 0.2, 3) for _ in range(3)]
    dets = [_surface_box(m, R, a, P) for m, R, a in zip(mus, Rs, axs)]
    dets.append(np.array([10.0, 10.0, 40.0, 40.0]))          # nothing there
    perm = [2, 3, 0, 1]
    dets = np.array(dets)[perm]
    boxes, ok = A.projected_boxes(mus, Rs, axs, P, (640, 480))
    assert ok.all()
    iou = A.iou_matrix(boxes, ok, dets)
    m = A.coarse_match(iou)
    np.testing.assert_array_equal(m, [2, -1, 0, 1])
    assert (iou[m[m >= 0], np.nonzero(m >= 0)[0]] > 0.99).all()


def test_decide_hand_case():
    """QD filter of the coarse matches and the occlusion merge on hand boxes
    whose ratios follow from the geometry (worked out by hand below)."""
    boxes = np.array([[0, 0, 100, 100],       # 0 large, label 1
                      [10, 10, 105, 60],      # 1 t[0][1] = 4500/4750 = 0.947 -> piece of 0
                      [98, 20, 104, 26],      # 2 inside 1 (t = 1); t[0][2] = 12/36 -> piece of 1 only
                      [60, 60, 80, 80],       # 3 inside 0 but label 2
                      [30, 70, 40, 80],       # 4 inside 0, but its quadric is too far from 0's
                      [200, 200, 260, 260],   # 5 disjoint
                      [12, 12, 14, 14],       # 6 inside 0 and 1 (t = 1 both): lower index 0
                      [90, 30, 101, 40]],     # 7 t[0][7] = 100/110, t[1][7] = 1: the larger ratio, 1
                     np.float64)
    label = [1, 1, 1, 2, 1, 1, 1, 1]
    occ = A.occlusion_ratio(boxes)
    np.testing.assert_allclose([occ[0, 1], occ[1, 2], occ[0, 2], occ[0, 7], occ[1, 7]],
                               [4500 / 4750, 1.0, 12 / 36, 100 / 110, 1.0])
    qd_det = np.full((8, 8), 0.5)
    qd_det[0, 4] = qd_det[4, 0] = 0.05
    match = [0, 0, 1, 1, -1, 0, 0, 0]
    qd_obs = np.array([[0.9, 0.0], [0.3, 0.0], [0.0, 0.6], [0.0, 0.5], [0.0, 0.0], [0.49, 0.0], [0.99, 0.0],
                       [0.7, 0.0]])
    d = A.decide(match, qd_obs, occ, qd_det, label)
    assert d["fine"].tolist() == [0, -1, 1, 1, -1, -1, 0, 0]       # 0.3, 0.49 < 0.5 dropped; 0.5 kept
    assert d["parent"].tolist() == [-1, 0, 1, -1, -1, -1, 0, 1]
    assert d["root"].tolist() == [0, 0, 0, 3, 4, 5, 0, 0]
    assert d["obj"].tolist() == [0, 0, 0, 1, -1, -1, 0, 0]


def test_decide_thresholds_are_strict_and_empty():
    occ = np.zeros((3, 3))
    occ[0, 1], occ[0, 2] = 0.85, 0.9          # exactly at the ratio threshold: not a piece
    qd_det = np.full((3, 3), 0.1)             # exactly at the QD threshold: not a piece
    d = A.decide([-1, -1, -1], np.zeros((3, 0)), occ, qd_det, [0, 0, 0])
    assert d["parent"].tolist() == [-1, -1, -1]
    qd_det[0, 2] = np.nextafter(0.1, 1.0)
    d = A.decide([-1, -1, -1], np.zeros((3, 0)), occ, qd_det, [0, 0, 0])
    assert d["parent"].tolist() == [-1, -1, 0] and d["root"].tolist() == [0, 1, 0]
    assert d["obj"].tolist() == [-1, -1, -1]
    e = A.decide(np.zeros(0, np.int32), np.zeros((0, 0)), np.zeros((0, 0)), np.zeros((0, 0)), [])
    assert all(len(v) == 0 for v in e.values())
