"""GPU parity of the association scores (Eq. (4)-(6)) against the FP64
oracle: IoU of projected object quadrics with the detections of several
frames, the coarse match (exact where the decision is not within 1e-9 of a
tie or of the threshold), the occlusion ratios of same-frame detections,
and the quadric distance of Eq. (5)."""
import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

import oracle as O
from oracle import associate as A
from paper_2503_02223_amd import binding as B
from paper_2503_02223_amd import scenes

pytestmark = pytest.mark.gpu
W, H = 640, 480


def _objects(rng, n):
    mu = rng.uniform(-0.6, 0.6, (n, 3))
    R = np.stack([Rotation.random(random_state=int(rng.integers(1 << 30))).as_matrix() for _ in range(n)])
    ax = rng.uniform(0.06, 0.3, (n, 3))
    return mu, R, ax


@pytest.mark.parametrize("n_obj,n_frames", [(12, 3), (40, 8)])
def test_association_scores_parity(n_obj, n_frames):
    rng = np.random.default_rng(n_obj)
    mu, R, ax = _objects(rng, n_obj)
    cams = scenes.ring_cameras(n_frames, radius=2.0, width=W, height=H, f=600.0,
                               angles=np.linspace(0.0, 2.0, n_frames))
    Ps = np.stack([O.camera_matrix(c) for c in cams])
    boxes, frames = [], []
    for f in range(n_frames):
        pb, ok = A.projected_boxes(mu, R, ax, Ps[f], (W, H))
        for k in rng.permutation(n_obj)[: n_obj * 3 // 4]:       # most objects detected, jittered
            if ok[k]:
                boxes.append(np.clip(pb[k] + rng.normal(0, 3.0, 4), 0, [W, H, W, H]))
                frames.append(f)
        boxes.append(np.array([5.0, 5.0, 60.0, 50.0]))           # a false detection
        frames.append(f)
    boxes, frames = np.array(boxes), np.array(frames, np.int32)
    d = lambda a, dt=torch.float64: torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    wh = d(np.array([[W, H]] * n_frames), torch.int32)
    out = B.associate(B.Context(), d(mu), d(R), d(ax), d(boxes), d(frames, torch.int32), d(Ps.reshape(-1, 12)), wh)
    torch.cuda.synchronize()
    iou, match, occ = out["iou"].cpu().numpy(), out["match"].cpu().numpy(), out["occ"].cpu().numpy()
    iou_o = np.zeros_like(iou)
    for f in range(n_frames):
        sel = frames == f
        pb, ok = A.projected_boxes(mu, R, ax, Ps[f], (W, H))
        iou_o[:, sel] = A.iou_matrix(pb, ok, boxes[sel])
    np.testing.assert_allclose(iou, iou_o, rtol=0, atol=1e-9)
    m_o = A.coarse_match(iou_o)
    srt = np.sort(iou_o, axis=0)
    top, gap = srt[-1], (srt[-1] - srt[-2]) if n_obj > 1 else np.full(srt.shape[1], np.inf)
    # below the threshold both sides answer -1 whatever the ties; above it the top must be unique
    clear = (top < A.IOU_MIN - 1e-9) | ((top > A.IOU_MIN + 1e-9) & (gap > 1e-9))
    assert clear.mean() > 0.9
    np.testing.assert_array_equal(match[clear], m_o[clear])
    assert (match >= 0).sum() > 0.5 * len(boxes)
    occ_o = np.zeros_like(occ)
    for f in range(n_frames):
        idx = np.nonzero(frames == f)[0]
        occ_o[np.ix_(idx, idx)] = A.occlusion_ratio(boxes[idx])
    np.testing.assert_allclose(occ, occ_o, rtol=0, atol=1e-12)


def test_quadric_distance_parity():
    rng = np.random.default_rng(5)
    a, b = _objects(rng, 9), _objects(rng, 14)
    d = lambda x: torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")
    qd = B.quadric_distance(B.Context(), dict(mu=d(a[0]), R=d(a[1]), axes=d(a[2])),
                            dict(mu=d(b[0]), R=d(b[1]), axes=d(b[2])), tau=1.3)
    torch.cuda.synchronize()
    want = np.array([[A.quadric_distance(a[0][i], a[1][i], a[2][i], b[0][j], b[1][j], b[2][j], tau=1.3)
                      for j in range(14)] for i in range(9)])
    np.testing.assert_allclose(qd.cpu().numpy(), want, rtol=1e-13)


def test_association_edge_cases():
    d = lambda a, dt=torch.float64: torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    cam = scenes.camera(fx=600.0, fy=600.0, cx=320.0, cy=240.0, width=W, height=H)
    P = d(O.camera_matrix(cam).reshape(1, 12))
    wh = d(np.array([[W, H]]), torch.int32)
    boxes = d(np.array([[300.0, 220.0, 340.0, 260.0]]))
    frames = d(np.zeros(1), torch.int32)
    # no objects: every detection is new
    e = torch.zeros(0, 3, dtype=torch.float64, device="cuda")
    out = B.associate(B.Context(), e, torch.zeros(0, 9, dtype=torch.float64, device="cuda"), e, boxes, frames, P, wh)
    torch.cuda.synchronize()
    assert out["match"].cpu().tolist() == [-1]
    # an object around the camera centre has no projected box: IoU 0, no match
    out = B.associate(B.Context(), d([[0.0, 0.0, 0.1]]), d(np.eye(3).reshape(1, 9)), d([[0.5, 0.5, 0.5]]), boxes,
                      frames, P, wh)
    torch.cuda.synchronize()
    assert float(out["iou"][0, 0]) == 0.0 and out["match"].cpu().tolist() == [-1]
    # an object straight ahead matching the detection exactly
    r = 0.3
    z = 3.0
    h = 600.0 * r / np.sqrt(z * z - r * r)
    exact = d(np.array([[320 - h, 240 - h, 320 + h, 240 + h]]))
    out = B.associate(B.Context(), d([[0.0, 0.0, z]]), d(np.eye(3).reshape(1, 9)), d([[r, r, r]]), exact, frames, P,
                      wh)
    torch.cuda.synchronize()
    assert abs(float(out["iou"][0, 0]) - 1.0) < 1e-12 and out["match"].cpu().tolist() == [0]


def _decide_dev(match, qd_obs, occ, qd_det, label):
    d = lambda a, dt: torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    out = B.associate_decide(B.Context(), d(match, torch.int32), d(qd_obs, torch.float64), d(occ, torch.float64),
                             d(qd_det, torch.float64), d(label, torch.int32))
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def _nested_frames(rng, n_frames, per_frame):
    """Boxes of several frames, built so that many are pieces of larger ones
    (chains of nested boxes, some only partly inside, some of another label)."""
    boxes, frames, labels = [], [], []
    for f in range(n_frames):
        for _ in range(per_frame // 4):
            x0, y0 = rng.uniform(0, 400), rng.uniform(0, 300)
            w, h = rng.uniform(60, 200), rng.uniform(60, 160)
            lab = int(rng.integers(3))
            b = np.array([x0, y0, x0 + w, y0 + h])
            for _ in range(4):
                boxes.append(b.copy())
                frames.append(f)
                labels.append(lab if rng.random() < 0.8 else int(rng.integers(3)))
                s = rng.uniform(0.4, 0.9)
                w2, h2 = (b[2] - b[0]) * s, (b[3] - b[1]) * s
                ox = rng.uniform(-0.15, 1.1) * (b[2] - b[0] - w2)     # sometimes sticks out
                oy = rng.uniform(0.0, 1.0) * (b[3] - b[1] - h2)
                b = np.array([b[0] + ox, b[1] + oy, b[0] + ox + w2, b[1] + oy + h2])
    return np.array(boxes), np.array(frames, np.int32), np.array(labels, np.int32)


@pytest.mark.parametrize("n_frames,per_frame,n_obj", [(1, 8, 2), (6, 40, 10), (10, 120, 25)])
def test_decide_parity(n_frames, per_frame, n_obj):
    rng = np.random.default_rng(per_frame)
    boxes, frames, label = _nested_frames(rng, n_frames, per_frame)
    n = len(boxes)
    occ = np.zeros((n, n))
    for f in range(n_frames):
        idx = np.nonzero(frames == f)[0]
        occ[np.ix_(idx, idx)] = A.occlusion_ratio(boxes[idx])
    qd_det = rng.uniform(0.0, 0.3, (n, n))
    qd_obs = rng.uniform(0.2, 1.0, (n, n_obj))
    match = rng.integers(-1, n_obj, n).astype(np.int32)
    want = A.decide(match, qd_obs, occ, qd_det, label)
    absorbed = want["parent"] >= 0
    assert absorbed.sum() > n // 8 and (absorbed & (want["root"] != want["parent"])).any()     # chains of 2+
    got = _decide_dev(match, qd_obs, occ, qd_det, label)
    for k in ("fine", "parent", "root", "obj"):
        np.testing.assert_array_equal(got[k], want[k], err_msg=k)


def test_decide_edge_cases():
    # no objects: every fine match is -1, pieces still merge
    occ = np.array([[0.0, 0.9], [0.0, 0.0]])
    got = _decide_dev([-1, -1], np.zeros((2, 0)), occ, np.full((2, 2), 0.5), [3, 3])
    assert got["parent"].tolist() == [-1, 0] and got["root"].tolist() == [0, 0] and got["obj"].tolist() == [-1, -1]
    # thresholds are strict for the merge and inclusive for the filter
    got = _decide_dev([0, 0], np.array([[0.5], [0.4999]]), np.array([[0.0, 0.85], [0.0, 0.0]]),
                      np.full((2, 2), 0.5), [1, 1])
    assert got["fine"].tolist() == [0, -1] and got["parent"].tolist() == [-1, -1]
    # no detections
    e = B.associate_decide(B.Context(), torch.zeros(0, dtype=torch.int32, device="cuda"),
                           torch.zeros(0, 0, dtype=torch.float64, device="cuda"),
                           torch.zeros(0, 0, dtype=torch.float64, device="cuda"),
                           torch.zeros(0, 0, dtype=torch.float64, device="cuda"),
                           torch.zeros(0, dtype=torch.int32, device="cuda"))
    torch.cuda.synchronize()
    assert all(v.numel() == 0 for v in e.values())


def test_decide_max_detections_known_chains():
    """32768 detections (the largest batch), as chains of 4 nested pieces of
    one label, each chain in a frame of its own: every piece's parent is the
    one before it, its root the chain's head, its object the head's match."""
    n = 1 << 15
    dev = "cuda"
    j = torch.arange(n, device=dev)
    head = j - j % 4
    occ = torch.zeros(n, n, dtype=torch.float64, device=dev)
    qd_det = torch.full((n, n), 0.5, dtype=torch.float64, device=dev)
    piece = j % 4 != 0
    occ[(j - 1)[piece], j[piece]] = 0.95          # the previous piece holds this one
    occ[head[piece], j[piece]] = torch.where(j[piece] % 4 == 1, 0.95, 0.9).to(torch.float64)
    n_obj = 64
    match = (head // 4 % n_obj).to(torch.int32)
    qd_obs = torch.full((n, n_obj), 0.9, dtype=torch.float64, device=dev)
    label = torch.zeros(n, dtype=torch.int32, device=dev)
    out = B.associate_decide(B.Context(), match, qd_obs, occ, qd_det, label)
    torch.cuda.synchronize()
    jj = j.cpu().numpy()
    hh = jj - jj % 4
    want_parent = np.where(jj % 4 == 0, -1, jj - 1)
    np.testing.assert_array_equal(out["parent"].cpu().numpy(), want_parent)
    np.testing.assert_array_equal(out["root"].cpu().numpy(), hh)
    np.testing.assert_array_equal(out["obj"].cpu().numpy(), hh // 4 % n_obj)
    np.testing.assert_array_equal(out["fine"].cpu().numpy(), match.cpu().numpy())
