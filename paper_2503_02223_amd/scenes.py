"""Seeded synthetic workloads (inputs only).

This module draws random numbers and builds cameras; it holds none of the
rasterization, loss or quadric arithmetic, so both the GPU library's tests and
the oracle's tests can take their inputs from it.  It imports numpy only.

Parameter layout everywhere: params[14][n] float64 with rows 0-2 mean,
3-5 log-scale, 6-9 quaternion (w, x, y, z), 10 opacity logit, 11-13 colour.

The paper's datasets (Cube-Diorama, Replica, Ai2-THOR captures) are not
available; these scenes stand in for them with the shapes of the workloads the
benchmarks use: a 2k-Gaussian single view, a 200k-Gaussian room of 20 object
blobs at 640x480, 8 ring keyframes over 1.2M Gaussians in 40 objects, and a 1M
Gaussian 1200x680 view.
"""
from __future__ import annotations

import numpy as np

ROOM_LO = np.array([-3.0, -1.5, -2.0])
ROOM_HI = np.array([3.0, 1.5, 2.0])


def camera(R=None, t=None, fx=110.0, fy=110.0, cx=64.0, cy=48.0, width=128, height=96):
    return dict(R=np.eye(3) if R is None else np.asarray(R, np.float64).reshape(3, 3),
                t=np.zeros(3) if t is None else np.asarray(t, np.float64).reshape(3),
                fx=float(fx), fy=float(fy), cx=float(cx), cy=float(cy),
                width=int(width), height=int(height))


def look_at(position, target, **intr):
    """World->camera pose of a camera at `position` looking at `target`
    (camera x right, y down, z forward; world y points down)."""
    c = np.asarray(position, np.float64)
    z = np.asarray(target, np.float64) - c
    z /= np.linalg.norm(z)
    x = np.cross(np.array([0.0, 1.0, 0.0]), z)
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    R = np.stack([x, y, z])
    return camera(R=R, t=-R @ c, **intr)


def ring_cameras(n_views=8, radius=2.0, width=640, height=480, f=600.0, angles=None):
    """Keyframes on a horizontal ring around the room centre, facing it, at
    the given angles (default: evenly spaced)."""
    cams = []
    if angles is None:
        angles = 2 * np.pi * np.arange(n_views) / n_views
    for a in angles:
        pos = np.array([radius * np.sin(a), 0.0, -radius * np.cos(a)])
        cams.append(look_at(pos, np.zeros(3), fx=f, fy=f, cx=width / 2, cy=height / 2,
                            width=width, height=height))
    return cams


def _random_quats(rng, n):
    q = rng.normal(size=(4, n))
    return q / np.linalg.norm(q, axis=0, keepdims=True)


def pack(mu, logscale, quat, eta, rgb):
    return np.ascontiguousarray(np.concatenate([mu, logscale, quat, eta[None], rgb], axis=0))


def single_view_scene(seed=0, n=2000):
    """2,000 Gaussians, means uniform in [-1,1]^3 placed 3 m in front of a
    128x96 pinhole camera (f = 110, c = (64, 48)); log-scales N(-3, 0.5),
    random unit quaternions, opacity logits N(0, 1), colours U[0,1], object ids
    uniform in {0, 1, 2}."""
    rng = np.random.default_rng(seed)
    mu = rng.uniform(-1, 1, size=(3, n)) + np.array([[0.0], [0.0], [3.0]])
    ls = rng.normal(-3.0, 0.5, size=(3, n))
    q = _random_quats(rng, n)
    eta = rng.normal(0.0, 1.0, size=n)
    rgb = rng.uniform(0, 1, size=(3, n))
    ids = rng.integers(0, 3, size=n).astype(np.int32)
    cam = camera()
    return dict(params=pack(mu, ls, q, eta, rgb), ids=ids, cams=[cam], K=3)


def _surface_points(rng, m):
    """Points uniform (by area) on the six faces of the room box."""
    lo, hi = ROOM_LO, ROOM_HI
    ext = hi - lo
    areas = np.array([ext[1] * ext[2], ext[1] * ext[2], ext[0] * ext[2], ext[0] * ext[2],
                      ext[0] * ext[1], ext[0] * ext[1]])
    face = rng.choice(6, size=m, p=areas / areas.sum())
    pts = rng.uniform(lo, hi, size=(m, 3))
    axis = face // 2
    pts[np.arange(m), axis] = np.where(face % 2 == 0, lo[axis], hi[axis])
    return pts


def room_scene(seed=0, n=200_000, n_objects=20, background_frac=0.3, blob_sigma=0.3,
               object_counts=None, logscale=(-4.0, 0.7), eta_sigma=1.5, background="volume", centres=None):
    """Gaussians clustered into object blobs (means N(centre, blob_sigma^2),
    centres uniform in the 6x4x3 m room unless given) plus background
    Gaussians with id 0, uniform in the room's volume or on its walls, floor
    and ceiling (background="surface"); objects have ids 1..n_objects."""
    rng = np.random.default_rng(seed)
    if object_counts is None:
        n_bg = int(round(background_frac * n))
        per = (n - n_bg) // n_objects
        counts = np.full(n_objects, per, dtype=np.int64)
        n_bg = n - counts.sum()
    else:
        counts = np.asarray(object_counts, dtype=np.int64)
        n_bg = n - counts.sum()
        assert n_bg >= 0
    drawn = rng.uniform(ROOM_LO, ROOM_HI, size=(n_objects, 3))
    centres = drawn if centres is None else np.asarray(centres, np.float64)
    bg = rng.uniform(ROOM_LO, ROOM_HI, size=(n_bg, 3)) if background == "volume" else _surface_points(rng, n_bg)
    mus, ids = [bg], [np.zeros(n_bg, np.int32)]
    for k in range(n_objects):
        mus.append(rng.normal(centres[k], blob_sigma, size=(counts[k], 3)))
        ids.append(np.full(counts[k], k + 1, np.int32))
    mu = np.concatenate(mus, axis=0).T
    ids = np.concatenate(ids)
    ls = rng.normal(logscale[0], logscale[1], size=(3, n))
    q = _random_quats(rng, n)
    eta = rng.normal(0.0, eta_sigma, size=n)
    rgb = rng.uniform(0, 1, size=(3, n))
    return dict(params=pack(mu, ls, q, eta, rgb), ids=ids.astype(np.int32), K=n_objects + 1,
                centres=centres)


def slam_view_scene(seed=0, n=200_000):
    """The 200k-Gaussian room at 640x480, f = 600, seen whole from
    (0, 0, -7.63) looking along +z."""
    sc = room_scene(seed=seed, n=n)
    sc["cams"] = [camera(t=[0.0, 0.0, 7.63], fx=600, fy=600, cx=320, cy=240, width=640, height=480)]
    return sc


def keyframe_scene(seed=0, n_total=1_200_000, n_objects=40, n_views=8):
    """40 objects with Gaussian counts log-uniform in [1k, 80k] (blob sigma
    0.06 m, log-scales N(-4.5, 0.4), so that objects mostly stay apart),
    topped up with background Gaussians on the room's walls, floor and ceiling
    to n_total (a volume-filling background would hide every object from
    cameras inside the room).  The 8 keyframes sit at seeded random angles on
    a 2 m ring at 640x480, facing the room centre; object centres are uniform
    in the upright cylinder of radius 1.2 m and height 1.6 m inside the ring,
    so that each object lies in front of the cameras."""
    rng = np.random.default_rng(seed + 1000)
    counts = np.exp(rng.uniform(np.log(1e3), np.log(8e4), size=n_objects)).astype(np.int64)
    r = 1.2 * np.sqrt(rng.uniform(0, 1, n_objects))
    phi = rng.uniform(0, 2 * np.pi, n_objects)
    centres = np.stack([r * np.cos(phi), rng.uniform(-0.8, 0.8, n_objects), r * np.sin(phi)], axis=1)
    angles = np.sort(rng.uniform(0, 2 * np.pi, n_views))
    sc = room_scene(seed=seed, n=n_total, n_objects=n_objects, object_counts=counts, background="surface",
                    blob_sigma=0.06, logscale=(-4.5, 0.4), centres=centres)
    sc["cams"] = ring_cameras(n_views, angles=angles)
    return sc


def large_view_scene(seed=0, n=1_000_000):
    """1M Gaussians of the room generator seen at 1200x680 from ring pose 0."""
    sc = room_scene(seed=seed, n=n)
    sc["cams"] = ring_cameras(1, width=1200, height=680)
    return sc


def tiny_scene(seed=0, n=64, width=32, height=32, f=40.0, depth=3.0, spread=0.6,
               logscale=(-2.2, 0.3), n_ids=3):
    """A small scene for finite differences: n Gaussians in front of a
    width x height camera."""
    rng = np.random.default_rng(seed)
    mu = np.stack([rng.uniform(-spread, spread, n), rng.uniform(-spread, spread, n),
                   rng.uniform(depth - 0.5, depth + 0.5, n)])
    ls = rng.normal(logscale[0], logscale[1], size=(3, n))
    q = _random_quats(rng, n)
    eta = rng.normal(0.5, 1.0, size=n)
    rgb = rng.uniform(0, 1, size=(3, n))
    ids = rng.integers(0, n_ids, size=n).astype(np.int32)
    cam = camera(fx=f, fy=f, cx=width / 2, cy=height / 2, width=width, height=height)
    return dict(params=pack(mu, ls, q, eta, rgb), ids=ids, cams=[cam], K=n_ids)


def perturb(params, seed):
    """A perturbed copy used to make targets: mean += N(0, 0.02 m),
    log-scale += N(0, 0.1), opacity logit += N(0, 0.3), colour += N(0, 0.05)
    clipped to [0, 1]; quaternions and ids unchanged."""
    rng = np.random.default_rng(seed)
    p = np.array(params, dtype=np.float64, copy=True)
    n = p.shape[1]
    p[0:3] += rng.normal(0, 0.02, size=(3, n))
    p[3:6] += rng.normal(0, 0.1, size=(3, n))
    p[10] += rng.normal(0, 0.3, size=n)
    p[11:14] = np.clip(p[11:14] + rng.normal(0, 0.05, size=(3, n)), 0.0, 1.0)
    return p


def random_image_grads(seed, shape_chw, K=None):
    """Seeded upstream gradients for adjoint tests."""
    rng = np.random.default_rng(seed)
    C, H, W = shape_chw
    out = dict(gC=rng.normal(size=(3, H, W)), gD=rng.normal(size=(H, W)),
               gT=rng.normal(size=(H, W)))
    if K:
        out["gP"] = rng.normal(size=(K, H, W))
    return out
