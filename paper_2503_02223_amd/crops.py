"""Seeded synthetic object crops (inputs only).

Each crop is one object seen by a 128x128 pinhole camera (f = 110, principal
point at the crop centre, camera frame = world frame): a superquadric with
random exponents in [0.3, 2] and semi-axes in [0.05, 0.3] m, randomly rotated,
textured with fractal Perlin noise blending two random colours and lit by one
directional light, ray-cast to an RGB image, a depth map (camera z, 0 where
the ray misses) and an instance mask.  They stand in for object crops of the
paper's RGB-D sequences, which are not available.

This module draws random numbers and ray-casts; it holds none of the
rasterization, initialization or network arithmetic, so the GPU library's
tests and the oracle's tests can both take their inputs from it.  numpy only.
"""
from __future__ import annotations

import numpy as np

CROP = 128
FOCAL = 110.0


def crop_camera(size=CROP, f=FOCAL):
    """Camera dict of a crop (identity pose)."""
    return dict(R=np.eye(3), t=np.zeros(3), fx=float(f), fy=float(f), cx=size / 2.0, cy=size / 2.0,
                width=int(size), height=int(size))


# ---------------------------------------------------------------- Perlin noise
def _fade(t):
    return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)


_GRAD = np.array([[1, 1, 0], [-1, 1, 0], [1, -1, 0], [-1, -1, 0], [1, 0, 1], [-1, 0, 1], [1, 0, -1], [-1, 0, -1],
                  [0, 1, 1], [0, -1, 1], [0, 1, -1], [0, -1, -1], [1, 1, 0], [0, -1, 1], [-1, 1, 0], [0, -1, -1]],
                 dtype=np.float64)


def perlin3(p, perm):
    """Gradient noise of K. Perlin's improved noise (SIGGRAPH 2002): a
    permutation-hashed gradient, one of the 12 cube-edge directions (4
    repeated to fill 16), at each integer lattice corner; the dot products
    with the offsets to the point are blended with the quintic fade curve.
    p: (..., 3) points; perm: 512 ints (a permutation of 0..255, twice).
    Zero at every lattice point; values lie within about [-1, 1]."""
    p = np.asarray(p, np.float64)
    fl = np.floor(p)
    cell = fl.astype(np.int64) & 255
    f = p - fl
    u = _fade(f)
    out = 0.0
    X, Y, Z = cell[..., 0], cell[..., 1], cell[..., 2]
    acc = np.zeros(p.shape[:-1])
    for dx in (0, 1):
        for dy in (0, 1):
            for dz in (0, 1):
                h = perm[perm[perm[X + dx] + Y + dy] + Z + dz] & 15
                g = _GRAD[h]
                off = f - np.array([dx, dy, dz], np.float64)
                dot = (g * off).sum(-1)
                wx = u[..., 0] if dx else 1.0 - u[..., 0]
                wy = u[..., 1] if dy else 1.0 - u[..., 1]
                wz = u[..., 2] if dz else 1.0 - u[..., 2]
                acc = acc + wx * wy * wz * dot
    return acc + out


def fractal_noise(p, perm, octaves=4, lacunarity=2.0, gain=0.5):
    total = np.zeros(np.asarray(p).shape[:-1])
    amp, freq = 1.0, 1.0
    for _ in range(octaves):
        total += amp * perlin3(np.asarray(p) * freq, perm)
        amp *= gain
        freq *= lacunarity
    return total


# ---------------------------------------------------------------- superquadric
def superquadric_f(y, axes, e1, e2):
    """Inside-outside function of a superquadric in its own frame:
    ((|x/a|^(2/e2) + |y/b|^(2/e2))^(e2/e1) + |z/c|^(2/e1)); <= 1 inside."""
    ax, ay, az = axes
    xy = np.abs(y[..., 0] / ax) ** (2.0 / e2) + np.abs(y[..., 1] / ay) ** (2.0 / e2)
    return xy ** (e2 / e1) + np.abs(y[..., 2] / az) ** (2.0 / e1)


def _rotation(q):
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def random_object(rng):
    """Shape, pose, texture and light of one object."""
    axes = rng.uniform(0.05, 0.3, 3)
    e1, e2 = rng.uniform(0.3, 2.0, 2)
    rho = float(np.linalg.norm(axes))  # bounding-sphere radius (|x| <= a etc. for exponents <= 2)
    z0 = max(FOCAL * rho / (0.42 * CROP), rho + 0.3)
    perm = rng.permutation(256)
    return dict(axes=axes, e1=float(e1), e2=float(e2), R=_rotation(rng.normal(size=4)),
                centre=np.array([0.0, 0.0, z0]), rho=rho,
                c1=rng.uniform(0, 1, 3), c2=rng.uniform(0, 1, 3), freq=float(rng.uniform(4.0, 14.0)),
                perm=np.concatenate([perm, perm]),
                light=np.array([-0.4, -0.6, -0.7]) / np.linalg.norm([-0.4, -0.6, -0.7]))


def render_object(obj, size=CROP, f=FOCAL, coarse=64, refine=24):
    """Ray-cast one object: returns rgb (3, H, W) in [0, 1], depth (H, W) camera
    z (0 = miss) and mask (H, W) bool.  Pixel (u, v) is sampled at
    (u + 1/2, v + 1/2); along each ray that meets the bounding sphere, the first
    surface crossing is found by uniform sampling of the ray's chord through
    the sphere followed by bisection."""
    c = size / 2.0
    v, u = np.mgrid[0:size, 0:size].astype(np.float64)
    d = np.stack([(u + 0.5 - c) / f, (v + 0.5 - c) / f, np.ones_like(u)], -1).reshape(-1, 3)  # t scales z
    R, cen, rho = obj["R"], obj["centre"], obj["rho"]
    # chord of each ray x = t d through the sphere |x - cen| <= rho
    dd = (d * d).sum(-1)
    dc = d @ cen
    disc = dc * dc - dd * (cen @ cen - rho * rho)
    rays = np.nonzero(disc > 0)[0]
    sq = np.sqrt(disc[rays])
    t0, t1 = (dc[rays] - sq) / dd[rays], (dc[rays] + sq) / dd[rays]
    dr = d[rays]

    # object frame: y = R^T (t d - c) = t (R^T d) - R^T c
    dro, co = dr @ R, cen @ R

    def F(t):  # t: (m, k) -> inside-outside value at the points t * d
        y = dro[:, None, :] * t[..., None] - co
        return superquadric_f(y, obj["axes"], obj["e1"], obj["e2"])

    ts = t0[:, None] + (t1 - t0)[:, None] * np.linspace(0.0, 1.0, coarse)[None, :]
    inside = F(ts) <= 1.0
    hit_r = inside.any(-1)
    first = np.argmax(inside, -1)
    idx = np.arange(rays.size)
    lo = ts[idx, np.maximum(first - 1, 0)]
    hi = ts[idx, first]
    for _ in range(refine):
        mid = 0.5 * (lo + hi)
        ins = F(mid[:, None])[:, 0] <= 1.0
        hi = np.where(ins, mid, hi)
        lo = np.where(ins, lo, mid)
    rays, t, dr, dro = rays[hit_r], hi[hit_r], dr[hit_r], dro[hit_r]
    y = dro * t[:, None] - co
    # surface normal from central differences of F in the object frame
    h = 1e-4 * rho
    grad = np.zeros_like(y)
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        grad[:, k] = (superquadric_f(y + e, obj["axes"], obj["e1"], obj["e2"])
                      - superquadric_f(y - e, obj["axes"], obj["e1"], obj["e2"])) / (2 * h)
    n = grad @ R.T
    n /= np.maximum(np.linalg.norm(n, axis=-1, keepdims=True), 1e-12)
    n = np.where((n * dr).sum(-1, keepdims=True) > 0, -n, n)  # facing the camera
    shade = 0.45 + 0.55 * np.clip((n * -obj["light"]).sum(-1), 0.0, 1.0)
    tex = np.clip(0.5 + 1.5 * fractal_noise(y * obj["freq"], obj["perm"]), 0.0, 1.0)
    albedo = obj["c1"] * (1.0 - tex[:, None]) + obj["c2"] * tex[:, None]
    rgb = np.zeros((size * size, 3))
    depth = np.zeros(size * size)
    mask = np.zeros(size * size, bool)
    rgb[rays] = albedo * shade[:, None]
    depth[rays] = t
    mask[rays] = True
    return (np.ascontiguousarray(rgb.reshape(size, size, 3).transpose(2, 0, 1)), depth.reshape(size, size),
            mask.reshape(size, size))


def make_crops(seed, count, size=CROP):
    """count crops from one seed: rgbdm (count, 5, H, W) float32 with channels
    r, g, b, depth, mask."""
    rng = np.random.default_rng(seed)
    out = np.zeros((count, 5, size, size), np.float32)
    for i in range(count):
        for _ in range(20):  # redraw the rare object that covers too few pixels
            rgb, depth, mask = render_object(random_object(rng), size=size)
            if mask.sum() >= 64:
                break
        out[i, 0:3] = rgb
        out[i, 3] = depth
        out[i, 4] = mask
    return out
