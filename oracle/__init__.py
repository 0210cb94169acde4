"""FP64 oracle for the object-aware Gaussian rasterization hot path.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg of
the benchmark use this package to decide what the right answer is.  The GPU
library never imports, links or calls it, and it imports nothing from the GPU
library.  Slow on purpose: every Gaussian is evaluated at every pixel.

Contents (each function states the passage of the paper it follows):
  project / render / render_backward   FP64 C (dqo_oracle.c), via ctypes
  tile_rects / pair_order              binning and (tile, depth) order, numpy
  object_loss                          Eq. (10)-(14) read as L1 colour, L1 depth,
                                       object cross-entropy
  job_targets / object_loss_views      the same loss over windows of whole-scene
                                       views and per-object jobs (Eq. (12)-(13))
  adam                                 the optimizer step (PyTorch semantics)
  dual_quadric_* / fit_dual_quadric    Eq. (1)-(4): quadric from boxes, its
                                       decomposition and its projection
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "libdqo_oracle.so")

# Readings of the rasterizer constants the paper leaves open (see the design notes):
DEFAULTS = dict(z_near=0.2, dilation=0.3, q_max=9.0, alpha_min=1.0 / 255.0,
                alpha_max=0.99, t_min=1e-4, bg=(0.0, 0.0, 0.0))
CE_EPS = 1e-6


class _OCam(ctypes.Structure):
    _fields_ = [("R", ctypes.c_double * 9), ("t", ctypes.c_double * 3),
                ("fx", ctypes.c_double), ("fy", ctypes.c_double),
                ("cx", ctypes.c_double), ("cy", ctypes.c_double),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


class _OCfg(ctypes.Structure):
    _fields_ = [("z_near", ctypes.c_double), ("dilation", ctypes.c_double),
                ("q_max", ctypes.c_double), ("alpha_min", ctypes.c_double),
                ("alpha_max", ctypes.c_double), ("t_min", ctypes.c_double),
                ("bg", ctypes.c_double * 3)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIBPATH):
            from . import build as _b
            _b.build()
        _lib = ctypes.CDLL(_LIBPATH)
        P = ctypes.POINTER
        d, i64, i32 = ctypes.c_double, ctypes.c_int64, ctypes.c_int32
        _lib.oracle_project.argtypes = [i64, P(d), P(_OCam), P(_OCfg), P(d)]
        _lib.oracle_render.argtypes = [i64, P(d), P(i32), P(_OCam), P(_OCfg), ctypes.c_int, i64,
                                       P(i64), P(d), P(d), P(d), P(d), P(i64), P(i32), P(d), P(d), P(d)]
        _lib.oracle_render.restype = ctypes.c_int
        _lib.oracle_render_backward.argtypes = [i64, P(d), P(i32), P(_OCam), P(_OCfg), ctypes.c_int,
                                                i64, P(i64), P(d), P(d), P(d), P(d), P(d), P(d)]
        _lib.oracle_render_backward.restype = ctypes.c_int
        _lib.oracle_num_threads.restype = ctypes.c_int
    return _lib


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def _ptr(a, ctype):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _cam(cam) -> _OCam:
    c = _OCam()
    R = np.asarray(cam["R"], dtype=np.float64).reshape(9)
    t = np.asarray(cam["t"], dtype=np.float64).reshape(3)
    for k in range(9):
        c.R[k] = float(R[k])
    for k in range(3):
        c.t[k] = float(t[k])
    c.fx, c.fy, c.cx, c.cy = (float(cam[k]) for k in ("fx", "fy", "cx", "cy"))
    c.width, c.height = int(cam["width"]), int(cam["height"])
    return c


def _cfg(cfg) -> _OCfg:
    v = dict(DEFAULTS)
    if cfg:
        v.update(cfg)
    c = _OCfg()
    for k in ("z_near", "dilation", "q_max", "alpha_min", "alpha_max", "t_min"):
        setattr(c, k, float(v[k]))
    for k in range(3):
        c.bg[k] = float(v["bg"][k])
    return c


def _params64(params):
    p = np.ascontiguousarray(np.asarray(params, dtype=np.float64))
    assert p.ndim == 2 and p.shape[0] == 14, "params must be [14][n]"
    return p


# ---------------------------------------------------------------- projection
def project(params, cam, cfg=None):
    """EWA projection of every Gaussian (the Gaussian/quadric shape of Eq. (2)).

    Returns a dict of FP64 arrays of length n: visible, x, y, z (camera frame),
    mx, my (2D mean, pixels), s00, s01, s11 (2D covariance incl. dilation),
    A, B, C (conic), ex, ey (3-sigma extents), o (opacity)."""
    p = _params64(params)
    n = p.shape[1]
    out = np.zeros((max(n, 1), 16), dtype=np.float64)
    c, g = _cam(cam), _cfg(cfg)
    _load().oracle_project(n, _ptr(p, ctypes.c_double), ctypes.byref(c), ctypes.byref(g),
                           _ptr(out, ctypes.c_double))
    out = out[:n]
    names = ["visible", "x", "y", "z", "mx", "my", "s00", "s01", "s11", "A", "B", "C",
             "ex", "ey", "o"]
    res = {k: out[:, j].copy() for j, k in enumerate(names)}
    res["visible"] = res["visible"] > 0.5
    return res


def _pixlist(cam, pix):
    W, H = int(cam["width"]), int(cam["height"])
    if pix is None:
        return np.arange(W * H, dtype=np.int64), True
    return np.ascontiguousarray(np.asarray(pix, dtype=np.int64)), False


# ------------------------------------------------------------------- forward
def render(params, ids, cam, cfg=None, K=0, pix=None, want_P=True):
    """Forward image formation: alpha blending of colour and depth (Sec. III-D)
    and the per-object instance channels ins_k of Eq. (12), read as
    transmittance-weighted sums so that sum_k P_k + T_final = 1.

    pix: flat pixel indices (v * W + u) to evaluate, or None for the whole image.
    Returns C (3, npix), D, Tf, P (K, npix) or None, last (Gaussian index or -1),
    nblend, margin, margin_clamp, depth_gap; reshaped to (…, H, W) when pix is None."""
    p = _params64(params)
    n = p.shape[1]
    ids = np.ascontiguousarray(np.asarray(ids, dtype=np.int32))
    assert ids.shape == (n,)
    px, full = _pixlist(cam, pix)
    npix = px.shape[0]
    C = np.zeros((3, npix))
    D = np.zeros(npix)
    Tf = np.zeros(npix)
    P = np.zeros((max(K, 1), npix)) if (want_P and K > 0) else None
    last = np.zeros(npix, dtype=np.int64)
    nb = np.zeros(npix, dtype=np.int32)
    mg = np.zeros(npix)
    mgc = np.zeros(npix)
    gap = np.zeros(npix)
    c, g = _cam(cam), _cfg(cfg)
    rc = _load().oracle_render(n, _ptr(p, ctypes.c_double), _ptr(ids, ctypes.c_int32), ctypes.byref(c),
                               ctypes.byref(g), int(K), npix, _ptr(px, ctypes.c_int64),
                               _ptr(C, ctypes.c_double), _ptr(D, ctypes.c_double),
                               _ptr(Tf, ctypes.c_double), _ptr(P, ctypes.c_double),
                               _ptr(last, ctypes.c_int64), _ptr(nb, ctypes.c_int32),
                               _ptr(mg, ctypes.c_double), _ptr(mgc, ctypes.c_double), _ptr(gap, ctypes.c_double))
    if rc != 0:
        raise MemoryError("oracle_render failed")
    out = dict(C=C, D=D, Tf=Tf, P=P, last=last, nblend=nb, margin=mg, margin_clamp=mgc, depth_gap=gap)
    if full:
        H, W = int(cam["height"]), int(cam["width"])
        for k, v in list(out.items()):
            if v is not None:
                out[k] = v.reshape(v.shape[:-1] + (H, W))
    return out


def id_map(P, Tf):
    """Object-ID map: argmax over (P_0..P_{K-1}, T_final); lowest index wins ties;
    the last slot means "no object" and is returned as -1."""
    stack = np.concatenate([np.asarray(P), np.asarray(Tf)[None]], axis=0)
    a = np.argmax(stack, axis=0).astype(np.int32)
    a[a == stack.shape[0] - 1] = -1
    return a


# ------------------------------------------------------------------ backward
def render_backward(params, ids, cam, cfg=None, K=0, gC=None, gD=None, gP=None, gT=None, pix=None):
    """Analytic FP64 adjoint of `render` (set of blended Gaussians held fixed),
    chained through the projection to the parameters.  Upstream gradients are
    given per evaluated pixel.  Returns (grads[14][n], g2d[n][10]) with
    g2d = (dmx, dmy, dA, dB, dC, dopacity, dr, dg, db, dz)."""
    p = _params64(params)
    n = p.shape[1]
    ids = np.ascontiguousarray(np.asarray(ids, dtype=np.int32))
    px, _ = _pixlist(cam, pix)
    npix = px.shape[0]

    def flat(a, rows):
        if a is None:
            return None
        a = np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(rows, npix) if rows > 1
                                 else np.asarray(a, dtype=np.float64).reshape(npix))
        return a

    gC = flat(gC, 3) if gC is not None else np.zeros((3, npix))
    gD, gT = flat(gD, 1), flat(gT, 1)
    gP = flat(gP, K) if (gP is not None and K > 1) else (flat(gP, 1) if gP is not None else None)
    grads = np.zeros((14, max(n, 1)))
    g2d = np.zeros((max(n, 1), 10))
    c, g = _cam(cam), _cfg(cfg)
    rc = _load().oracle_render_backward(n, _ptr(p, ctypes.c_double), _ptr(ids, ctypes.c_int32),
                                        ctypes.byref(c), ctypes.byref(g), int(K), npix,
                                        _ptr(px, ctypes.c_int64), _ptr(gC, ctypes.c_double),
                                        _ptr(gD, ctypes.c_double), _ptr(gP, ctypes.c_double),
                                        _ptr(gT, ctypes.c_double), _ptr(grads, ctypes.c_double),
                                        _ptr(g2d, ctypes.c_double))
    if rc != 0:
        raise MemoryError("oracle_render_backward failed")
    return grads[:, :n], g2d[:n]


# ------------------------------------------------------------------- binning
def tile_rects(proj, cam, tile=(16, 16), edge_tol=1e-3):
    """Tiles covered by each visible Gaussian's 3-sigma box, clipped to the tile
    grid: (x0, y0, x1, y1) inclusive, plus an `ambiguous` flag for Gaussians
    whose box edge lies within edge_tol pixels of a tile boundary or whose
    visibility decision is within 1e-6 of z_near."""
    tw, th = tile
    W, H = int(cam["width"]), int(cam["height"])
    tx, ty = (W + tw - 1) // tw, (H + th - 1) // th
    vis = proj["visible"]
    with np.errstate(invalid="ignore"):
        lo_x, hi_x = proj["mx"] - proj["ex"], proj["mx"] + proj["ex"]
        lo_y, hi_y = proj["my"] - proj["ey"], proj["my"] + proj["ey"]
        x0 = np.maximum(np.floor(lo_x / tw), 0)
        x1 = np.minimum(np.floor(hi_x / tw), tx - 1)
        y0 = np.maximum(np.floor(lo_y / th), 0)
        y1 = np.minimum(np.floor(hi_y / th), ty - 1)
    ok = vis & (x0 <= x1) & (y0 <= y1)
    amb = np.zeros_like(vis)
    with np.errstate(invalid="ignore"):
        for v, t in ((lo_x, tw), (hi_x, tw), (lo_y, th), (hi_y, th)):
            frac = np.abs(v / t - np.round(v / t)) * t
            amb |= vis & (frac < edge_tol)
    amb |= np.abs(proj["z"] - DEFAULTS["z_near"]) < 1e-6 * DEFAULTS["z_near"]
    rect = np.stack([x0, y0, x1, y1], axis=1)
    rect = np.where(np.isfinite(rect), rect, -1).astype(np.int64)
    rect[~ok] = [0, 0, -1, -1]
    return rect, amb


def pair_order(proj, rect, cam, tile=(16, 16)):
    """All (tile, Gaussian) pairs in the order blending needs them: by tile,
    then camera depth ascending, then Gaussian index (a stable lexsort)."""
    tw = tile[0]
    W = int(cam["width"])
    tx = (W + tw - 1) // tw
    tiles, gs = [], []
    for i in np.nonzero(rect[:, 2] >= rect[:, 0])[0]:
        x0, y0, x1, y1 = rect[i]
        for yy in range(y0, y1 + 1):
            for xx in range(x0, x1 + 1):
                tiles.append(yy * tx + xx)
                gs.append(i)
    tiles = np.asarray(tiles, dtype=np.int64)
    gs = np.asarray(gs, dtype=np.int64)
    if tiles.size == 0:
        return tiles, gs
    o = np.lexsort((gs, proj["z"][gs], tiles))
    return tiles[o], gs[o]


# ---------------------------------------------------------------------- loss
def object_loss(C, D, p_t, tC, tD, t_id, w_rgb=1.0, w_depth=1.0, lam=1.0, eps=CE_EPS):
    """Object loss of Eq. (10)-(14): L = w_rgb L_rgb + w_depth L_depth + lam L_obj
    with L_rgb the mean absolute colour residual over all channels and pixels,
    L_depth the mean absolute depth residual over pixels with valid target depth
    (target > 0), and L_obj the mean of -log max(p_t, eps) where p_t is the
    rendered probability of the pixel's target object (T_final for "no object").
    Returns the scalars and the upstream gradients dL/dC, dL/dD, dL/dp_t."""
    C, D, p_t = (np.asarray(a, dtype=np.float64) for a in (C, D, p_t))
    tC, tD = np.asarray(tC, dtype=np.float64), np.asarray(tD, dtype=np.float64)
    npix = D.size
    r = C - tC
    l_rgb = np.abs(r).sum() / (3 * npix) if npix else 0.0
    valid = tD > 0
    nv = int(valid.sum())
    dr = np.where(valid, D - tD, 0.0)
    l_d = np.abs(dr).sum() / nv if nv else 0.0
    pc = np.maximum(p_t, eps)
    l_obj = (-np.log(pc)).sum() / npix if npix else 0.0
    total = w_rgb * l_rgb + w_depth * l_d + lam * l_obj
    gC = w_rgb * np.sign(r) / (3 * npix) if npix else np.zeros_like(C)
    gD = w_depth * np.sign(dr) / nv if nv else np.zeros_like(D)
    gp = np.where(p_t >= eps, -lam / (npix * np.where(p_t >= eps, p_t, 1.0)), 0.0) if npix else p_t * 0
    return dict(loss=total, l_rgb=l_rgb, l_depth=l_d, l_obj=l_obj, n_valid=nv, gC=gC, gD=gD, gp=gp)


def job_targets(t_id, job):
    """Target of a per-object job (Sec. III-D; objects are optimised in
    parallel, each on its own Gaussians G^k): the job of object k renders
    only G^k, so its instance channel ins_k of Eq. (12) is 1 - T_final, and
    Eq. (13) compares it with the observed mask of k.  As a target map: k
    where the pixel is observed as k, -1 ("not this object", probability
    T_final) elsewhere.  job < 0 (a whole-scene view) keeps t_id."""
    t_id = np.asarray(t_id)
    if job < 0:
        return t_id
    return np.where(t_id == job, job, -1).astype(t_id.dtype)


def object_loss_views(C, D, P, Tf, tC, tD, t_id, jobs=None, windows=None, w_rgb=1.0, w_depth=1.0, lam=1.0,
                      eps=CE_EPS):
    """Object loss of Eq. (10)-(14) over views that are whole-scene renders
    or per-object jobs, each restricted to a pixel window.

    Per view v (images [V][...][H][W]; jobs[v] = -1 or the job's object k;
    windows[v] = (x0, y0, x1, y1), pixels x0 <= u < x1, y0 <= v < y1):
      * the cross-entropy term covers every window pixel, on the probability
        of the target of job_targets (P_t, or T_final for -1);
      * the colour and depth terms cover the window pixels of a whole-scene
        view, and of a job only those observed as its object (Eq. (10)-(11)
        sum over the object's own pixels); depth only where the observed
        depth is > 0.
    Each term is one mean over its pixels of all views together:
    L = w_rgb * sum|C - C^| / (3 N_c) + w_depth * sum|D - D^| / N_d
        + lam * sum -log max(p_t, eps) / N_o.
    Returns the scalars, the counts and dL/dC, dL/dD, dL/dP, dL/dT_final
    (zero outside the counted pixels; no CE gradient where p_t < eps)."""
    C, D, P, Tf = (np.asarray(a, dtype=np.float64) for a in (C, D, P, Tf))
    tC, tD = np.asarray(tC, dtype=np.float64), np.asarray(tD, dtype=np.float64)
    t_id = np.asarray(t_id)
    V, H, W = D.shape
    K = P.shape[1]
    jobs = [-1] * V if jobs is None else list(jobs)
    windows = [(0, 0, W, H)] * V if windows is None else [tuple(w) for w in windows]
    win = np.zeros((V, H, W), bool)
    tgt = np.empty((V, H, W), np.int64)
    for v in range(V):
        x0, y0, x1, y1 = windows[v]
        win[v, max(y0, 0):max(y1, 0), max(x0, 0):max(x1, 0)] = True
        tgt[v] = job_targets(t_id[v], jobs[v])
    colour = win.copy()
    for v in range(V):
        if jobs[v] >= 0:
            colour[v] &= t_id[v] == jobs[v]
    depth_ok = colour & (tD > 0)
    n_c, n_d, n_o = int(colour.sum()), int(depth_ok.sum()), int(win.sum())
    r = C - tC
    l_rgb = np.abs(np.where(colour[:, None], r, 0.0)).sum() / (3 * n_c) if n_c else 0.0
    dr = np.where(depth_ok, D - tD, 0.0)
    l_d = np.abs(dr).sum() / n_d if n_d else 0.0
    p_t = np.where(tgt >= 0, np.take_along_axis(P, np.clip(tgt, 0, K - 1)[:, None], 1)[:, 0], Tf)
    ce = np.where(win, -np.log(np.maximum(p_t, eps)), 0.0)
    l_obj = ce.sum() / n_o if n_o else 0.0
    total = w_rgb * l_rgb + w_depth * l_d + lam * l_obj
    gC = np.where(colour[:, None], w_rgb * np.sign(r) / (3 * n_c), 0.0) if n_c else np.zeros_like(C)
    gD = w_depth * np.sign(dr) / n_d if n_d else np.zeros_like(D)
    gq = np.where(win & (p_t >= eps), -lam / (max(n_o, 1) * np.where(p_t >= eps, p_t, 1.0)), 0.0)
    gP = np.zeros_like(P)
    for k in range(K):
        gP[:, k] = np.where(tgt == k, gq, 0.0)
    gT = np.where(tgt == -1, gq, 0.0)
    return dict(loss=total, l_rgb=l_rgb, l_depth=l_d, l_obj=l_obj, n_colour=n_c, n_depth=n_d, n_obj=n_o,
                gC=gC, gD=gD, gP=gP, gT=gT, gp=gq, target=tgt)


# ---------------------------------------------------------------------- adam
def adam(params, grads, m, v, step, lrs, beta1=0.9, beta2=0.999, eps=1e-15):
    """One Adam step with bias correction (PyTorch semantics), per-row learning
    rate lrs[14].  Returns new (params, m, v)."""
    p, g = np.asarray(params, np.float64), np.asarray(grads, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1 - beta2) * g * g
    bc1 = 1 - beta1 ** step
    bc2 = 1 - beta2 ** step
    lr = np.asarray(lrs, np.float64).reshape(-1, 1)
    p = p - lr * (m / bc1) / (np.sqrt(v / bc2) + eps)
    return p, m, v


# ------------------------------------------------------------------ quadrics
def dual_quadric_from_ellipsoid(mu, R, axes):
    """Q* = Z diag(a^2, b^2, c^2, -1) Z^T with Z = [[R, mu], [0, 1]]: the dual
    quadric of an ellipsoid with centre mu, rotation R and semi-axes (a, b, c),
    the shape that Eq. (2)-(3) decouple."""
    Z = np.eye(4)
    Z[:3, :3] = np.asarray(R, np.float64)
    Z[:3, 3] = np.asarray(mu, np.float64)
    a = np.asarray(axes, np.float64)
    return Z @ np.diag([a[0] ** 2, a[1] ** 2, a[2] ** 2, -1.0]) @ Z.T


def camera_matrix(cam):
    """P = K [R | t] (Eq. (4))."""
    Kc = np.array([[cam["fx"], 0, cam["cx"]], [0, cam["fy"], cam["cy"]], [0, 0, 1.0]])
    Rt = np.concatenate([np.asarray(cam["R"], np.float64).reshape(3, 3),
                         np.asarray(cam["t"], np.float64).reshape(3, 1)], axis=1)
    return Kc @ Rt


def project_dual_quadric(Q, P):
    """Dual conic of a dual quadric, C* = P Q* P^T (Eq. (4), read with the
    transpose on the right so that the product is 3x3 for P in R^{3x4})."""
    return np.asarray(P) @ np.asarray(Q) @ np.asarray(P).T


def conic_box(Cs):
    """Axis-aligned box (x0, y0, x1, y1) tangent to the conic with dual Cs:
    vertical lines l = (1, 0, -x) with l^T Cs l = 0, horizontal likewise."""
    C = np.asarray(Cs, np.float64) / Cs[2, 2]
    dx = np.sqrt(C[0, 2] ** 2 - C[0, 0])
    dy = np.sqrt(C[1, 2] ** 2 - C[1, 1])
    return np.array([C[0, 2] - dx, C[1, 2] - dy, C[0, 2] + dx, C[1, 2] + dy])


QUADRIC_OK, QUADRIC_DEGENERATE, QUADRIC_NOT_ELLIPSOID = 0, 1, 2


def quadric_rows(boxes, Ps, box_view, img_wh=None, border=1.0):
    """Constraint rows of Eq. (1): for each box edge line l, the back-projected
    plane pi = P^T l (normalised) gives pi^T Q* pi = 0, linear in the 10 unique
    entries (Q11,Q12,Q13,Q14,Q22,Q23,Q24,Q33,Q34,Q44).  Edges within `border`
    pixels of the image border are dropped (the object may be truncated)."""
    rows = []
    for b, v in zip(np.asarray(boxes, np.float64), np.asarray(box_view)):
        x0, y0, x1, y1 = b
        P = np.asarray(Ps[v], np.float64)
        lines = []
        Wv, Hv = (img_wh[v] if img_wh is not None else (None, None))
        if Wv is None or x0 > border:
            lines.append((1.0, 0.0, -x0))
        if Wv is None or x1 < Wv - border:
            lines.append((1.0, 0.0, -x1))
        if Hv is None or y0 > border:
            lines.append((0.0, 1.0, -y0))
        if Hv is None or y1 < Hv - border:
            lines.append((0.0, 1.0, -y1))
        for l in lines:
            pi = P.T @ np.asarray(l)
            pi = pi / np.linalg.norm(pi)
            a, b_, c, d = pi
            rows.append([a * a, 2 * a * b_, 2 * a * c, 2 * a * d, b_ * b_, 2 * b_ * c, 2 * b_ * d,
                         c * c, 2 * c * d, d * d])
    return np.asarray(rows, np.float64).reshape(-1, 10)


def _q_from_vec(q):
    i = [[0, 1, 2, 3], [1, 4, 5, 6], [2, 5, 7, 8], [3, 6, 8, 9]]
    return np.asarray(q)[np.asarray(i)]


def fit_dual_quadric(boxes, box_obj, box_view, Ps, n_obj, img_wh=None, border=1.0):
    """Per object: least-squares solution of Eq. (1) over all its box-edge planes
    (the right singular vector of the smallest singular value), scaled so that
    Q*_44 = -1, then decoupled as in Eq. (2)-(3): mu = -Q*[0:3, 3] and
    Q*[0:3, 0:3] + mu mu^T = R diag(a^2, b^2, c^2) R^T.
    Returns dict(Q (n_obj,4,4), mu, R, axes, status)."""
    boxes = np.asarray(boxes, np.float64).reshape(-1, 4)
    box_obj, box_view = np.asarray(box_obj), np.asarray(box_view)
    Q = np.zeros((n_obj, 4, 4))
    mu = np.zeros((n_obj, 3))
    R = np.tile(np.eye(3), (n_obj, 1, 1))
    axes = np.zeros((n_obj, 3))
    status = np.zeros(n_obj, np.int32)
    for k in range(n_obj):
        sel = box_obj == k
        A = quadric_rows(boxes[sel], Ps, box_view[sel], img_wh, border)
        if A.shape[0] < 9:
            status[k] = QUADRIC_DEGENERATE
            continue
        _, s, Vt = np.linalg.svd(A, full_matrices=True)
        if s[8] <= 1e-10 * s[0]:
            status[k] = QUADRIC_DEGENERATE
            continue
        q = Vt[-1]
        Qk = _q_from_vec(q)
        if abs(Qk[3, 3]) <= 1e-12 * np.abs(q).max():
            status[k] = QUADRIC_NOT_ELLIPSOID
            Q[k] = Qk
            continue
        Qk = Qk / (-Qk[3, 3])
        Q[k] = Qk
        mu[k] = -Qk[:3, 3]
        M = Qk[:3, :3] + np.outer(mu[k], mu[k])
        ev, V = np.linalg.eigh(0.5 * (M + M.T))
        if ev.min() <= 0:
            status[k] = QUADRIC_NOT_ELLIPSOID
            continue
        if np.linalg.det(V) < 0:
            V[:, 0] = -V[:, 0]
        axes[k] = np.sqrt(ev)
        R[k] = V
    return dict(Q=Q, mu=mu, R=R, axes=axes, status=status)
