"""Oracle of the incremental update (test infrastructure only; numpy, FP64:
images given in FP32 are widened first, and the returned margin tells a test
which pixels sit too close to a threshold for the two precisions to agree).

Sec. III-C, Eq. (7)-(8): after a frame is rendered, the pixels of object k
whose geometry is missing or unstable form Mask_geo (the rendered instance
probability of the observed object falls below theta_alpha, or the rendered
depth is off the observed depth by more than theta_d) and the pixels whose
colour is wrong form Mask_rgb (colour error above theta_c); Eq. (8) restricts
both to the pixels observed as object k.  New opaque Gaussians (OG, opacity
0.9) are added at Mask_geo pixels for geometry and transparent ones (TG,
opacity 0.1, Sec. IV) at the remaining Mask_rgb pixels for colour, each
back-projected from the observed depth.

Readings: theta_alpha = 0.5 (unstated in the paper); theta_d = theta_c = 0.1
(stated); the depth test applies where the observed depth is > 0; the colour
error is the mean absolute difference over r, g, b; ins of a pixel is the
rendered probability of the object it is observed as (P_t), and pixels
observed as no object (t = -1) are in no mask.
"""
from __future__ import annotations

import numpy as np

THETA_ALPHA, THETA_D, THETA_C = 0.5, 0.1, 0.1
OG, TG = 0.9, 0.1
GEO, RGB = 1, 2


def masks(C, D, P, target_color, target_depth, target_id, theta_alpha=THETA_ALPHA, theta_d=THETA_D,
          theta_c=THETA_C):
    """Per view: C (3, H, W), D (H, W), P (K, H, W) rendered; targets (3, H,
    W), (H, W), id (H, W).  Returns the mask (H, W) uint8 (bit 0 geo, bit 1
    rgb) and, per object k < K, the geo and rgb pixel counts (K, 2), plus the
    margin of each pixel's decisions to their thresholds (H, W) (relative,
    for tests that exclude near-threshold pixels)."""
    K = P.shape[0]
    t = np.asarray(target_id)
    obj = (t >= 0) & (t < K)
    tt = np.where(obj, t, 0)
    ins = np.take_along_axis(np.asarray(P, np.float64), tt[None], 0)[0]
    d_obs = np.asarray(target_depth, np.float64)
    derr = np.abs(np.asarray(D, np.float64) - d_obs)
    cerr = np.abs(np.asarray(C, np.float64) - np.asarray(target_color, np.float64)).mean(0)
    geo = obj & ((ins < theta_alpha) | ((d_obs > 0) & (derr > theta_d)))
    rgb = obj & (cerr > theta_c)
    m = (geo * GEO + rgb * RGB).astype(np.uint8)
    counts = np.zeros((K, 2), np.int64)
    for k in range(K):
        sel = t == k
        counts[k, 0] = (geo & sel).sum()
        counts[k, 1] = (rgb & sel).sum()
    margin = np.minimum(np.abs(ins - theta_alpha) / theta_alpha,
                        np.minimum(np.where(d_obs > 0, np.abs(derr - theta_d) / theta_d, np.inf),
                                   np.abs(cerr - theta_c) / theta_c))
    return m, counts, margin


def densify(mask, target_color, target_depth, target_id, cam):
    """New Gaussians of one view, in raster order: at pixels with observed
    depth d > 0 that are in Mask_geo an OG Gaussian, else in Mask_rgb a TG
    Gaussian; mean = back-projection of the pixel centre (u + 1/2, v + 1/2)
    at depth d through the inverse of x_c = R x_w + t, isotropic log-scale
    log(d / fx), identity rotation, opacity logit of 0.9 or 0.1, the observed
    colour, id = the observed id.  Returns params (14, n) and ids (n,)."""
    m = np.asarray(mask)
    d = np.asarray(target_depth, np.float64)
    sel = ((m & GEO) > 0) | ((m & RGB) > 0)
    sel &= d > 0
    vs, us = np.nonzero(sel)
    dd = d[vs, us]
    xc = np.stack([dd * (us + 0.5 - cam["cx"]) / cam["fx"], dd * (vs + 0.5 - cam["cy"]) / cam["fy"], dd])
    R, tr = np.asarray(cam["R"], np.float64), np.asarray(cam["t"], np.float64)
    p = np.zeros((14, vs.size))
    p[0:3] = R.T @ (xc - tr[:, None])
    p[3:6] = np.log(dd / cam["fx"])[None]
    p[6] = 1.0
    og = (m[vs, us] & GEO) > 0
    p[10] = np.where(og, np.log(OG / (1 - OG)), np.log(TG / (1 - TG)))
    p[11:14] = np.asarray(target_color, np.float64)[:, vs, us]
    return p, np.asarray(target_id)[vs, us].astype(np.int32)
