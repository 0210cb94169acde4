"""Oracle of the learned-initialization path (test infrastructure only).

Plain FP64 numpy, written from the definitions; only tests/, the smoke check
and the benchmark's CPU-baseline leg may import it.  It shares no code with
the GPU library.

What it computes:
  * plain initialization: one Gaussian per valid crop pixel, back-projected
    from depth (the paper spawns Gaussians from RGB-D observations, Sec. III-C
    with Eq. (7)-(8); initial opacity 0.9 of opaque Gaussians, Sec. IV);
  * the learned initialization: the same Gaussians with the network's
    per-pixel log-scale offset, opacity logit and colour offset applied, or
    the plain ones for a crop whose predicted error exceeds a threshold;
  * the network: four 3x3 convolutions (5 -> 32 -> 64 -> 64 -> 6 channels,
    zero padding, ReLU between layers) with BF16 weights and BF16 activations
    and exact (here FP64) accumulation, its loss and its gradients;
  * training labels from the Gaussians the plain optimizer converged to.
The network is not in the paper: it is the project's own extension, so its
forward, adjoint and loss are pinned by a library convolution, finite
differences and closed forms rather than by the paper.
"""
from __future__ import annotations

import numpy as np

NET_IN, NET_OUT = 5, 6
NET_CHANNELS = (5, 32, 64, 64, 6)
OPACITY0 = 0.9           # initial opacity of an opaque Gaussian
DEPTH_SCALE = 4.0        # relative-depth input: 4 (d - d_min) / d_min
LOGERR_FLOOR = 1e-4      # realised log-error = log(weighted squared error + floor)


def valid_pixels(rgbdm):
    """A pixel spawns a Gaussian where the mask is set (> 1/2) and depth > 0."""
    return (rgbdm[4] > 0.5) & (rgbdm[3] > 0)


# ------------------------------------------------------------ initialization
def plain_init(rgbdm, cam):
    """One Gaussian per valid pixel, in raster order: mean = back-projection of
    the pixel centre (u + 1/2, v + 1/2) at its depth d (camera -> world with
    the inverse of x_c = R x_w + t), isotropic log-scale log(d / fx) (one pixel
    footprint), identity rotation, opacity 0.9, the pixel's colour.
    Returns params[14][n] and the (v, u) pixel of each Gaussian."""
    ok = valid_pixels(rgbdm)
    vs, us = np.nonzero(ok)
    d = rgbdm[3][vs, us].astype(np.float64)
    xc = np.stack([d * (us + 0.5 - cam["cx"]) / cam["fx"], d * (vs + 0.5 - cam["cy"]) / cam["fy"], d])
    R, t = np.asarray(cam["R"], np.float64), np.asarray(cam["t"], np.float64)
    mu = R.T @ (xc - t[:, None])
    n = d.size
    p = np.zeros((14, n))
    p[0:3] = mu
    p[3:6] = np.log(d / cam["fx"])[None]
    p[6] = 1.0
    p[10] = np.log(OPACITY0 / (1.0 - OPACITY0))
    p[11:14] = rgbdm[0:3][:, vs, us]
    return p, np.stack([vs, us])


def learned_init(rgbdm, cam, pred, use_pred):
    """plain_init with, when use_pred, log-scale += pred[0] (all three axes),
    opacity logit = pred[1], colour += pred[2:5], read at each Gaussian's
    pixel.  pred: (6, H, W)."""
    p, pix = plain_init(rgbdm, cam)
    if use_pred:
        vs, us = pix
        pv = np.asarray(pred, np.float64)[:, vs, us]
        p[3:6] += pv[0][None]
        p[10] = pv[1]
        p[11:14] += pv[2:5]
    return p, pix


def labels(rgbdm, cam, converged):
    """Per valid pixel, from the converged Gaussian spawned there: mean
    log-scale minus the plain value log(d / fx), the opacity logit, and the
    colour minus the pixel's colour.  Returns (5, H, W), zero elsewhere."""
    p0, (vs, us) = plain_init(rgbdm, cam)
    c = np.asarray(converged, np.float64)
    out = np.zeros((5,) + rgbdm.shape[1:])
    out[0][vs, us] = c[3:6].mean(0) - p0[3]
    out[1][vs, us] = c[10]
    out[2:5][:, vs, us] = c[11:14] - p0[11:14]
    return out


def masked_psnr(color, rgbdm):
    """PSNR (peak 1) of a rendered colour image (3, H, W) against the crop's
    colour over its valid pixels."""
    ok = valid_pixels(rgbdm)
    mse = ((np.asarray(color, np.float64) - rgbdm[0:3]) ** 2)[:, ok].mean()
    return 10.0 * np.log10(1.0 / mse)


# ------------------------------------------------------------ the network
def bf16(x):
    """Round to the nearest BF16 value (8 significant bits, ties to even)."""
    x = np.asarray(x, np.float64)
    m, e = np.frexp(x)
    return np.ldexp(np.round(m * 256.0), e - 8)


def net_input(rgbdm):
    """Input channels: r, g, b, 4 (d - d_min) / d_min over valid pixels (0
    elsewhere, d_min the crop's smallest valid depth), valid mask; BF16."""
    ok = valid_pixels(rgbdm)
    x = np.zeros((NET_IN,) + rgbdm.shape[1:])
    x[0:3] = rgbdm[0:3]
    if ok.any():
        d = rgbdm[3].astype(np.float32)
        dmin = d[ok].min()
        rel = (DEPTH_SCALE * ((d - dmin) / dmin).astype(np.float32)).astype(np.float32)
        x[3] = np.where(ok, rel, 0.0)
    x[4] = ok
    return bf16(x)


def conv3x3(x, w, b):
    """Zero-padded 3x3 cross-correlation: z[o, y, x] = b[o] +
    sum_{c, i, j} w[o, c, i, j] x[c, y + i - 1, x + j - 1].  x (C, H, W)."""
    C, H, W = x.shape
    xp = np.zeros((C, H + 2, W + 2))
    xp[:, 1:-1, 1:-1] = x
    z = np.zeros((w.shape[0], H, W)) + np.asarray(b, np.float64)[:, None, None]
    for i in range(3):
        for j in range(3):
            z += np.einsum("oc,chw->ohw", w[:, :, i, j], xp[:, i:i + H, j:j + W])
    return z


def conv3x3_adjoint(g, w, x):
    """Gradients of sum(g * conv3x3(x, w, b)): w.r.t. x, w and b."""
    C, H, W = x.shape
    xp = np.zeros((C, H + 2, W + 2))
    xp[:, 1:-1, 1:-1] = x
    gxp = np.zeros_like(xp)
    gw = np.zeros_like(w, dtype=np.float64)
    for i in range(3):
        for j in range(3):
            gw[:, :, i, j] = np.einsum("ohw,chw->oc", g, xp[:, i:i + H, j:j + W])
            gxp[:, i:i + H, j:j + W] += np.einsum("oc,ohw->chw", w[:, :, i, j], g)
    return gxp[:, 1:-1, 1:-1], gw, g.sum((1, 2))


def init_net(seed):
    """He-normal weights (std sqrt(2 / (9 cin))), zero biases: a list of
    (w (cout, cin, 3, 3), b (cout,)) in FP64."""
    rng = np.random.default_rng(seed)
    layers = []
    for cin, cout in zip(NET_CHANNELS[:-1], NET_CHANNELS[1:]):
        layers.append((rng.normal(0.0, np.sqrt(2.0 / (9 * cin)), size=(cout, cin, 3, 3)), np.zeros(cout)))
    return layers


def net_forward(x, layers, rounding=True):
    """Activations a0 = x, a_l = bf16(relu(conv(a_{l-1}))) for l < 4 and the
    FP32-exact output z4 = conv(a3) (not rounded).  Weights enter rounded to
    BF16 (biases stay exact).  rounding=False gives the same network without
    any BF16 rounding (for finite differences).  Returns (acts, out)."""
    r = bf16 if rounding else (lambda v: np.asarray(v, np.float64))
    acts = [r(x)]
    for li, (w, b) in enumerate(layers):
        z = conv3x3(acts[-1], r(w), b)
        if li < len(layers) - 1:
            acts.append(r(np.maximum(z, 0.0)))
        else:
            return acts, z


def net_loss(out, lab, ok, chan_w):
    """Loss over the valid pixels (M of them, summed over crops):
      e_c = out_c - label_c (c < 5),  s = sum_c w_c e_c^2,
      r = log(s + 1e-4) taken as a constant (the realised log-error),
      L = (1/M) sum_p [ s + (out_5 - r)^2 ].
    out (B, 6, H, W), lab (B, 5, H, W), ok (B, H, W) bool.  Returns (L, dL/dout)."""
    out = np.asarray(out, np.float64)
    M = max(int(ok.sum()), 1)
    w = np.asarray(chan_w, np.float64)[None, :, None, None]
    e = out[:, 0:5] - lab
    s = (w * e * e).sum(1)
    r = np.log(s + LOGERR_FLOOR)
    d5 = out[:, 5] - r
    L = float(((s + d5 * d5) * ok).sum() / M)
    g = np.zeros_like(out)
    g[:, 0:5] = 2.0 * w * e * ok[:, None] / M
    g[:, 5] = 2.0 * d5 * ok / M
    return L, g


def net_backward(acts, layers, g_out, rounding=True):
    """Adjoint of net_forward for one crop: g4 = bf16(dL/dz4); for l = 4..1:
    dW_l, db_l from g_l and a_{l-1}; g_{l-1} = bf16(conv^T(g_l) * [a_{l-1} > 0]).
    Returns [(dW_l, db_l)] in layer order."""
    r = bf16 if rounding else (lambda v: np.asarray(v, np.float64))
    g = r(g_out)
    grads = [None] * len(layers)
    for li in range(len(layers) - 1, -1, -1):
        w, _ = layers[li]
        gx, gw, gb = conv3x3_adjoint(g, r(w), acts[li])
        grads[li] = (gw, gb)
        if li > 0:
            g = r(gx * (acts[li] > 0))
    return grads
