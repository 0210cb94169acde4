"""Pins for the learned-initialization oracle: the convolution against
torch's conv2d (a library routine), adjoints against central finite
differences, BF16 rounding against torch's float32 -> bfloat16 conversion,
the plain initialization against the pinhole model, and label/initialization
round trips."""
import numpy as np
import pytest
import torch

from oracle import learned as OL
from paper_2503_02223_amd import crops


def _rng_crop(seed, H=12, W=10):
    rng = np.random.default_rng(seed)
    c = np.zeros((5, H, W), np.float32)
    c[0:3] = rng.uniform(0, 1, (3, H, W))
    c[3] = rng.uniform(0.5, 1.5, (H, W))
    c[4] = rng.uniform(0, 1, (H, W)) > 0.3
    c[3][rng.uniform(0, 1, (H, W)) < 0.1] = 0.0  # a few holes in the depth
    return c


def test_conv_matches_torch_conv2d():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(7, 9, 11))
    w = rng.normal(size=(5, 7, 3, 3))
    b = rng.normal(size=5)
    ref = torch.nn.functional.conv2d(torch.tensor(x)[None], torch.tensor(w), torch.tensor(b), padding=1)[0].numpy()
    np.testing.assert_allclose(OL.conv3x3(x, w, b), ref, rtol=1e-12, atol=1e-12)


def test_conv_adjoint_matches_torch_and_fd():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(4, 6, 5))
    w = rng.normal(size=(3, 4, 3, 3))
    g = rng.normal(size=(3, 6, 5))
    gx, gw, gb = OL.conv3x3_adjoint(g, w, x)
    xt = torch.tensor(x, requires_grad=True)
    wt = torch.tensor(w, requires_grad=True)
    bt = torch.zeros(3, dtype=torch.float64, requires_grad=True)
    (torch.nn.functional.conv2d(xt[None], wt, bt, padding=1)[0] * torch.tensor(g)).sum().backward()
    np.testing.assert_allclose(gx, xt.grad.numpy(), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(gw, wt.grad.numpy(), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(gb, bt.grad.numpy(), rtol=1e-12, atol=1e-12)
    h = 1e-6
    for idx in [(0, 0, 0, 0), (2, 3, 1, 2), (1, 1, 2, 0)]:
        wp, wm = w.copy(), w.copy()
        wp[idx] += h
        wm[idx] -= h
        fd = ((OL.conv3x3(x, wp, np.zeros(3)) - OL.conv3x3(x, wm, np.zeros(3))) * g).sum() / (2 * h)
        assert gw[idx] == pytest.approx(fd, rel=1e-6)


def test_bf16_matches_torch_bfloat16():
    rng = np.random.default_rng(2)
    x = np.concatenate([rng.normal(size=2000) * 10.0 ** rng.integers(-8, 8, 2000),
                        [0.0, 1.0, 1 + 2.0 ** -8, 1 + 3 * 2.0 ** -9, -(1 + 2.0 ** -8), 255.5, 1 + 2.0 ** -7]])
    x32 = x.astype(np.float32)
    ref = torch.tensor(x32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(OL.bf16(x32.astype(np.float64)), ref)
    assert OL.bf16(1 + 2.0 ** -8) == 1.0          # tie -> even
    assert OL.bf16(1 + 3 * 2.0 ** -9) == 1 + 2.0 ** -7


def test_network_adjoint_matches_fd_without_rounding():
    rng = np.random.default_rng(3)
    crop = _rng_crop(3, 8, 8)
    x = OL.net_input(crop)
    layers = OL.init_net(5)
    layers = [(w, rng.normal(0, 0.1, size=b.shape)) for w, b in layers]
    g_out = rng.normal(size=(6, 8, 8))

    def L(ls):
        _, out = OL.net_forward(x, ls, rounding=False)
        return (out * g_out).sum()

    acts, _ = OL.net_forward(x, layers, rounding=False)
    grads = OL.net_backward(acts, layers, g_out, rounding=False)
    h = 1e-6
    for li in range(4):
        w, b = layers[li]
        for idx in [tuple(rng.integers(0, s) for s in w.shape) for _ in range(3)]:
            wp = [(ww.copy(), bb) for ww, bb in layers]
            wm = [(ww.copy(), bb) for ww, bb in layers]
            wp[li][0][idx] += h
            wm[li][0][idx] -= h
            fd = (L(wp) - L(wm)) / (2 * h)
            assert grads[li][0][idx] == pytest.approx(fd, rel=1e-5, abs=1e-8), (li, idx)
        k = int(rng.integers(0, b.shape[0]))
        bp = [(ww, bb.copy()) for ww, bb in layers]
        bm = [(ww, bb.copy()) for ww, bb in layers]
        bp[li][1][k] += h
        bm[li][1][k] -= h
        assert grads[li][1][k] == pytest.approx((L(bp) - L(bm)) / (2 * h), rel=1e-5, abs=1e-8)


def test_loss_closed_form_and_gradient():
    out = np.zeros((1, 6, 1, 2))
    lab = np.zeros((1, 5, 1, 2))
    out[0, 0, 0, 0], lab[0, 0, 0, 0] = 0.5, 0.25       # e0 = 0.25
    out[0, 2, 0, 0] = -0.1                              # e2 = -0.1
    out[0, 5, 0, 0] = -2.0
    out[0, 1, 0, 1] = 7.0                               # masked out
    ok = np.array([[[True, False]]])
    w = np.array([2.0, 1.0, 3.0, 1.0, 1.0])
    L, g = OL.net_loss(out, lab, ok, w)
    s = 2 * 0.25 ** 2 + 3 * 0.01
    r = np.log(s + 1e-4)
    assert L == pytest.approx(s + (-2.0 - r) ** 2, rel=1e-14)
    assert g[0, 0, 0, 0] == pytest.approx(2 * 2 * 0.25)
    assert g[0, 2, 0, 0] == pytest.approx(2 * 3 * -0.1)
    assert g[0, 5, 0, 0] == pytest.approx(2 * (-2.0 - r))
    assert not g[..., 1].any()


def test_plain_init_back_projects_to_pixel_centres_with_one_pixel_footprint():
    crop = _rng_crop(4)
    cam = dict(crops.crop_camera(size=10), fx=90.0, fy=80.0, cx=4.7, cy=6.1, height=12, width=10)
    a = 0.3
    cam["R"] = np.array([[np.cos(a), 0, np.sin(a)], [0, 1, 0], [-np.sin(a), 0, np.cos(a)]])
    cam["t"] = np.array([0.1, -0.2, 0.3])
    p, (vs, us) = OL.plain_init(crop, cam)
    ok = OL.valid_pixels(crop)
    assert p.shape[1] == ok.sum() and (ok[vs, us]).all()
    assert (np.diff(vs * 10 + us) > 0).all()  # raster order
    xc = cam["R"] @ p[0:3] + cam["t"][:, None]
    np.testing.assert_allclose(cam["fx"] * xc[0] / xc[2] + cam["cx"], us + 0.5, atol=1e-9)
    np.testing.assert_allclose(cam["fy"] * xc[1] / xc[2] + cam["cy"], vs + 0.5, atol=1e-9)
    np.testing.assert_allclose(xc[2], crop[3][vs, us], rtol=1e-7)
    np.testing.assert_allclose(cam["fx"] * np.exp(p[3]) / xc[2], 1.0, rtol=1e-7)
    assert np.allclose(p[6], 1) and not p[7:10].any()
    np.testing.assert_allclose(1 / (1 + np.exp(-p[10])), 0.9, rtol=1e-14)
    np.testing.assert_array_equal(p[11:14], crop[0:3][:, vs, us])


def test_labels_invert_learned_init():
    crop = _rng_crop(5)
    cam = crops.crop_camera(size=10)
    cam.update(height=12, width=10, cy=6.0)
    rng = np.random.default_rng(6)
    pred = rng.normal(size=(6, 12, 10))
    conv, (vs, us) = OL.learned_init(crop, cam, pred, True)
    lab = OL.labels(crop, cam, conv)
    np.testing.assert_allclose(lab[:, vs, us], pred[0:5][:, vs, us], atol=1e-12)
    ok = OL.valid_pixels(crop)
    assert not lab[:, ~ok].any()
    plain, _ = OL.plain_init(crop, cam)
    np.testing.assert_array_equal(OL.learned_init(crop, cam, pred, False)[0], plain)


def test_net_input_and_psnr():
    crop = _rng_crop(7)
    x = OL.net_input(crop)
    ok = OL.valid_pixels(crop)
    np.testing.assert_array_equal(x[4], ok)
    assert not x[3][~ok].any() and (x[3][ok] >= 0).all()
    assert x[3][ok].min() == 0.0
    np.testing.assert_array_equal(x[0:3], OL.bf16(crop[0:3].astype(np.float64)))
    col = crop[0:3] + 0.01
    assert OL.masked_psnr(col, crop) == pytest.approx(40.0, abs=1e-4)
