"""GPU: the learned-initialization path against its oracle — network forward,
loss and weight gradients (MFMA BF16 kernels), crop initialization (plain and
learned), labels, masked PSNR and the fallback decision; crops batched with
per-view Gaussian segments render exactly like crops rendered one by one.

Network tolerance: both sides round weights and activations to BF16; they
differ by FP32 (GPU) versus FP64 (oracle) accumulation, which flips the BF16
rounding of about one activation in a few thousand by one BF16 step (2^-8
relative).  A flip moves a sum by at most |w| 2^-8 |a| of the term it enters,
so each entry is held to the dot-product error bound
|g - o| <= 2^-6 sum |w| |a| (four BF16 steps of the sum of absolute terms,
computed by the oracle with absolute values), and every result to 2e-3
normwise."""
import numpy as np
import pytest
import torch

from oracle import learned as OL
from paper_2503_02223_amd import binding as B
from paper_2503_02223_amd import crops as CR
from paper_2503_02223_amd import learned as L
from tests.gpu_util import FWD_RTOL, close, to_dev

pytestmark = pytest.mark.gpu

NET_ULPS = 2.0 ** -6
NET_NORM = 2e-3


def _close_net(g, o, bound, what):
    g, o = np.asarray(g, np.float64), np.asarray(o, np.float64)
    err = np.abs(g - o)
    tol = NET_ULPS * np.asarray(bound) + 1e-12
    bad = err > tol
    assert not bad.any(), (f"{what}: {bad.sum()} / {bad.size} entries beyond 2^-6 sum|w||a|; worst ratio "
                           f"{(err / tol).max():.2f}")
    rel = np.linalg.norm(g - o) / np.linalg.norm(o)
    assert rel <= NET_NORM, f"{what}: normwise {rel:.2e}"


def _abs_layers(layers):
    return [(np.abs(w), np.zeros_like(b)) for w, b in layers]


def _layers(seed):
    rng = np.random.default_rng(seed)
    return [(w, rng.normal(0, 0.05, size=b.shape)) for w, b in L.he_init(seed)]


def _small_crops(seed, count, H, W):
    """Crops of H x W cut from the centre of 128 x 128 renders."""
    full = CR.make_crops(seed, count)
    y0, x0 = (128 - H) // 2, (128 - W) // 2
    return np.ascontiguousarray(full[:, :, y0:y0 + H, x0:x0 + W])


@pytest.mark.parametrize("shape", [(2, 128, 128), (3, 48, 32)])
def test_net_forward_matches_oracle(shape):
    Bn, H, W = shape
    crops = _small_crops(11, Bn, H, W)
    layers = _layers(1)
    net = L.Net(theta=L.pack_layers(layers))
    out = net.forward(to_dev(crops)).cpu().numpy()
    # the packed theta round-trips
    for (w0, b0), (w1, b1) in zip(layers, L.unpack_theta(net.theta.cpu().numpy())):
        np.testing.assert_array_equal(np.float32(w0), w1)
        np.testing.assert_array_equal(np.float32(b0), b1)
    layers32 = [(np.float32(w).astype(np.float64), np.float32(b).astype(np.float64)) for w, b in layers]
    for b in range(Bn):
        acts, ref = OL.net_forward(OL.net_input(crops[b]), layers32)
        bound = OL.conv3x3(acts[3], OL.bf16(np.abs(layers32[3][0])), np.zeros(6))
        _close_net(out[b], ref, bound, f"net output crop {b}")


def test_net_loss_and_weight_gradients_match_oracle():
    Bn, H, W = 2, 64, 48
    crops = _small_crops(12, Bn, H, W)
    layers = _layers(2)
    layers32 = [(np.float32(w).astype(np.float64), np.float32(b).astype(np.float64)) for w, b in layers]
    rng = np.random.default_rng(3)
    labels = rng.normal(0, 0.5, size=(Bn, 5, H, W)).astype(np.float32)
    chan_w = [2.0, 0.5, 4.0, 4.0, 4.0]
    net = L.Net(theta=L.pack_layers(layers))
    rg = to_dev(crops)
    out = net.forward(rg)
    net.loss_backward(rg, out, to_dev(labels), chan_w)
    torch.cuda.synchronize()
    out_np = out.cpu().numpy()
    acts, outs = [], []
    for b in range(Bn):
        a, o = OL.net_forward(OL.net_input(crops[b]), layers32)
        acts.append(a)
        outs.append(o)
    ok = np.stack([OL.valid_pixels(c) for c in crops])
    # the loss of the GPU's own output (its FP32 output is the input of the loss)
    Lg, g_out = OL.net_loss(out_np, labels, ok, chan_w)
    lo = net.loss.cpu().numpy()
    assert lo[0] == pytest.approx(Lg, rel=1e-5)
    Lo, g_out_o = OL.net_loss(np.stack(outs), labels, ok, chan_w)
    assert lo[0] == pytest.approx(Lo, rel=5e-3)
    grads, bounds = None, None
    add = lambda u, v: v if u is None else [(x[0] + y[0], x[1] + y[1]) for x, y in zip(u, v)]
    for b in range(Bn):
        grads = add(grads, OL.net_backward(acts[b], layers32, g_out_o[b]))
        bounds = add(bounds, OL.net_backward(acts[b], _abs_layers(layers32), np.abs(g_out_o[b])))
    got = L.unpack_theta(net.grad.cpu().numpy())
    for l in range(4):
        _close_net(got[l][0], grads[l][0], bounds[l][0], f"dW layer {l + 1}")
        _close_net(got[l][1], grads[l][1], bounds[l][1], f"db layer {l + 1}")
    # padded weight entries receive exactly zero gradient
    g_all = net.grad.cpu().numpy()
    mask = L.pack_layers([(np.ones_like(w), np.ones_like(b)) for w, b in layers]) != 0
    assert not g_all[~mask].any()


def test_net_training_step_reduces_loss():
    crops = _small_crops(13, 4, 64, 64)
    rng = np.random.default_rng(4)
    labels = np.zeros((4, 5, 64, 64), np.float32)
    labels[:, 0] = 0.3 * crops[:, 3] - 0.1
    labels[:, 1] = 2.0 + crops[:, 0]
    labels[:, 2:5] = 0.1 * (crops[:, 0:3] - 0.5) + 0.01 * rng.normal(size=(4, 3, 64, 64))
    net = L.Net(seed=5)
    rg, lab = to_dev(crops), to_dev(labels)
    losses = []
    for _ in range(60):
        net.train_step(rg, lab, [1.0] * 5, 3e-3)
        losses.append(float(net.loss[0].item()))
    assert losses[-1] < 0.5 * losses[0], losses[::10]
    assert int(net.d_step.item()) == 60


def _rot_cam(size=128):
    cam = CR.crop_camera(size)
    a = 0.2
    cam["R"] = np.array([[np.cos(a), -np.sin(a), 0], [np.sin(a), np.cos(a), 0], [0, 0, 1.0]])
    cam["t"] = np.array([0.05, 0.1, -0.2])
    return cam


def test_init_gaussians_plain_and_learned_match_oracle():
    crops = CR.make_crops(21, 3)
    cams = [CR.crop_camera(), _rot_cam(), CR.crop_camera()]
    counts = L.valid_counts(crops)
    offsets = np.concatenate([[0], np.cumsum(counts)])
    rng = np.random.default_rng(5)
    pred = rng.normal(0, 0.3, size=(3, 6, 128, 128)).astype(np.float32)
    use = torch.tensor([1, 1, 0], dtype=torch.int32, device="cuda")
    ctx = B.Context()
    rg = to_dev(crops)
    p_plain, ids, _ = L.init_gaussians(ctx, rg, cams, offsets, obj_id=7)
    p_learn, _, _ = L.init_gaussians(ctx, rg, cams, offsets, pred=to_dev(pred), use_pred=use)
    torch.cuda.synchronize()
    assert (ids.cpu().numpy() == 7).all()
    for b in range(3):
        s = slice(offsets[b], offsets[b + 1])
        ref, _ = OL.plain_init(crops[b], cams[b])
        close(p_plain.cpu().numpy()[:, s], ref, 1e-5, what=f"plain crop {b}")
        refl, _ = OL.learned_init(crops[b], cams[b], pred[b], bool(use[b].item()))
        close(p_learn.cpu().numpy()[:, s], refl, 1e-5, what=f"learned crop {b}")


def test_labels_match_oracle():
    crops = CR.make_crops(22, 2)
    cams = [CR.crop_camera()] * 2
    counts = L.valid_counts(crops)
    offsets = np.concatenate([[0], np.cumsum(counts)])
    rng = np.random.default_rng(6)
    conv = []
    for b in range(2):
        p, _ = OL.learned_init(crops[b], cams[b], rng.normal(0, 0.3, size=(6, 128, 128)), True)
        p[3:6] += rng.normal(0, 0.05, size=p[3:6].shape)  # anisotropic after optimization
        conv.append(p)
    conv = np.concatenate(conv, 1)
    ctx = B.Context()
    off = torch.tensor(offsets, device="cuda")
    lab = L.init_labels(ctx, to_dev(crops), cams, off, to_dev(conv)).cpu().numpy()
    for b in range(2):
        ref = OL.labels(crops[b], cams[b], conv[:, offsets[b]:offsets[b + 1]])
        # the log-scale label is a difference of two ~ -5 values held in FP32
        close(lab[b], ref, FWD_RTOL, what=f"labels crop {b}")


def test_masked_psnr_and_fallback_match_oracle():
    crops = CR.make_crops(23, 3)
    rng = np.random.default_rng(7)
    color = (crops[:, 0:3] + rng.normal(0, 0.05, size=(3, 3, 128, 128))).astype(np.float32)
    ctx = B.Context()
    ps = L.masked_psnr(ctx, to_dev(color), to_dev(crops)).cpu().numpy()
    for b in range(3):
        assert ps[b] == pytest.approx(OL.masked_psnr(color[b], crops[b]), rel=1e-9)
    out = rng.normal(0, 1, size=(3, 6, 128, 128)).astype(np.float32)
    means = np.array([out[b, 5][OL.valid_pixels(crops[b])].mean() for b in range(3)])
    srt = np.sort(means)
    thr = float(0.5 * (srt[0] + srt[1]))  # away from every crop's mean
    net = L.Net(ctx=ctx)
    use, mean = net.fallback(to_dev(crops), to_dev(out), thr)
    np.testing.assert_allclose(mean.cpu().numpy(), means, rtol=1e-4, atol=1e-6)
    np.testing.assert_array_equal(use.cpu().numpy(), (means <= thr).astype(np.int32))


def test_segmented_crop_batch_renders_like_single_crops(oracle):
    crops = CR.make_crops(24, 3)
    ctx = B.Context()
    rg = to_dev(crops)
    batch = L.CropOptimizer(ctx, rg, crops)
    r = batch.tr.r
    img = r.frame.new_images()
    r.bin(batch.tr.params, batch.tr.ids, grow=False)
    r.frame.render_forward(img)
    torch.cuda.synchronize()
    cb = img["color"].cpu().numpy()
    for b in range(3):
        single = L.CropOptimizer(ctx, rg[b:b + 1].contiguous(), crops[b:b + 1])
        rs = single.tr.r
        im1 = rs.frame.new_images()
        rs.bin(single.tr.params, single.tr.ids, grow=False)
        rs.frame.render_forward(im1)
        torch.cuda.synchronize()
        assert np.array_equal(im1["color"][0].cpu().numpy(), cb[b]), f"crop {b}"
        p, _ = OL.plain_init(crops[b], CR.crop_camera())
        ref = oracle.render(p, np.zeros(p.shape[1], np.int32), CR.crop_camera(), K=1)
        ok = (ref["margin"] > 1e-4) & (ref["depth_gap"] > 1e-6)
        close(cb[b], ref["C"], FWD_RTOL, ok, f"colour crop {b}")


def test_plain_optimizer_on_crops_improves_psnr():
    crops = CR.make_crops(25, 2)
    ctx = B.Context()
    rgbdm, labels, opt = L.label_batch(ctx, crops, iters=0)
    p0 = opt.final_psnr().cpu().numpy()
    opt.reset()
    opt.run(80, record_psnr=True)
    p1 = opt.final_psnr().cpu().numpy()
    hist = opt.psnr_hist.cpu().numpy()
    np.testing.assert_allclose(hist[0], p0, rtol=1e-9)
    assert (p1 > p0 + 1.0).all(), (p0, p1)
    opt.tr.check()


def test_trained_network_reaches_plain_psnr_in_fewer_iterations():
    """The committed network (trained by bench.py --workload learned-init on
    16,000 crops, 12,000 steps) against the plain initialization on held-out objects: the
    learned start reaches the PSNR that the plain start has after 300
    iterations in fewer iterations."""
    import os
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2503_02223_amd", "data",
                        "learned_init.npz")
    ctx = L.crop_context()
    net, _, thr = L.load_model(path, ctx=ctx)
    crops = L.make_crop_set(3, 8)  # the held-out seed of the benchmark
    recs, summary = L.time_to_psnr(ctx, net, thr, crops, iters=300)
    assert summary["median_iters_learned"] < 300, recs
    assert summary["mean_iters_learned"] < 300, recs
    assert summary["mean_seconds_learned"] < summary["mean_seconds_plain"], summary
