"""GPU: the segmented backward's stored state (boundary states, tile ends and
segment list, kept by the last forward of a frame) when other forwards run
between a forward and its backward.  The backward of the alpha blending
(Sec. III-D) must give the gradients of the images it is handed, whichever
forward ran last; compared with the oracle's adjoint."""
import numpy as np
import pytest
import torch

from paper_2503_02223_amd import binding as B
from paper_2503_02223_amd import scenes
from tests.gpu_util import GRAD_RTOL, close, to_dev, unambiguous

pytestmark = pytest.mark.gpu


def _dense(seed=12):
    # 30k Gaussians on 128x96 with 8x8 tiles: tile ranges of several 64-pair
    # segments, so the backward of a loss-mode forward runs segmented
    return scenes.single_view_scene(seed=seed, n=30000)


def _restarts(r, img, H, W, keep):
    """Pixels whose last blended pair lies past the first segment boundary."""
    rng_t = r.frame.buf("ranges", torch.int32).cpu().numpy().reshape(-1, 2)
    lastpos = img["last"][0].cpu().numpy() if isinstance(img, dict) else img
    ys, xs = np.mgrid[0:H, 0:W]
    tile = (ys // 8) * ((W + 7) // 8) + xs // 8
    return ((lastpos - rng_t[tile, 0]) >= 64) & keep


def ctx_last(C):
    """The `last` image saved by the autograd Function for output C."""
    return C.grad_fn.last[0].cpu().numpy()


def test_autograd_backward_after_another_forward(oracle):
    """Forward A, forward B (other parameters) through one Rasterizer, then
    the backward of A and then that of B: each re-bins from its saved
    parameters, and the segment state of the last forward is not theirs."""
    sc = _dense()
    cam = sc["cams"][0]
    H, W, K = cam["height"], cam["width"], sc["K"]
    pa = sc["params"]
    pb = scenes.perturb(sc["params"], 9)
    r = B.Rasterizer(sc["cams"], pa.shape[1], K, ctx=B.Context(tile_w=8, tile_h=8))
    ids = torch.tensor(sc["ids"], device="cuda")
    ta = to_dev(pa).requires_grad_(True)
    tb = to_dev(pb).requires_grad_(True)
    Ca, Da, Ta, _ = B.rasterize(ta, ids, r, want_probs=False)
    restart_a = _restarts(r, ctx_last(Ca), H, W, True)
    Cb, Db, Tb, _ = B.rasterize(tb, ids, r, want_probs=False)
    for name, params, C, D, T, t, seed in (("A", pa, Ca, Da, Ta, ta, 51), ("B", pb, Cb, Db, Tb, tb, 52)):
        ref = oracle.render(params, sc["ids"], cam, K=K)
        keep = unambiguous(ref, grads=True)
        assert keep.mean() > 0.9
        up = scenes.random_image_grads(seed, (3, H, W))
        for k in up:
            up[k] = up[k] * keep
        L = ((C[0] * to_dev(up["gC"])).sum() + (D[0] * to_dev(up["gD"])).sum() + (T[0] * to_dev(up["gT"])).sum())
        L.backward()
        torch.cuda.synchronize()
        go, _ = oracle.render_backward(params, sc["ids"], cam, K=K, gC=up["gC"], gD=up["gD"], gT=up["gT"])
        assert np.abs(t.grad.cpu().numpy()).max() > 0
        close(t.grad.cpu().numpy(), go, GRAD_RTOL, what=f"grads of forward {name}")
    # the case that needs the check: pixels of A blend past a segment boundary
    assert restart_a.sum() > 100


def test_backward_with_images_of_an_earlier_forward(oracle):
    """One binning, two loss-mode forwards with different targets into
    different images; the backward of the first forward's images (colour,
    depth and target-probability gradients) against the oracle's adjoint, and
    against the same backward run right after its own forward."""
    sc = _dense(13)
    cam = sc["cams"][0]
    H, W, K = cam["height"], cam["width"], sc["K"]
    tg = oracle.render(scenes.perturb(sc["params"], 1), sc["ids"], cam, K=K)
    ta_id = oracle.id_map(tg["P"], tg["Tf"])
    tb_id = np.roll(ta_id, 7, axis=1)
    ref = oracle.render(sc["params"], sc["ids"], cam, K=K)
    keep = unambiguous(ref, grads=True)
    rng = np.random.default_rng(61)
    gC = rng.normal(size=(3, H, W)) * keep
    gD = rng.normal(size=(H, W)) * keep
    gpt = rng.normal(size=(H, W)) * keep
    gP = np.zeros((K, H, W))
    for k in range(K):
        gP[k] = np.where(ta_id == k, gpt, 0.0)
    gT = np.where(ta_id == -1, gpt, 0.0)
    go, _ = oracle.render_backward(sc["params"], sc["ids"], cam, K=K, gC=gC, gD=gD, gP=gP, gT=gT)

    r = B.Rasterizer(sc["cams"], sc["params"].shape[1], K, ctx=B.Context(tile_w=8, tile_h=8))
    p = to_dev(sc["params"])
    ids = torch.tensor(sc["ids"], device="cuda")
    r.bin(p, ids)
    f = r.frame
    target_a = torch.tensor(ta_id[None], dtype=torch.int32, device="cuda")
    target_b = torch.tensor(tb_id[None], dtype=torch.int32, device="cuda")
    grads = dict(d_color=to_dev(gC[None]), d_depth=to_dev(gD[None]), d_p_target=to_dev(gpt[None]))

    img_a = f.new_images(target=target_a)
    f.render_forward(img_a)
    out = torch.empty_like(p)
    f.render_backward(img_a, grads)            # segmented: the states are A's
    f.project_backward(p, out)
    g_direct = out.cpu().numpy()
    assert _restarts(r, img_a, H, W, keep).sum() > 100

    img_b = f.new_images(target=target_b)
    f.render_forward(img_b)                    # the stored states are now B's
    f.render_backward(img_a, grads)            # must not restart from them
    f.project_backward(p, out)
    torch.cuda.synchronize()
    g_after = out.cpu().numpy()
    close(g_direct, go, GRAD_RTOL, what="grads right after the forward")
    close(g_after, go, GRAD_RTOL, what="grads after another forward")


def test_restart_suffix_precision_per_tile(oracle):
    """Per-(tile, Gaussian) gradients at restarts where little transmittance
    is left: upstream gradients on the pixels of single tiles whose pixels
    blend past a segment boundary and end nearly opaque, so the sums behind
    the boundary are small next to the pixel totals.  With the upstream
    confined to one tile, each Gaussian's gradient is its partial in that
    tile, compared with the oracle's adjoint."""
    sc = _dense(14)
    cam = sc["cams"][0]
    H, W, K = cam["height"], cam["width"], sc["K"]
    ref = oracle.render(sc["params"], sc["ids"], cam, K=K)
    keep = unambiguous(ref, grads=True)
    r = B.Rasterizer(sc["cams"], sc["params"].shape[1], K, ctx=B.Context(tile_w=8, tile_h=8))
    p = to_dev(sc["params"])
    ids = torch.tensor(sc["ids"], device="cuda")
    img = r.forward(p, ids)
    torch.cuda.synchronize()
    restart = _restarts(r, img, H, W, keep)
    tf = img["t_final"][0].cpu().numpy()
    ys, xs = np.mgrid[0:H, 0:W]
    tile = (ys // 8) * ((W + 7) // 8) + xs // 8
    n_tiles = tile.max() + 1
    # tiles ranked by their restarted pixels' smallest T_final
    score = np.full(n_tiles, np.inf)
    np.minimum.at(score, tile[restart], tf[restart])
    chosen = np.argsort(score)[:3]
    assert np.isfinite(score[chosen]).all() and score[chosen].max() < 1e-2
    rng = np.random.default_rng(81)
    for t in chosen:
        m = (tile == t) & keep
        gC = rng.normal(size=(3, H, W)) * m
        gD = rng.normal(size=(H, W)) * m
        gT = rng.normal(size=(H, W)) * m
        go, _ = oracle.render_backward(sc["params"], sc["ids"], cam, K=K, gC=gC, gD=gD, gT=gT)
        grads = dict(d_color=to_dev(gC[None]), d_depth=to_dev(gD[None]), d_t_final=to_dev(gT[None]))
        g = r.backward(p, img, grads)
        torch.cuda.synchronize()
        g = g.cpu().numpy()
        touched = np.abs(go).sum(0) > 0
        assert touched.sum() > 20
        close(g[:, touched], go[:, touched], GRAD_RTOL, what=f"tile {t} grads (restart T_final {score[t]:.1e})")
