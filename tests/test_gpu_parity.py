"""GPU parity: every step of the hot path through the C ABI against the FP64
oracle on the same seeded inputs.  Discrete results (binning, sort order, last
contributor, object-id argmax) are compared exactly outside the ambiguity band;
colour/depth to 1e-4 relative; gradients to 1e-3 relative."""
import numpy as np
import pytest
import torch

from paper_2503_02223_amd import binding as B
from paper_2503_02223_amd import scenes
from tests.gpu_util import BAND, FWD_RTOL, GRAD_RTOL, close, pair_items, to_dev, unambiguous

pytestmark = pytest.mark.gpu


def _frame(sc, capacity=None, dtype=torch.float32, ctx=None, K=None):
    n = sc["params"].shape[1]
    K = sc["K"] if K is None else K
    r = B.Rasterizer(sc["cams"], n, K, capacity=capacity, dtype=dtype, ctx=ctx)
    p = to_dev(sc["params"], dtype)
    ids = torch.tensor(sc["ids"], dtype=torch.int32, device="cuda")
    return r, p, ids


@pytest.mark.parametrize("seed", [0, 1])
def test_projection_binning_and_sort(oracle, seed):
    sc = scenes.single_view_scene(seed=seed, n=2000)
    cam = sc["cams"][0]
    r, p, ids = _frame(sc)
    r.bin(p, ids)
    f = r.frame
    torch.cuda.synchronize()
    rc, st, P = f.read_status()
    assert rc == 0 and st == 0
    pr = oracle.project(sc["params"], cam)
    spl = f.buf("splats", torch.float32, 2000 * B.SPLAT_WORDS).view(2000, B.SPLAT_WORDS).cpu().numpy()
    vis = pr["visible"]
    for k, name in ((0, "mx"), (1, "my"), (2, "A"), (3, "B"), (4, "C"), (5, "o"), (6, "z")):
        close(spl[vis, k], pr[name][vis], FWD_RTOL, what=name)
    assert (spl[vis, 7].view(np.int32) == sc["ids"][vis]).all()
    # tile rectangles: exact outside the ambiguity band
    rect_o, amb = oracle.tile_rects(pr, cam, (16, 16))
    rect_g = f.buf("rects", torch.int16, 2000 * 4).view(2000, 4).cpu().numpy().astype(np.int64)
    empty_o = rect_o[:, 2] < rect_o[:, 0]
    empty_g = rect_g[:, 2] < rect_g[:, 0]
    ok = ~amb
    assert (empty_o[ok] == empty_g[ok]).all()
    both = ok & ~empty_o
    assert (rect_o[both] == rect_g[both]).all()
    assert amb.sum() < 20
    # the record's pair-slot words: first slot (the emission offset), x0 | y0 << 16, width
    cnt = f.buf("counts", torch.int32, 2000).cpu().numpy()
    off = f.buf("offsets", torch.int32, 2000).cpu().numpy()
    words = spl.view(np.int32)
    has = cnt > 0
    assert has.sum() > 1000
    assert (words[has, 12] == off[has]).all()
    assert (words[has, 13] == rect_g[has, 0] + (rect_g[has, 1] << 16)).all()
    assert (words[has, 14] == rect_g[has, 2] - rect_g[has, 0] + 1).all()
    assert (cnt[has] == (rect_g[has, 2] - rect_g[has, 0] + 1) * (rect_g[has, 3] - rect_g[has, 1] + 1)).all()
    # pair list: GPU order is exactly the stable (tile, depth bits, index) lexsort of its own keys
    keys = f.buf("pair_keys", torch.int32, P).cpu().numpy().astype(np.int64)
    vals = f.buf("pair_vals", torch.int32, P).cpu().numpy().astype(np.int64)
    zbits = spl[:, 6].astype(np.float32).view(np.uint32).astype(np.int64)
    order = np.lexsort((vals, zbits[vals], keys))
    assert (order == np.arange(P)).all()
    # same pair multiset as the oracle's brute-force binning (unambiguous Gaussians)
    tiles_o, gs_o = oracle.pair_order(pr, rect_o, cam, (16, 16))
    sel_o = ~amb[gs_o]
    sel_g = ~amb[vals]
    a = sorted(zip(tiles_o[sel_o].tolist(), gs_o[sel_o].tolist()))
    b = sorted(zip(keys[sel_g].tolist(), vals[sel_g].tolist()))
    assert a == b
    # no inversions against the FP64 depth order among well-separated depths
    for t in np.unique(keys):
        g = vals[keys == t]
        z = pr["z"][g]
        d = np.diff(z)
        assert (d >= -1e-6 * np.abs(z[1:])).all()
    # ranges
    rng = f.buf("ranges", torch.int32).cpu().numpy().reshape(-1, 2)
    for t in range(rng.shape[0]):
        s, e = rng[t]
        assert (keys[s:e] == t).all()
        assert e - s == (keys == t).sum()


def test_pair_list_of_large_splats(oracle):
    """Gaussians four times the usual size (about 36 tiles each), so that an
    emission block (512 items in depth order) holds more pairs than the
    emission stages in LDS and stores each pair where it goes: the pair list
    is still the stable (tile, depth bits, index) order of exactly the pairs
    of the tile rectangles, and the images match the oracle."""
    sc = scenes.single_view_scene(seed=7, n=3000)
    sc["params"][3:6] += 1.4
    r, p, ids = _frame(sc, ctx=B.Context(tile_w=8, tile_h=8))
    img = r.forward(p, ids, probs=True)
    torch.cuda.synchronize()
    f = r.frame
    rc, st, P = f.read_status()
    assert rc == 0 and st == 0
    cnt = f.buf("counts", torch.int32, 3000).cpu().numpy().astype(np.int64)
    dorder = f.buf("depth_order", torch.int32, 3000).cpu().numpy()
    per_block = [int(cnt[dorder[i:i + 512]].sum()) for i in range(0, 3000, 512)]
    assert max(per_block) > 6144, per_block  # the LDS stage holds 12 pairs per record
    keys = f.buf("pair_keys", torch.int32, P).cpu().numpy().astype(np.int64)
    vals = pair_items(f.buf("pair_vals", torch.int32, P).cpu().numpy()).astype(np.int64)
    spl = f.buf("splats", torch.float32, 3000 * B.SPLAT_WORDS).view(3000, B.SPLAT_WORDS).cpu().numpy()
    zbits = spl[:, 6].astype(np.float32).view(np.uint32).astype(np.int64)
    assert (np.lexsort((vals, zbits[vals], keys)) == np.arange(P)).all()
    rect = f.buf("rects", torch.int16, 3000 * 4).view(3000, 4).cpu().numpy().astype(np.int64)
    want = sorted((int(y * 16 + x), g) for g in range(3000) if cnt[g]
                  for y in range(rect[g, 1], rect[g, 3] + 1) for x in range(rect[g, 0], rect[g, 2] + 1))
    assert P == len(want) and sorted(zip(keys.tolist(), vals.tolist())) == want
    ref = _oracle_fwd(oracle, sc)
    ok = unambiguous(ref)
    assert ok.mean() > 0.9
    close(img["color"][0].cpu().numpy(), ref["C"], FWD_RTOL, ok, "colour")
    close(img["depth"][0].cpu().numpy(), ref["D"], FWD_RTOL, ok, "depth")
    close(img["t_final"][0].cpu().numpy(), ref["Tf"], FWD_RTOL, ok, "T_final")


def _oracle_fwd(oracle, sc, cfg=None, pix=None):
    return oracle.render(sc["params"], sc["ids"], sc["cams"][0], cfg=cfg, K=sc["K"], pix=pix)


@pytest.mark.parametrize("seed,tile", [(0, (16, 16)), (3, (16, 16)), (4, (8, 8)), (5, (16, 8)), (6, (8, 32))])
def test_render_forward_parity(oracle, seed, tile):
    sc = scenes.single_view_scene(seed=seed, n=2000)
    r, p, ids = _frame(sc, ctx=B.Context(tile_w=tile[0], tile_h=tile[1]))
    img = r.forward(p, ids, probs=True, id_map=True)
    torch.cuda.synchronize()
    ref = _oracle_fwd(oracle, sc)
    ok = unambiguous(ref)
    assert ok.mean() > 0.98
    C = img["color"][0].cpu().numpy()
    close(C, ref["C"], FWD_RTOL, ok, "colour")
    close(img["depth"][0].cpu().numpy(), ref["D"], FWD_RTOL, ok, "depth")
    close(img["t_final"][0].cpu().numpy(), ref["Tf"], FWD_RTOL, ok, "T_final")
    close(img["probs"][0].cpu().numpy(), ref["P"], FWD_RTOL, ok, "instance")
    # last blended Gaussian: exact
    vals = pair_items(r.frame.buf("pair_vals", torch.int32).cpu().numpy())
    lastpos = img["last"][0].cpu().numpy()
    lastg = np.where(lastpos >= 0, vals[np.maximum(lastpos, 0)], -1)
    assert (lastg[ok] == ref["last"][ok]).all()
    # object-id argmax: exact where the oracle's top-2 gap exceeds 1e-5
    st = np.concatenate([ref["P"], ref["Tf"][None]], 0)
    srt = np.sort(st, axis=0)
    clear = ok & (srt[-1] - srt[-2] > 1e-5)
    idm = img["id_map"][0].cpu().numpy()
    assert (idm[clear] == oracle.id_map(ref["P"], ref["Tf"])[clear]).all()


def test_forward_tile_shape_invariance_bitwise():
    sc = scenes.single_view_scene(seed=5, n=2000)
    outs = []
    for tw, th in ((16, 16), (8, 8), (16, 8), (32, 8), (8, 32)):
        ctx = B.Context(tile_w=tw, tile_h=th)
        r, p, ids = _frame(sc, ctx=ctx)
        img = r.forward(p, ids, probs=True)
        torch.cuda.synchronize()
        outs.append({k: img[k].cpu().numpy() for k in ("color", "depth", "t_final", "probs")})
    for o in outs[1:]:
        for k in o:
            assert np.array_equal(o[k], outs[0][k]), k


def _sparse_upstream(seed, ref, H, W, K, keep):
    rng = np.random.default_rng(seed)
    g = dict(gC=rng.normal(size=(3, H, W)), gD=rng.normal(size=(H, W)), gT=rng.normal(size=(H, W)),
             gP=rng.normal(size=(K, H, W)))
    for k in g:
        g[k] = g[k] * keep
    return g


@pytest.mark.parametrize("seed,tile", [(0, (16, 16)), (2, (16, 16)), (0, (8, 8)), (1, (32, 8)), (3, (16, 8)),
                                       (4, (8, 32))])
def test_render_backward_parity(oracle, seed, tile):
    sc = scenes.single_view_scene(seed=seed, n=2000)
    cam = sc["cams"][0]
    H, W, K = cam["height"], cam["width"], sc["K"]
    r, p, ids = _frame(sc, ctx=B.Context(tile_w=tile[0], tile_h=tile[1]))
    img = r.forward(p, ids, probs=True)
    ref = _oracle_fwd(oracle, sc)
    keep = unambiguous(ref, grads=True)
    up = _sparse_upstream(10 + seed, ref, H, W, K, keep)
    grads = dict(d_color=to_dev(up["gC"][None]), d_depth=to_dev(up["gD"][None]), d_t_final=to_dev(up["gT"][None]),
                 d_probs=to_dev(up["gP"][None]))
    g = r.backward(p, img, grads)
    torch.cuda.synchronize()
    go, _ = oracle.render_backward(sc["params"], sc["ids"], cam, K=K, **up)
    close(g.cpu().numpy(), go, GRAD_RTOL, what="param grads")



@pytest.mark.parametrize("probs", [True, False])
def test_backward_past_batches_that_cannot_contribute(oracle, probs):
    """A veil of faint Gaussians (opacity below alpha_min: they never blend)
    in front of an opaque background: every tile's pair range opens with more
    than 128 of them, all of which the forward marks as contributing nowhere,
    so the backward meets whole 64-pair batches (and, on the segmented path,
    whole segments) with no record to load, and walks past them.  Whole tiles
    with instance channels (probs) and the segmented path without them,
    against the oracle's adjoint."""
    rng = np.random.default_rng(5)
    nb, nf = 80, 400
    mu = np.concatenate([np.stack([rng.uniform(-1.6, 1.6, nb), rng.uniform(-1.6, 1.6, nb), rng.uniform(3.8, 4.2, nb)]),
                         np.stack([rng.uniform(-0.9, 0.9, nf), rng.uniform(-0.9, 0.9, nf), rng.uniform(1.9, 2.1, nf)])],
                        axis=1)
    ls = np.concatenate([rng.normal(-1.8, 0.2, (3, nb)), rng.normal(-1.5, 0.1, (3, nf))], axis=1)
    q = rng.normal(size=(4, nb + nf))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    eta = np.concatenate([rng.normal(1.0, 0.5, nb), np.full(nf, -9.0)])
    rgb = rng.uniform(0, 1, (3, nb + nf))
    ids = rng.integers(0, 3, nb + nf).astype(np.int32)
    cam = scenes.camera(fx=40.0, fy=40.0, cx=16.0, cy=16.0, width=32, height=32)
    sc = dict(params=scenes.pack(mu, ls, q, eta, rgb), ids=ids, cams=[cam], K=3)
    H, W, K = 32, 32, 3
    r, p, ids_d = _frame(sc, ctx=B.Context(tile_w=8, tile_h=8))
    img = r.forward(p, ids_d, probs=probs)
    ref = _oracle_fwd(oracle, sc)
    keep = unambiguous(ref, grads=True)
    up = _sparse_upstream(77, ref, H, W, K, keep)
    grads = dict(d_color=to_dev(up["gC"][None]), d_depth=to_dev(up["gD"][None]), d_t_final=to_dev(up["gT"][None]))
    if probs:
        grads["d_probs"] = to_dev(up["gP"][None])
    else:
        up["gP"] = None
    g = r.backward(p, img, grads)
    torch.cuda.synchronize()
    # the case arises: tiles whose range opens with >= 128 faint pairs while
    # some pixel blends a background Gaussian behind them
    rng_t = r.frame.buf("ranges", torch.int32).cpu().numpy().reshape(-1, 2)
    rc, st, P = r.frame.read_status()
    assert rc == 0
    raw = r.frame.buf("pair_vals", torch.int32, P).cpu().numpy()
    vals = pair_items(raw)
    # the forward marked every faint pair (the backward skips them unloaded)
    assert (raw[vals >= nb] < 0).all()
    last = img["last"][0].cpu().numpy().reshape(H // 8, 8, W // 8, 8).transpose(0, 2, 1, 3).reshape(-1, 64)
    lead = np.array([np.argmax(np.append(vals[s:e], 0) < nb) for s, e in rng_t])
    assert ((lead >= 128) & (last.max(1) >= rng_t[:, 0] + lead)).sum() >= 4
    go, _ = oracle.render_backward(sc["params"], sc["ids"], cam, K=K, **up)
    assert np.abs(go[:, nb:]).max() == 0.0
    close(g.cpu().numpy(), go, GRAD_RTOL, what="param grads")


def test_reproducible_bitwise():
    sc = scenes.single_view_scene(seed=7, n=2000)
    res = []
    for _ in range(2):
        r, p, ids = _frame(sc)
        img = r.forward(p, ids, probs=True)
        up = scenes.random_image_grads(3, (3, 96, 128), K=3)
        grads = dict(d_color=to_dev(up["gC"][None]), d_depth=to_dev(up["gD"][None]),
                     d_t_final=to_dev(up["gT"][None]), d_probs=to_dev(up["gP"][None]))
        g = r.backward(p, img, grads)
        torch.cuda.synchronize()
        res.append((img["color"].cpu().numpy(), g.cpu().numpy()))
    assert np.array_equal(res[0][0], res[1][0])
    assert np.array_equal(res[0][1], res[1][1])


def test_object_loss_parity(oracle):
    rng = np.random.default_rng(4)
    V, H, W = 2, 37, 53
    C, tC = rng.uniform(size=(V, 3, H, W)), rng.uniform(size=(V, 3, H, W))
    D, tD = rng.uniform(1, 3, size=(V, H, W)), rng.uniform(-1, 3, size=(V, H, W))
    pt = rng.uniform(0, 1, size=(V, H, W))
    pt[0, 0, :5] = 1e-8
    tid = rng.integers(-1, 3, size=(V, H, W)).astype(np.int32)
    cams = [scenes.camera(width=W, height=H)] * V
    f = B.Frame(B.Context(), cams, 10, 3, 100)
    img = dict(color=to_dev(C), depth=to_dev(D), p_target=to_dev(pt), t_final=to_dev(D), last=None,
               target=torch.tensor(tid, device="cuda"))
    grads = dict(d_color=torch.empty(V, 3, H, W, device="cuda"), d_depth=torch.empty(V, H, W, device="cuda"),
                 d_p_target=torch.empty(V, H, W, device="cuda"))
    loss = torch.zeros(4, dtype=torch.float64, device="cuda")
    f.object_loss(img, dict(color=to_dev(tC), depth=to_dev(tD), id=img["target"]), grads, loss, 0.8, 1.2, 0.5)
    torch.cuda.synchronize()
    ref = oracle.object_loss(C.astype(np.float32), D.astype(np.float32), pt.astype(np.float32),
                             tC.astype(np.float32), tD.astype(np.float32), tid, 0.8, 1.2, 0.5)
    lv = loss.cpu().numpy()
    np.testing.assert_allclose(lv, [ref["loss"], ref["l_rgb"], ref["l_depth"], ref["l_obj"]], rtol=1e-6)
    close(grads["d_color"].cpu().numpy(), ref["gC"], 1e-5, what="dL/dC")
    close(grads["d_depth"].cpu().numpy(), ref["gD"], 1e-5, what="dL/dD")
    close(grads["d_p_target"].cpu().numpy(), ref["gp"], 1e-5, what="dL/dp")
    # bitwise reproducible
    loss2 = torch.zeros(4, dtype=torch.float64, device="cuda")
    f.object_loss(img, dict(color=to_dev(tC), depth=to_dev(tD), id=img["target"]), None, loss2, 0.8, 1.2, 0.5)
    assert torch.equal(loss, loss2)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_adam_parity(oracle, dtype):
    rng = np.random.default_rng(8)
    for n in (1000, 1001):
        p0 = rng.normal(size=(14, n))
        lrs = B.default_lrs(3.0)
        p, m, v = to_dev(p0, dtype), torch.zeros(14, n, dtype=dtype, device="cuda"), \
            torch.zeros(14, n, dtype=dtype, device="cuda")
        po, mo, vo = p0.copy(), np.zeros_like(p0), np.zeros_like(p0)
        ctx = B.Context()
        for step in range(1, 4):
            g = rng.normal(size=(14, n))
            B.adam_step(ctx, p, to_dev(g, dtype), m, v, lrs, step)
            po, mo, vo = oracle.adam(po, g, mo, vo, step, lrs)
        torch.cuda.synchronize()
        tol = 1e-6 if dtype == torch.float32 else 1e-12
        np.testing.assert_allclose(p.cpu().numpy(), po, rtol=tol, atol=tol)
        np.testing.assert_allclose(m.cpu().numpy(), mo, rtol=1e-5 if dtype == torch.float32 else 1e-12, atol=1e-7)


def test_end_to_end_step_gradient(oracle):
    """forward + object loss + backward on the GPU against the oracle's own
    forward + loss + adjoint on the same scene and targets."""
    sc = scenes.single_view_scene(seed=0, n=2000)
    cam = sc["cams"][0]
    tg = oracle.render(scenes.perturb(sc["params"], 1), sc["ids"], cam, K=3)
    t_id = oracle.id_map(tg["P"], tg["Tf"])
    # Shifted targets keep every L1 residual away from the kink of |x| (so the
    # sign, a discrete decision, is the same in FP32 and FP64); a band of pixels
    # carries no valid target depth.
    tg["C"] = tg["C"] + 2.0
    tg["D"] = tg["D"] + 10.0
    tg["D"][40:50, :] = 0.0
    ref = oracle.render(sc["params"], sc["ids"], cam, K=3)
    p_t = np.where(t_id >= 0, np.take_along_axis(ref["P"], np.maximum(t_id, 0)[None], 0)[0], ref["Tf"])
    lo = oracle.object_loss(ref["C"], ref["D"], p_t, tg["C"], tg["D"], t_id)
    # Pixels where a discrete decision of the forward is within the band get zero
    # upstream gradient on both sides (the loss value still covers every pixel).
    keep = unambiguous(ref, grads=True)
    assert keep.mean() > 0.97
    # oracle adjoint of the loss: gP only at the target channel, gT where target = none
    gp = lo["gp"] * keep
    gP = np.zeros((3,) + t_id.shape)
    for k in range(3):
        gP[k] = np.where(t_id == k, gp, 0.0)
    gT = np.where(t_id == -1, gp, 0.0)
    go, _ = oracle.render_backward(sc["params"], sc["ids"], cam, K=3, gC=lo["gC"] * keep, gD=lo["gD"] * keep,
                                   gP=gP, gT=gT)
    r, p, ids = _frame(sc)
    target = torch.tensor(t_id[None], dtype=torch.int32, device="cuda")
    img = r.forward(p, ids, target=target)
    grads = dict(d_color=torch.empty_like(img["color"]), d_depth=torch.empty_like(img["depth"]),
                 d_p_target=torch.empty_like(img["depth"]))
    loss = torch.zeros(4, dtype=torch.float64, device="cuda")
    r.frame.object_loss(img, dict(color=to_dev(tg["C"][None]), depth=to_dev(tg["D"][None]), id=target), grads, loss)
    torch.cuda.synchronize()
    np.testing.assert_allclose(loss.cpu().numpy(), [lo["loss"], lo["l_rgb"], lo["l_depth"], lo["l_obj"]], rtol=1e-4)
    close(grads["d_color"][0].cpu().numpy(), lo["gC"], FWD_RTOL, keep, "dL/dC")
    close(grads["d_depth"][0].cpu().numpy(), lo["gD"], FWD_RTOL, keep, "dL/dD")
    close(grads["d_p_target"][0].cpu().numpy(), lo["gp"], FWD_RTOL, keep, "dL/dp_t")
    m = torch.tensor(keep[None], dtype=torch.float32, device="cuda")
    grads = dict(d_color=(grads["d_color"] * m[:, None]).contiguous(), d_depth=(grads["d_depth"] * m).contiguous(),
                 d_p_target=(grads["d_p_target"] * m).contiguous())
    g = r.backward(p, img, grads)
    torch.cuda.synchronize()
    close(g.cpu().numpy(), go, GRAD_RTOL, what="end-to-end grads")


def test_quadric_fit_parity(oracle):
    from scipy.spatial.transform import Rotation
    rng = np.random.default_rng(11)
    cams = scenes.ring_cameras(8, radius=2.5)
    Ps = np.stack([oracle.camera_matrix(c) for c in cams])
    boxes, bo, bv, objs = [], [], [], []
    for k in range(40):
        mu = rng.uniform(-0.5, 0.5, 3)
        R = Rotation.random(random_state=int(rng.integers(1 << 30))).as_matrix()
        ax = rng.uniform(0.1, 0.4, 3)
        objs.append((mu, R, ax))
        Q = oracle.dual_quadric_from_ellipsoid(mu, R, ax)
        views = range(8) if k != 39 else range(2)   # the last object is seen twice only
        for v in views:
            boxes.append(oracle.conic_box(oracle.project_dual_quadric(Q, Ps[v])))
            bo.append(k)
            bv.append(v)
    boxes, bo, bv = np.array(boxes), np.array(bo, np.int32), np.array(bv, np.int32)
    ref = oracle.fit_dual_quadric(boxes, bo, bv, Ps, 41)
    out = B.fit_dual_quadric(B.Context(), to_dev(boxes, torch.float64), torch.tensor(bo, device="cuda"),
                             torch.tensor(bv, device="cuda"), to_dev(Ps.reshape(8, 12), torch.float64), 41)
    torch.cuda.synchronize()
    st = out["status"].cpu().numpy()
    assert (st == ref["status"]).all()
    assert st[39] == oracle.QUADRIC_DEGENERATE and st[40] == oracle.QUADRIC_DEGENERATE
    Qg = out["Q"].cpu().numpy()
    for k in range(39):
        np.testing.assert_allclose(Qg[k], ref["Q"][k], atol=1e-9 * np.abs(ref["Q"][k]).max())
        np.testing.assert_allclose(out["mu"].cpu().numpy()[k], objs[k][0], atol=1e-8)
        np.testing.assert_allclose(out["axes"].cpu().numpy()[k], np.sort(objs[k][2]), rtol=1e-7)
        Rg = out["R"].cpu().numpy()[k]
        M = Rg @ np.diag(out["axes"].cpu().numpy()[k] ** 2) @ Rg.T
        R0 = objs[k][1]
        np.testing.assert_allclose(M, R0 @ np.diag(objs[k][2] ** 2) @ R0.T, atol=1e-9)
        assert abs(np.linalg.det(Rg) - 1) < 1e-9


def test_jacobian_frustum_limit_parity(oracle):
    """A narrow field of view (f = 300 on 128x96): most Gaussians sit beyond
    1.3x the half field of view, and a quarter of them are large enough to
    reach into the image, so the clamped Jacobian and its adjoint are used."""
    sc = scenes.single_view_scene(seed=9, n=2000)
    sc["params"][3:6, ::4] += 1.5
    cam = scenes.camera(fx=300, fy=300, cx=64, cy=48, width=128, height=96)
    sc["cams"] = [cam]
    p0 = sc["params"]
    u, v = p0[0] / p0[2], p0[1] / p0[2]
    clamped = (np.abs(u) > 1.3 * 64 / 300) | (np.abs(v) > 1.3 * 48 / 300)
    assert clamped.mean() > 0.3
    H, W, K = cam["height"], cam["width"], sc["K"]
    r, p, ids = _frame(sc, ctx=B.Context(tile_w=16, tile_h=16))
    img = r.forward(p, ids, probs=True)
    torch.cuda.synchronize()
    pr = oracle.project(p0, cam)
    spl = r.frame.buf("splats", torch.float32, 2000 * B.SPLAT_WORDS).view(2000, B.SPLAT_WORDS).cpu().numpy()
    vis = pr["visible"] & clamped
    for k, name in ((2, "A"), (3, "B"), (4, "C")):
        close(spl[vis, k], pr[name][vis], FWD_RTOL, what=name)
    ref = _oracle_fwd(oracle, sc)
    ok = unambiguous(ref)
    assert ok.mean() > 0.95
    close(img["color"][0].cpu().numpy(), ref["C"], FWD_RTOL, ok, "colour")
    close(img["depth"][0].cpu().numpy(), ref["D"], FWD_RTOL, ok, "depth")
    keep = unambiguous(ref, grads=True)
    up = _sparse_upstream(31, ref, H, W, K, keep)
    grads = dict(d_color=to_dev(up["gC"][None]), d_depth=to_dev(up["gD"][None]), d_t_final=to_dev(up["gT"][None]),
                 d_probs=to_dev(up["gP"][None]))
    g = r.backward(p, img, grads)
    torch.cuda.synchronize()
    go, _ = oracle.render_backward(p0, sc["ids"], cam, K=K, **up)
    # the clamped Gaussians receive gradient, and it matches
    assert np.abs(go[:6][:, clamped]).max() > 0
    close(g.cpu().numpy(), go, GRAD_RTOL, what="param grads")


def test_dense_view_loss_mode_parity(oracle):
    """Dense view (30k Gaussians on 128x96, 8x8 tiles; many tiles hold more
    than 256 pairs): the loss-mode forward (no instance channels) and its
    backward against the oracle, and bitwise run-to-run reproducibility."""
    sc = scenes.single_view_scene(seed=12, n=30000)
    cam = sc["cams"][0]
    H, W, K = cam["height"], cam["width"], sc["K"]
    ref = _oracle_fwd(oracle, sc)
    keep = unambiguous(ref, grads=True)
    up = _sparse_upstream(40, ref, H, W, K, keep)
    go, _ = oracle.render_backward(sc["params"], sc["ids"], cam, K=K, gC=up["gC"], gD=up["gD"], gT=up["gT"],
                                   gP=np.zeros_like(up["gP"]))
    ok = unambiguous(ref)
    assert ok.mean() > 0.9
    runs = []
    for _ in range(2):
        r, p, ids = _frame(sc, ctx=B.Context(tile_w=8, tile_h=8))
        img = r.forward(p, ids)
        grads = dict(d_color=to_dev(up["gC"][None]), d_depth=to_dev(up["gD"][None]),
                     d_t_final=to_dev(up["gT"][None]))
        g = r.backward(p, img, grads)
        torch.cuda.synchronize()
        runs.append((img, g.cpu().numpy(), r))
    img, g, r = runs[0]
    rng = r.frame.buf("ranges", torch.int32).cpu().numpy().reshape(-1, 2)
    assert (rng[:, 1] - rng[:, 0]).max() > 256
    close(img["color"][0].cpu().numpy(), ref["C"], FWD_RTOL, ok, "colour")
    close(img["depth"][0].cpu().numpy(), ref["D"], FWD_RTOL, ok, "depth")
    close(img["t_final"][0].cpu().numpy(), ref["Tf"], FWD_RTOL, ok, "T_final")
    vals = pair_items(r.frame.buf("pair_vals", torch.int32).cpu().numpy())
    lastpos = img["last"][0].cpu().numpy()
    lastg = np.where(lastpos >= 0, vals[np.maximum(lastpos, 0)], -1)
    assert (lastg[ok] == ref["last"][ok]).all()
    close(g, go, GRAD_RTOL, what="param grads (dense view)")
    img2, g2 = runs[1][0], runs[1][1]
    assert torch.equal(img["color"], img2["color"]) and torch.equal(img["last"], img2["last"])
    assert np.array_equal(g, g2)


def test_segmented_backward_with_target_parity(oracle):
    """Dense view with 8x8 tiles (tile ranges of several 64-pair segments):
    the backward runs one wavefront per segment, each restarted from the
    forward's stored state at the segment's end.  Upstream gradients on colour,
    depth and the target-object probability (through the target channel, or
    the background transmittance where the target is none) against the
    oracle's adjoint; some pixels blend past the first boundary of their tile."""
    sc = scenes.single_view_scene(seed=12, n=30000)
    cam = sc["cams"][0]
    H, W, K = cam["height"], cam["width"], sc["K"]
    tg = oracle.render(scenes.perturb(sc["params"], 1), sc["ids"], cam, K=K)
    t_id = oracle.id_map(tg["P"], tg["Tf"])
    ref = _oracle_fwd(oracle, sc)
    keep = unambiguous(ref, grads=True)
    rng = np.random.default_rng(41)
    gC = rng.normal(size=(3, H, W)) * keep
    gD = rng.normal(size=(H, W)) * keep
    gpt = rng.normal(size=(H, W)) * keep
    gP = np.zeros((K, H, W))
    for k in range(K):
        gP[k] = np.where(t_id == k, gpt, 0.0)
    gT = np.where(t_id == -1, gpt, 0.0)
    go, _ = oracle.render_backward(sc["params"], sc["ids"], cam, K=K, gC=gC, gD=gD, gP=gP, gT=gT)
    r, p, ids = _frame(sc, ctx=B.Context(tile_w=8, tile_h=8))
    target = torch.tensor(t_id[None], dtype=torch.int32, device="cuda")
    img = r.forward(p, ids, target=target)
    grads = dict(d_color=to_dev(gC[None]), d_depth=to_dev(gD[None]), d_p_target=to_dev(gpt[None]))
    g = r.backward(p, img, grads)
    torch.cuda.synchronize()
    rng_t = r.frame.buf("ranges", torch.int32).cpu().numpy().reshape(-1, 2)
    lastpos = img["last"][0].cpu().numpy()
    ys, xs = np.mgrid[0:H, 0:W]
    tile = (ys // 8) * ((W + 7) // 8) + xs // 8
    rel = lastpos - rng_t[tile, 0]
    assert ((rel >= 128) & keep).sum() > 100 and ((rel >= 256) & keep).any()
    close(g.cpu().numpy(), go, GRAD_RTOL, what="param grads (segmented, target channel)")
