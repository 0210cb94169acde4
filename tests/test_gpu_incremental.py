"""GPU parity of the incremental update (Eq. (7)-(8)): the unstable-pixel
masks and per-object counts, and the Gaussians back-projected at them,
through the C ABI against the FP64 oracle on the same seeded inputs.

Masks are integer decisions: on images quantised to a 1/64 grid (every test
value exactly representable, none within 1% of theta_d or theta_c, and
probabilities that hit theta_alpha exactly) they must agree bit for bit; on
rendered images they agree outside the oracle's near-threshold margin.
Densification is compared with masks fed to both sides: ids and counts
exactly, the Gaussian parameters to 1e-5 (FP32) / 1e-12 (FP64) relative."""
import numpy as np
import pytest
import torch

from oracle import incremental as OI
from paper_2503_02223_amd import binding as B
from paper_2503_02223_amd import scenes
from tests.gpu_util import to_dev, unambiguous

pytestmark = pytest.mark.gpu


def _quantised_views(rng, V, H, W, K):
    """Rendered and observed images on the 1/64 grid with every test firing."""
    q = lambda a: np.round(a * 64) / 64
    C = q(rng.uniform(0, 1, (V, 3, H, W)))
    tc = np.clip(C + q(rng.choice([-0.25, -0.1, 0, 0.05, 0.1, 0.3], (V, 3, H, W))), 0, 1)
    D = q(rng.uniform(0.5, 4.0, (V, H, W)))
    td = D + q(rng.choice([-0.5, -0.125, -0.0625, 0.0, 0.0625, 0.125, 0.5], (V, H, W)))
    td[rng.uniform(size=(V, H, W)) < 0.1] = 0.0                     # no observed depth
    pt = q(rng.choice([0.0, 0.25, 0.5, 0.75, 1.0], (V, H, W)))       # 0.5 = theta_alpha exactly: not below
    tid = rng.integers(-1, K + 1, (V, H, W)).astype(np.int32)        # -1 (no object) and K (out of range)
    return C, D, pt, tc, td, tid


def _oracle_masks(C, D, pt, tc, td, tid, K):
    """Oracle masks per view; P holds ins of the observed object in its channel."""
    V = C.shape[0]
    out, cnt = [], np.zeros((K, 2), np.int64)
    for v in range(V):
        P = np.zeros((K,) + D.shape[1:])
        t = tid[v]
        for k in range(K):
            P[k][t == k] = pt[v][t == k]
        m, c, _ = OI.masks(C[v], D[v], P, tc[v], td[v], t)
        out.append(m)
        cnt += c
    return np.stack(out), cnt


def _run_masks(cams, K, C, D, pt, tc, td, tid, dtype):
    V, H, W = D.shape
    f = B.Frame(B.Context(), cams, 0, K, 0, dtype=dtype)
    img = dict(color=to_dev(C, dtype), depth=to_dev(D, dtype), p_target=to_dev(pt, dtype),
               target=torch.tensor(tid, device="cuda"))
    tgt = dict(color=to_dev(tc, dtype), depth=to_dev(td, dtype), id=img["target"])
    masks = torch.full((V, H, W), 0xAB, dtype=torch.uint8, device="cuda")
    counts = torch.full((K, 2), -7, dtype=torch.int32, device="cuda")
    f.incremental_masks(img, tgt, masks, counts)
    torch.cuda.synchronize()
    return masks.cpu().numpy(), counts.cpu().numpy()


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("shape", [(1, 29, 37, 3), (3, 64, 80, 5)])
def test_masks_exact_on_quantised_images(shape, dtype):
    V, H, W, K = shape
    rng = np.random.default_rng(11 + V)
    imgs = _quantised_views(rng, V, H, W, K)
    cams = scenes.ring_cameras(V, width=W, height=H)
    m, c = _run_masks(cams, K, *imgs, dtype)
    m_o, c_o = _oracle_masks(*imgs, K)
    np.testing.assert_array_equal(m, m_o)
    np.testing.assert_array_equal(c, c_o)
    assert (m == 1).any() and (m == 2).any() and (m == 3).any() and (m == 0).any()


def test_masks_full_frame_640x480():
    """Full frame, four views: exact against the oracle, counts summing to the masks."""
    V, H, W, K = 4, 480, 640, 8
    rng = np.random.default_rng(5)
    imgs = _quantised_views(rng, V, H, W, K)
    cams = scenes.ring_cameras(V, width=W, height=H)
    m, c = _run_masks(cams, K, *imgs, torch.float32)
    m_o, c_o = _oracle_masks(*imgs, K)
    np.testing.assert_array_equal(m, m_o)
    np.testing.assert_array_equal(c, c_o)


def test_masks_on_a_loss_mode_render(oracle):
    """Masks from the library's own loss-mode forward against the oracle's
    masks of the oracle's render, outside near-threshold and ambiguous pixels."""
    sc = scenes.single_view_scene(seed=4, n=2000)
    cam, K = sc["cams"][0], sc["K"]
    tg = oracle.render(scenes.perturb(sc["params"], 2), sc["ids"], cam, K=K)
    tid = oracle.id_map(tg["P"], tg["Tf"]).astype(np.int32)
    ref = oracle.render(sc["params"], sc["ids"], cam, K=K)
    m_o, c_o, margin = OI.masks(ref["C"], ref["D"], ref["P"], tg["C"], tg["D"], tid)
    r = B.Rasterizer(sc["cams"], sc["params"].shape[1], K)
    p = to_dev(sc["params"])
    ids = torch.tensor(sc["ids"], device="cuda")
    target = torch.tensor(tid[None], device="cuda")
    img = r.forward(p, ids, target=target)
    tgt = dict(color=to_dev(tg["C"][None]), depth=to_dev(tg["D"][None]), id=target)
    masks = torch.empty((1, cam["height"], cam["width"]), dtype=torch.uint8, device="cuda")
    counts = torch.empty((K, 2), dtype=torch.int32, device="cuda")
    r.frame.incremental_masks(img, tgt, masks, counts)
    torch.cuda.synchronize()
    m = masks[0].cpu().numpy()
    ok = unambiguous(ref) & (margin > 1e-3)
    assert ok.mean() > 0.9
    np.testing.assert_array_equal(m[ok], m_o[ok])
    assert (m_o > 0).sum() > 100
    # the counts are those of the library's own masks, and agree with the oracle's up to the excluded pixels
    c = counts.cpu().numpy()
    for k in range(K):
        sel = tid == k
        assert c[k, 0] == ((m & 1) > 0)[sel].sum() and c[k, 1] == ((m & 2) > 0)[sel].sum()
    assert np.abs(c - c_o).sum() <= (~ok).sum()


def _dens_inputs(rng, V, H, W):
    masks = rng.integers(0, 4, (V, H, W)).astype(np.uint8)
    masks[rng.uniform(size=masks.shape) < 0.5] = 0
    tc = rng.uniform(0, 1, (V, 3, H, W))
    td = rng.uniform(0.4, 5.0, (V, H, W))
    td[rng.uniform(size=td.shape) < 0.15] = 0.0
    tid = rng.integers(-1, 6, (V, H, W)).astype(np.int32)
    return masks, tc, td, tid


def _oracle_densify(masks, tc, td, tid, cams):
    ps, ids, per_view = [], [], []
    for v in range(masks.shape[0]):
        p, i = OI.densify(masks[v], tc[v], td[v], tid[v], cams[v])
        ps.append(p)
        ids.append(i)
        per_view.append(p.shape[1])
    return np.concatenate(ps, 1), np.concatenate(ids), per_view


def _run_densify(cams, masks, tc, td, tid, n_old, n_cap, dtype, old=None):
    V = masks.shape[0]
    f = B.Frame(B.Context(), cams, 0, 1, 0, dtype=dtype)
    params = torch.full((B.NUM_PARAMS, n_cap), 123.0, dtype=dtype, device="cuda")
    ids = torch.full((n_cap,), -99, dtype=torch.int32, device="cuda")
    if old is not None:
        params[:, :n_old] = to_dev(old, dtype)
    counts = torch.full((V + 1,), -1, dtype=torch.int64, device="cuda")
    tgt = dict(color=to_dev(tc, dtype), depth=to_dev(td, dtype), id=torch.tensor(tid, device="cuda"))
    f.densify(tgt, torch.tensor(masks, device="cuda"), params, ids, n_old, counts)
    torch.cuda.synchronize()
    return params.cpu().numpy().astype(np.float64), ids.cpu().numpy(), counts.cpu().numpy()


def _check_params(got, want, dtype):
    rtol = 1e-5 if dtype == torch.float32 else 1e-12
    scale = np.maximum(np.abs(want), 1.0)
    err = (np.abs(got - want) / scale).max() if want.size else 0.0
    assert err < rtol, f"densify parameters off by {err:.3e}"


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_densify_matches_oracle(dtype):
    V, H, W = 3, 45, 61
    rng = np.random.default_rng(8)
    masks, tc, td, tid = _dens_inputs(rng, V, H, W)
    cams = scenes.ring_cameras(V, width=W, height=H)
    # the densifier takes the observed inputs at the frame's precision; the oracle gets the same values
    tc = tc.astype(np.float32).astype(np.float64) if dtype == torch.float32 else tc
    td = td.astype(np.float32).astype(np.float64) if dtype == torch.float32 else td
    p_o, id_o, per_view = _oracle_densify(masks, tc, td, tid, cams)
    n_new = p_o.shape[1]
    n_old = 17
    old = rng.normal(size=(B.NUM_PARAMS, n_old))
    p, ids, counts = _run_densify(cams, masks, tc, td, tid, n_old, n_old + n_new + 5, dtype, old=old)
    assert counts[0] == n_new and list(counts[1:]) == per_view
    np.testing.assert_array_equal(ids[n_old:n_old + n_new], id_o)
    _check_params(p[:, n_old:n_old + n_new], p_o, dtype)
    # columns below n_old and beyond the new ones are left as they were
    want_old = old.astype(np.float32).astype(np.float64) if dtype == torch.float32 else old
    np.testing.assert_array_equal(p[:, :n_old], want_old)
    assert (p[:, n_old + n_new:] == 123.0).all() and (ids[n_old + n_new:] == -99).all()


def test_densify_capacity_and_empty():
    V, H, W = 2, 33, 40
    rng = np.random.default_rng(9)
    masks, tc, td, tid = _dens_inputs(rng, V, H, W)
    cams = scenes.ring_cameras(V, width=W, height=H)
    tc, td = tc.astype(np.float32).astype(np.float64), td.astype(np.float32).astype(np.float64)
    p_o, id_o, per_view = _oracle_densify(masks, tc, td, tid, cams)
    n_new = p_o.shape[1]
    # capacity for only part of them: the total is still reported, nothing is written past n_cap
    cap = n_new // 3
    p, ids, counts = _run_densify(cams, masks, tc, td, tid, 0, cap, torch.float32)
    assert counts[0] == n_new and list(counts[1:]) == per_view
    np.testing.assert_array_equal(ids, id_o[:cap])
    _check_params(p, p_o[:, :cap], torch.float32)
    # no mask set: nothing added
    z = np.zeros_like(masks)
    p, ids, counts = _run_densify(cams, z, tc, td, tid, 4, 10, torch.float32)
    assert (counts == 0).all() and (ids == -99).all()


def test_incremental_step_round_trip(oracle):
    """Loss-mode render -> masks -> densify on the device; every added
    Gaussian projects onto the centre of its own unstable pixel at the
    observed depth (a property that holds at any size)."""
    sc = scenes.single_view_scene(seed=6, n=3000)
    cam, K = sc["cams"][0], sc["K"]
    tg = oracle.render(scenes.perturb(sc["params"], 3), sc["ids"], cam, K=K)
    tid = oracle.id_map(tg["P"], tg["Tf"]).astype(np.int32)
    n = sc["params"].shape[1]
    r = B.Rasterizer(sc["cams"], n, K)
    p = to_dev(sc["params"])
    target = torch.tensor(tid[None], device="cuda")
    img = r.forward(p, torch.tensor(sc["ids"], device="cuda"), target=target)
    tgt = dict(color=to_dev(tg["C"][None]), depth=to_dev(tg["D"][None]), id=target)
    H, W = cam["height"], cam["width"]
    masks = torch.empty((1, H, W), dtype=torch.uint8, device="cuda")
    counts_obj = torch.empty((K, 2), dtype=torch.int32, device="cuda")
    r.frame.incremental_masks(img, tgt, masks, counts_obj)
    cap = n + H * W
    grown = torch.zeros((B.NUM_PARAMS, cap), device="cuda")
    grown[:, :n] = p
    ids = torch.full((cap,), -1, dtype=torch.int32, device="cuda")
    counts = torch.empty(2, dtype=torch.int64, device="cuda")
    r.frame.densify(tgt, masks, grown, ids, n, counts)
    torch.cuda.synchronize()
    m = masks[0].cpu().numpy()
    a = int(counts[0])
    assert a == ((m > 0) & (tg["D"].astype(np.float32) > 0)).sum() and a > 0
    new = grown[:, n:n + a].double().cpu().numpy()
    R, t = np.asarray(cam["R"]), np.asarray(cam["t"])
    xc = R @ new[0:3] + t[:, None]
    vs, us = np.nonzero((m > 0) & (tg["D"].astype(np.float32) > 0))
    np.testing.assert_allclose(cam["fx"] * xc[0] / xc[2] + cam["cx"], us + 0.5, atol=2e-3)
    np.testing.assert_allclose(cam["fy"] * xc[1] / xc[2] + cam["cy"], vs + 0.5, atol=2e-3)
    np.testing.assert_allclose(xc[2], tg["D"][vs, us], rtol=1e-5)
    np.testing.assert_array_equal(ids[n:n + a].cpu().numpy(), tid[vs, us])
    og = (m[vs, us] & 1) > 0
    op = 1 / (1 + np.exp(-new[10]))
    np.testing.assert_allclose(op, np.where(og, 0.9, 0.1), rtol=1e-5)
