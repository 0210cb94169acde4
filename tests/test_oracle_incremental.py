"""Pins for the incremental-update oracle: hand-made images with known mask
membership for every criterion of Eq. (7), the per-object restriction of
Eq. (8), and back-projection of the spawned Gaussians onto their pixel
centres with one-pixel footprints and the OG / TG opacities."""
import numpy as np
import pytest

from oracle import incremental as OI
from paper_2503_02223_amd import scenes


def _frame():
    H, W, K = 4, 5, 3
    C = np.full((3, H, W), 0.5)
    D = np.full((H, W), 2.0)
    P = np.zeros((K, H, W))
    P[1] = 0.9
    tc = np.full((3, H, W), 0.5)
    td = np.full((H, W), 2.0)
    tid = np.ones((H, W), np.int32)
    return C, D, P, tc, td, tid


def test_each_criterion_alone():
    C, D, P, tc, td, tid = _frame()
    P[1, 0, 0] = 0.3                 # ins below theta_alpha -> geo
    D[0, 1] = 2.25                   # depth off by 0.25 > 0.1 -> geo
    D[0, 2] = 2.05                   # off by 0.05 -> nothing
    td[0, 3] = 0.0                   # no observed depth: the depth test does not apply
    D[0, 3] = 5.0
    C[:, 1, 0] = [0.9, 0.5, 0.5]     # mean colour error 0.4 / 3 = 0.133 > 0.1 -> rgb
    C[:, 1, 1] = [0.7, 0.5, 0.5]     # 0.2 / 3 = 0.067 -> nothing
    tid[2, 0] = -1                   # observed as no object: in no mask
    P[1, 2, 0] = 0.0
    tid[2, 1] = 2                    # observed as object 2, rendered P_2 = 0 -> geo for object 2
    m, counts, _ = OI.masks(C, D, P, tc, td, tid)
    assert m[0, 0] == OI.GEO and m[0, 1] == OI.GEO and m[0, 2] == 0 and m[0, 3] == 0
    assert m[1, 0] == OI.RGB and m[1, 1] == 0
    assert m[2, 0] == 0 and m[2, 1] == OI.GEO
    assert (m == OI.GEO).sum() == 3 and (m == OI.RGB).sum() == 1 and (m == OI.GEO | OI.RGB).sum() == 0
    np.testing.assert_array_equal(counts, [[0, 0], [2, 1], [1, 0]])


def test_masks_on_a_render_match_direct_definition(oracle):
    sc = scenes.tiny_scene(seed=3, n=40, width=24, height=20, f=30.0)
    cam = sc["cams"][0]
    r = oracle.render(sc["params"], sc["ids"], cam, K=sc["K"])
    tg = oracle.render(scenes.perturb(sc["params"], 4), sc["ids"], cam, K=sc["K"])
    tid = oracle.id_map(tg["P"], tg["Tf"])
    m, counts, margin = OI.masks(r["C"], r["D"], r["P"], tg["C"], tg["D"], tid)
    for v in range(cam["height"]):
        for u in range(cam["width"]):
            t = tid[v, u]
            if t < 0:
                assert m[v, u] == 0
                continue
            geo = r["P"][t, v, u] < 0.5 or (tg["D"][v, u] > 0 and abs(r["D"][v, u] - tg["D"][v, u]) > 0.1)
            rgb = np.abs(r["C"][:, v, u] - tg["C"][:, v, u]).mean() > 0.1
            assert m[v, u] == geo * 1 + rgb * 2
    assert counts.sum() == (m & 1).astype(bool).sum() + ((m & 2) > 0).sum()
    assert np.isfinite(margin).any()


def test_densify_back_projects_with_og_and_tg():
    H, W = 6, 7
    rng = np.random.default_rng(0)
    cam = scenes.camera(fx=50.0, fy=45.0, cx=3.3, cy=2.9, width=W, height=H)
    a = 0.4
    cam["R"] = np.array([[1, 0, 0], [0, np.cos(a), -np.sin(a)], [0, np.sin(a), np.cos(a)]])
    cam["t"] = np.array([0.2, -0.1, 0.5])
    m = rng.integers(0, 4, size=(H, W)).astype(np.uint8)
    td = rng.uniform(0.5, 3.0, size=(H, W))
    td[0, :3] = 0.0
    tc = rng.uniform(0, 1, size=(3, H, W))
    tid = rng.integers(0, 5, size=(H, W)).astype(np.int32)
    p, ids = OI.densify(m, tc, td, tid, cam)
    sel = (m > 0) & (td > 0)
    vs, us = np.nonzero(sel)
    assert p.shape[1] == sel.sum() and (ids == tid[vs, us]).all()
    xc = cam["R"] @ p[0:3] + cam["t"][:, None]
    np.testing.assert_allclose(cam["fx"] * xc[0] / xc[2] + cam["cx"], us + 0.5, atol=1e-9)
    np.testing.assert_allclose(cam["fy"] * xc[1] / xc[2] + cam["cy"], vs + 0.5, atol=1e-9)
    np.testing.assert_allclose(xc[2], td[vs, us], rtol=1e-12)
    np.testing.assert_allclose(cam["fx"] * np.exp(p[3]) / xc[2], 1.0, rtol=1e-12)
    op = 1 / (1 + np.exp(-p[10]))
    np.testing.assert_allclose(op, np.where((m[vs, us] & 1) > 0, 0.9, 0.1), rtol=1e-12)
    np.testing.assert_array_equal(p[11:14], tc[:, vs, us])
