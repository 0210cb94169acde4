"""Pins for the oracle's forward image formation (alpha blending of colour,
depth and the instance channels of Eq. (12)).  References: closed forms for
one and two Gaussians, the transmittance telescoping identity, and the early
stop count."""
import numpy as np
import pytest

from paper_2503_02223_amd import scenes


def _one(mu, ls, q, eta, rgb):
    return scenes.pack(np.asarray(mu, float).reshape(3, 1), np.asarray(ls, float).reshape(3, 1),
                       np.asarray(q, float).reshape(4, 1), np.array([float(eta)]),
                       np.asarray(rgb, float).reshape(3, 1))


def _logit(o):
    return np.log(o / (1 - o))


def _grid(cam):
    u, v = np.meshgrid(np.arange(cam["width"]) + 0.5, np.arange(cam["height"]) + 0.5)
    return u, v


def _alpha_closed(cam, mx, my, S2, o):
    inv = np.linalg.inv(S2)
    u, v = _grid(cam)
    dx, dy = u - mx, v - my
    Q = inv[0, 0] * dx * dx + 2 * inv[0, 1] * dx * dy + inv[1, 1] * dy * dy
    a = np.minimum(0.99, o * np.exp(-0.5 * Q))
    a[(Q > 9) | (a < 1 / 255)] = 0.0
    return a


@pytest.mark.parametrize("o", [0.3, 0.8, 0.999])
def test_single_isotropic_gaussian_closed_form(oracle, o):
    cam = scenes.camera(width=40, height=30, cx=20, cy=15, fx=110, fy=110)
    z, s, rgb = 3.0, 0.08, np.array([0.2, 0.5, 0.9])
    p = _one([0, 0, z], [np.log(s)] * 3, [1, 0, 0, 0], _logit(o), rgb)
    out = oracle.render(p, np.array([1], np.int32), cam, K=2)
    var = (110 * s / z) ** 2 + 0.3
    u, v = _grid(cam)
    r2 = (u - 20) ** 2 + (v - 15) ** 2
    a = np.minimum(0.99, o * np.exp(-r2 / (2 * var)))
    a[(r2 > 9 * var) | (a < 1 / 255)] = 0
    for k in range(3):
        np.testing.assert_allclose(out["C"][k], rgb[k] * a, atol=1e-13)
    np.testing.assert_allclose(out["D"], z * a, atol=1e-12)
    np.testing.assert_allclose(out["Tf"], 1 - a, atol=1e-13)
    np.testing.assert_allclose(out["P"][1], a, atol=1e-13)
    np.testing.assert_allclose(out["P"][0], 0 * a, atol=0)
    assert ((out["last"] == 0) == (a > 0)).all()


def test_single_anisotropic_rotated_about_axis(oracle):
    cam = scenes.camera(width=64, height=48, cx=32, cy=24, fx=100, fy=100)
    th = 0.7
    z, sx, sy = 2.5, 0.12, 0.04
    q = [np.cos(th / 2), 0, 0, np.sin(th / 2)]
    p = _one([0, 0, z], [np.log(sx), np.log(sy), np.log(0.05)], q, _logit(0.9), [1, 0, 0])
    out = oracle.render(p, np.array([0], np.int32), cam, K=1)
    Rt = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    S2 = Rt @ np.diag([(100 * sx / z) ** 2, (100 * sy / z) ** 2]) @ Rt.T + 0.3 * np.eye(2)
    a = _alpha_closed(cam, 32.0, 24.0, S2, 0.9)
    np.testing.assert_allclose(out["C"][0], a, atol=1e-12)
    np.testing.assert_allclose(out["Tf"], 1 - a, atol=1e-12)


def test_two_gaussians_compose_front_to_back_and_swap(oracle):
    cam = scenes.camera(width=32, height=24, cx=16, cy=12, fx=80, fy=80)
    c1, c2 = np.array([1.0, 0.2, 0.0]), np.array([0.0, 0.4, 1.0])
    g1 = _one([0.01, 0.0, 2.0], [np.log(0.06)] * 3, [1, 0, 0, 0], _logit(0.7), c1)
    g2 = _one([-0.02, 0.01, 2.5], [np.log(0.1)] * 3, [1, 0, 0, 0], _logit(0.6), c2)
    ids = np.array([0, 1], np.int32)
    both = oracle.render(np.concatenate([g1, g2], 1), ids, cam, K=2)
    a1 = oracle.render(g1, ids[:1], cam, K=2)["P"][0]
    a2 = oracle.render(g2, ids[1:], cam, K=2)["P"][1]
    for k in range(3):
        np.testing.assert_allclose(both["C"][k], c1[k] * a1 + c2[k] * a2 * (1 - a1), atol=1e-13)
    np.testing.assert_allclose(both["D"], 2.0 * a1 + 2.5 * a2 * (1 - a1), atol=1e-12)
    # swap the depths: g2 now in front
    g1s, g2s = g1.copy(), g2.copy()
    g1s[2], g2s[2] = 2.5, 2.0
    sw = oracle.render(np.concatenate([g1s, g2s], 1), ids, cam, K=2)
    b1 = oracle.render(g1s, ids[:1], cam, K=2)["P"][0]
    b2 = oracle.render(g2s, ids[1:], cam, K=2)["P"][1]
    for k in range(3):
        np.testing.assert_allclose(sw["C"][k], c2[k] * b2 + c1[k] * b1 * (1 - b2), atol=1e-13)


def test_partition_of_unity_and_transmittance_bounds(oracle):
    sc = scenes.single_view_scene(seed=3, n=600)
    cam = sc["cams"][0]
    out = oracle.render(sc["params"], sc["ids"], cam, K=sc["K"])
    s = out["P"].sum(0) + out["Tf"]
    np.testing.assert_allclose(s, 1.0, atol=1e-12)
    assert (out["Tf"] >= 1e-4).all() and (out["Tf"] <= 1).all()
    assert (out["P"] >= 0).all()
    # depth is a weighted mean of camera depths: within [z_min, z_max] * (1 - Tf)
    pr = oracle.project(sc["params"], cam)
    z = pr["z"][pr["visible"]]
    w = 1 - out["Tf"]
    assert (out["D"] <= z.max() * w + 1e-12).all() and (out["D"] >= z.min() * w - 1e-12).all()
    # pixels with nothing blended are exactly background
    empty = out["nblend"] == 0
    assert (out["Tf"][empty] == 1).all() and (out["C"][:, empty] == 0).all()


def test_transmittance_is_product_over_blended(oracle):
    """T_final equals the product of (1 - alpha) over the Gaussians blended at the
    pixel, recomputed here from single-Gaussian renders."""
    sc = scenes.tiny_scene(seed=5, n=12, width=16, height=16, f=20.0)
    cam = sc["cams"][0]
    full = oracle.render(sc["params"], sc["ids"], cam, K=sc["K"])
    pr = oracle.project(sc["params"], cam)
    order = np.lexsort((np.arange(12), pr["z"]))
    alphas = []
    for i in range(12):
        one = oracle.render(sc["params"][:, i:i + 1], sc["ids"][i:i + 1], cam, K=sc["K"])
        alphas.append(1 - one["Tf"])
    alphas = np.array(alphas)
    T = np.ones((16, 16))
    stopped = np.zeros((16, 16), bool)
    for i in order:
        if not pr["visible"][i]:
            continue
        Tn = T * (1 - alphas[i])
        stop = (Tn < 1e-4) & (alphas[i] > 0)
        stopped |= stop
        T = np.where(stopped, T, Tn)
    np.testing.assert_allclose(full["Tf"], T, rtol=1e-12, atol=1e-15)


def test_early_stop_exact_count(oracle):
    """Ten o = 0.95 Gaussians projecting onto one pixel's sample point: three
    blend (T = 0.05^3 = 1.25e-4); a fourth would give 6.25e-6 < 1e-4."""
    cam = scenes.camera(width=16, height=16, cx=8, cy=8, fx=100, fy=100)
    gs = []
    for k in range(10):
        z = 2.0 + 0.1 * k
        x = 0.5 * z / 100.0   # projects to u = 8.5, the centre of pixel column 8
        y = 0.5 * z / 100.0
        gs.append(_one([x, y, z], [np.log(0.004)] * 3, [1, 0, 0, 0], _logit(0.95), [k / 10, 0, 0]))
    p = np.concatenate(gs, 1)
    out = oracle.render(p, np.zeros(10, np.int32), cam, K=1)
    assert out["nblend"][8, 8] == 3
    assert out["Tf"][8, 8] == pytest.approx(0.05 ** 3, rel=1e-12)
    assert out["last"][8, 8] == 2
    expect = 0.0 * 0.95 + 0.1 * 0.95 * 0.05 + 0.2 * 0.95 * 0.05 ** 2
    assert out["C"][0, 8, 8] == pytest.approx(expect, rel=1e-12)


def test_pixel_subset_matches_full_image(oracle):
    sc = scenes.single_view_scene(seed=2, n=300)
    cam = sc["cams"][0]
    full = oracle.render(sc["params"], sc["ids"], cam, K=3)
    pix = np.array([0, 17, 500, 128 * 96 - 1, 6000])
    sub = oracle.render(sc["params"], sc["ids"], cam, K=3, pix=pix)
    np.testing.assert_array_equal(sub["C"], full["C"].reshape(3, -1)[:, pix])
    np.testing.assert_array_equal(sub["last"], full["last"].reshape(-1)[pix])


def test_id_map_is_argmax_with_empty(oracle):
    P = np.array([[0.1, 0.5, 0.0], [0.3, 0.5, 0.0]])
    Tf = np.array([0.6, 0.0, 1.0])
    np.testing.assert_array_equal(oracle.id_map(P, Tf), [-1, 0, -1])
