"""The C-ABI library loads, exports every symbol include/dqo.h declares, and
validates arguments on the host (no GPU needed: nothing is launched)."""
import ctypes
import os
import re

import pytest

from paper_2503_02223_amd import binding as B
from paper_2503_02223_amd import scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header="dqo.h"):
    src = open(os.path.join(ROOT, "include", header)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dqo_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    L = B.lib()
    names = _declared()
    assert len(names) >= 18
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(B.EXPORTED)
    learned = _declared("dqo_learned.h")
    for name in learned:
        assert hasattr(L, name), name
    assert set(learned) == set(B.EXPORTED_LEARNED)


def test_net_layout_and_learned_validation_on_host():
    L = B.lib()
    lay = B.NetLayout()
    assert L.dqo_net_layout_get(ctypes.byref(lay)) == 0
    assert list(lay.cin) == [5, 32, 64, 64] and list(lay.cout) == [32, 64, 64, 6]
    assert list(lay.cin_pad) == [16, 32, 64, 64] and list(lay.cout_pad) == [32, 64, 64, 16]
    n = 0
    for l in range(4):
        assert lay.w_offset[l] == n
        n += lay.cout_pad[l] * 9 * lay.cin_pad[l]
        assert lay.b_offset[l] == n
        n += lay.cout_pad[l]
    assert lay.n_params == n
    nb = ctypes.c_int64()
    assert L.dqo_net_workspace_size(4, 128, 128, ctypes.byref(nb)) == 0 and nb.value > 4 * 128 * 128 * 300
    assert L.dqo_net_workspace_size(4, 120, 128, ctypes.byref(nb)) == B.EINVAL
    ctx = B.Context()
    assert L.dqo_net_forward(ctx.h, 2, 100, 128, None, None, None, None, None, None) == B.EINVAL
    assert b"multiples of 16" in L.dqo_last_error(ctx.h)
    assert L.dqo_net_forward(ctx.h, 2, 128, 128, None, None, None, None, None, None) == B.EINVAL
    cams = B.make_cameras([{"R": [1, 0, 0, 0, 1, 0, 0, 0, 1], "t": [0, 0, 0], "fx": 110.0, "fy": 110.0,
                            "cx": 64.0, "cy": 64.0, "width": 128, "height": 128}] * 17)
    p = ctypes.c_void_p(16)
    assert L.dqo_init_gaussians(ctx.h, 17, 128, 128, p, cams, p, None, None, 10, p, p, 0, None) == B.EINVAL
    assert L.dqo_adam_flat(ctx.h, p, p, p, p, 10, 1e-3, 0.9, 1.5, 1e-8, p, None) == B.EINVAL


def test_version_and_status_strings():
    L = B.lib()
    assert b"gfx950" in L.dqo_version()
    assert L.dqo_status_string(B.ECAPACITY) == b"pair capacity exceeded"


def test_layout_and_validation_on_host():
    ctx = B.Context()
    sc = scenes.single_view_scene(n=100)
    cams = B.make_cameras(sc["cams"])
    d = B.FrameDesc(n=100, n_views=1, K=3, pair_capacity=5000, dtype=B.F32)
    L = B.Layout()
    assert B.lib().dqo_state_layout(ctx.h, ctypes.byref(d), cams, ctypes.byref(L)) == 0
    assert (L.tiles_x, L.tiles_y) == (8, 6)
    assert L.pair_key_bits == 6
    assert all(L.offset[i] % 256 == 0 for i in range(12))
    assert L.total >= L.offset[11] + L.bytes[11]
    assert L.bytes[0] == 100 * B.SPLAT_WORDS * 4 and L.bytes[9] == 5000 * 10 * 4
    for bad in (dict(n_views=0), dict(n_views=17), dict(K=65), dict(dtype=7), dict(n=-1),
                dict(pair_capacity=(1 << 30) + 1)):
        kw = dict(n=100, n_views=1, K=3, pair_capacity=5000, dtype=B.F32)
        kw.update(bad)
        d2 = B.FrameDesc(**kw)
        nv = max(1, min(kw["n_views"], 16))
        cams2 = B.make_cameras(sc["cams"] * nv)
        rc = B.lib().dqo_state_layout(ctx.h, ctypes.byref(d2), cams2, ctypes.byref(L))
        assert rc == B.EINVAL, bad
        assert B.lib().dqo_last_error(ctx.h)
    # mismatched view sizes
    c2 = dict(sc["cams"][0])
    c2["width"] = 64
    d3 = B.FrameDesc(n=100, n_views=2, K=3, pair_capacity=5000, dtype=B.F32)
    assert B.lib().dqo_state_layout(ctx.h, ctypes.byref(d3), B.make_cameras([sc["cams"][0], c2]),
                                    ctypes.byref(L)) == B.EINVAL


def test_bad_tile_config_rejected():
    cfg = B.default_config(tile_w=12, tile_h=12)
    with pytest.raises(B.DqoError):
        B.Context(cfg)
    for bad in (dict(depth_order=3), dict(depth_order=-1), dict(tile_sort_lds=4097), dict(tile_sort_lds=-1)):
        with pytest.raises(B.DqoError):
            B.Context(B.default_config(**bad))
    assert B.default_config().depth_order == B.DEPTH_ORDER_AUTO and B.default_config().tile_sort_lds == 0
    B.Context(B.default_config(depth_order=B.DEPTH_ORDER_TILE, tile_sort_lds=4096))


def test_null_pointers_rejected_before_launch():
    ctx = B.Context()
    sc = scenes.single_view_scene(n=10)
    cams = B.make_cameras(sc["cams"])
    d = B.FrameDesc(n=10, n_views=1, K=3, pair_capacity=100, dtype=B.F32)
    L = B.lib()
    assert L.dqo_project_cull_bin(ctx.h, ctypes.byref(d), cams, None, None, None, None) == B.EINVAL
    img = B.Images()
    assert L.dqo_render_forward(ctx.h, ctypes.byref(d), cams, ctypes.c_void_p(1), ctypes.byref(img), None) == B.EINVAL
    hp = B.AdamParams()
    assert L.dqo_adam_step(ctx.h, B.F32, None, None, None, None, 10, ctypes.byref(hp), 1, None) == B.EINVAL
    assert L.dqo_adam_step(ctx.h, B.F32, None, None, None, None, 0, ctypes.byref(hp), 0, None) == B.EINVAL
    assert L.dqo_fit_dual_quadric(ctx.h, 2, 4, None, None, None, 1, None, None, 1.0, None, None, None, None,
                                  None, None) == B.EINVAL


def test_segments_validated_on_host():
    ctx = B.Context()
    sc = scenes.single_view_scene(n=100)
    cams = B.make_cameras(sc["cams"] * 2)
    L = B.Layout()
    for seg, ok in (([0, 60, 60, 40], True), ([0, 100, 0, 100], True), ([0, 0, 100, 0], True),
                    ([0, 60, 60, 41], False), ([-1, 10, 0, 5], False), ([0, -2, 0, 5], False)):
        arr = (ctypes.c_int64 * 4)(*seg)
        d = B.FrameDesc(n=100, n_views=2, K=3, pair_capacity=5000, dtype=B.F32,
                        segments=ctypes.cast(arr, ctypes.POINTER(ctypes.c_int64)))
        rc = B.lib().dqo_state_layout(ctx.h, ctypes.byref(d), cams, ctypes.byref(L))
        assert (rc == 0) == ok, seg


def test_jobs_and_windows_validated_on_host():
    ctx = B.Context()
    sc = scenes.single_view_scene(n=100)
    cams = B.make_cameras(sc["cams"] * 2)
    L = B.Layout()
    for jobs, ok in (([-1, 2], True), ([0, 1], True), ([3, -1], False), ([-2, 0], False)):
        arr = (ctypes.c_int32 * 2)(*jobs)
        d = B.FrameDesc(n=100, n_views=2, K=3, pair_capacity=5000, dtype=B.F32,
                        jobs=ctypes.cast(arr, ctypes.POINTER(ctypes.c_int32)))
        rc = B.lib().dqo_state_layout(ctx.h, ctypes.byref(d), cams, ctypes.byref(L))
        assert (rc == 0) == ok, jobs
    # windows are clipped to the image (any values are accepted)
    win = (ctypes.c_int32 * 8)(-5, -5, 500, 500, 10, 10, 5, 5)
    d = B.FrameDesc(n=100, n_views=2, K=3, pair_capacity=5000, dtype=B.F32,
                    windows=ctypes.cast(win, ctypes.POINTER(ctypes.c_int32)))
    assert B.lib().dqo_state_layout(ctx.h, ctypes.byref(d), cams, ctypes.byref(L)) == 0
    # the loss of per-object jobs needs the observed ids
    arr = (ctypes.c_int32 * 2)(-1, 1)
    d = B.FrameDesc(n=100, n_views=2, K=3, pair_capacity=5000, dtype=B.F32,
                    jobs=ctypes.cast(arr, ctypes.POINTER(ctypes.c_int32)))
    fake = ctypes.c_void_p(1)   # never dereferenced: validation fails first
    img = B.Images(fake, fake, fake, fake, None, None, fake, fake, None)
    tgt = B.Targets(fake, fake, None)
    w = B.LossWeights(1.0, 1.0, 1.0, 1e-6)
    assert B.lib().dqo_object_loss(ctx.h, ctypes.byref(d), cams, ctypes.byref(img), ctypes.byref(tgt),
                                   ctypes.byref(w), fake, None, fake, None) == B.EINVAL
    assert b"target ids" in B.lib().dqo_last_error(ctx.h)


def test_new_entry_points_validate_on_host():
    """Incremental update, quadric refinement, pose gradient, fused backward +
    Adam and association: bad arguments are rejected with EINVAL and a
    message, before anything is launched."""
    ctx = B.Context()
    L = B.lib()
    sc = scenes.single_view_scene(n=10)
    cams = B.make_cameras(sc["cams"])
    d = B.FrameDesc(n=10, n_views=1, K=3, pair_capacity=100, dtype=B.F32)
    fake = ctypes.c_void_p(1)   # never dereferenced: validation fails first
    cfg = B.IncrementCfg(**B.INCREMENT_DEFAULTS)
    img, tgt = B.Images(), B.Targets()
    assert L.dqo_incremental_masks(ctx.h, ctypes.byref(d), cams, ctypes.byref(img), ctypes.byref(tgt),
                                   ctypes.byref(cfg), fake, fake, None) == B.EINVAL
    bad = B.IncrementCfg(**{**B.INCREMENT_DEFAULTS, "og_opacity": 1.0})
    assert L.dqo_densify(ctx.h, ctypes.byref(d), cams, ctypes.byref(B.Targets(fake, fake, fake)), fake,
                         ctypes.byref(bad), 0, 10, fake, fake, fake, None) == B.EINVAL
    assert b"opacit" in L.dqo_last_error(ctx.h)
    assert L.dqo_densify(ctx.h, ctypes.byref(d), cams, ctypes.byref(B.Targets(fake, fake, fake)), fake,
                         ctypes.byref(cfg), 10, 5, fake, fake, fake, None) == B.EINVAL   # n_cap < n_old
    rc = B.RefineCfg(**{**B.REFINE_DEFAULTS, "iterations": -1})
    assert L.dqo_refine_quadrics(ctx.h, 1, 1, fake, fake, fake, 1, fake, None, None, ctypes.byref(rc), fake, fake,
                                 fake, None, fake, None, None) == B.EINVAL
    rc = B.RefineCfg(**{**B.REFINE_DEFAULTS, "eps": 0.0})
    assert L.dqo_refine_quadrics(ctx.h, 1, 1, fake, fake, fake, 1, fake, None, None, ctypes.byref(rc), fake, fake,
                                 fake, None, fake, None, None) == B.EINVAL
    assert L.dqo_quadric_iou_grad(ctx.h, 1, 1, fake, fake, fake, 1, fake, None, None, None, None, None,
                                  None) == B.EINVAL
    assert L.dqo_pose_backward(ctx.h, ctypes.byref(d), cams, fake, fake, None, None) == B.EINVAL
    hp = B.AdamParams()
    hp.beta1, hp.beta2, hp.eps = 0.9, 1.0, 1e-15      # beta2 outside [0, 1)
    assert L.dqo_project_backward_adam(ctx.h, ctypes.byref(d), cams, fake, fake, fake, fake, ctypes.byref(hp),
                                       fake, None, None) == B.EINVAL
    assert L.dqo_associate(ctx.h, 1, fake, fake, fake, 2, fake, fake, 0, fake, fake, 0.3, fake, fake, None,
                           None) == B.EINVAL           # detections without frames
    assert L.dqo_quadric_distance(ctx.h, 1, fake, fake, fake, 1, fake, fake, fake, -1.0, fake, None) == B.EINVAL
    assert L.dqo_associate_decide(ctx.h, 40000, 0, fake, None, fake, fake, fake, 0.5, 0.85, 0.1, fake, fake, fake,
                                  fake, None) == B.EINVAL   # too many detections
    assert L.dqo_associate_decide(ctx.h, 3, 2, fake, None, fake, fake, fake, 0.5, 0.85, 0.1, fake, fake, fake, fake,
                                  None) == B.EINVAL         # objects without their QD
    assert L.dqo_associate_decide(ctx.h, 3, 0, fake, None, fake, fake, fake, 0.5, float("nan"), 0.1, fake, fake,
                                  fake, fake, None) == B.EINVAL
