"""GPU: the allocation-free object loss (dqo_object_loss_noalloc, partial sums
in the library's per-device scratch) against dqo_object_loss (partial sums in
the frame's state buffer) through the C ABI: the same kernels and reduction
order, so loss values and upstream gradients agree bitwise.  Calls in a row
with shrinking frames (the scratch keeps the previous call's partials)."""
import numpy as np
import pytest
import torch

from paper_2503_02223_amd import binding as B
from paper_2503_02223_amd import scenes
from tests.gpu_util import to_dev

pytestmark = pytest.mark.gpu


def _inputs(seed, V, H, W):
    rng = np.random.default_rng(seed)
    C, tC = rng.uniform(size=(V, 3, H, W)), rng.uniform(size=(V, 3, H, W))
    D, tD = rng.uniform(1, 3, size=(V, H, W)), rng.uniform(-1, 3, size=(V, H, W))
    pt = rng.uniform(0, 1, size=(V, H, W))
    pt.reshape(-1)[:5] = 1e-8
    tid = torch.tensor(rng.integers(-1, 3, size=(V, H, W)).astype(np.int32), device="cuda")
    img = dict(color=to_dev(C), depth=to_dev(D), p_target=to_dev(pt), t_final=to_dev(pt), target=tid)
    tgt = dict(color=to_dev(tC), depth=to_dev(tD), id=tid)
    return img, tgt


def _grads(V, H, W):
    return dict(d_color=torch.full((V, 3, H, W), np.nan, device="cuda"),
                d_depth=torch.full((V, H, W), np.nan, device="cuda"),
                d_p_target=torch.full((V, H, W), np.nan, device="cuda"))


@pytest.mark.parametrize("with_grads", [True, False])
def test_noalloc_loss_matches_state_loss(with_grads):
    ctx = B.Context()
    # largest first: 640x480 uses the most partial rows (511), the later
    # frames fewer, so a call that read rows beyond its own would see stale ones
    for seed, (V, H, W) in enumerate(((1, 480, 640), (2, 37, 53), (1, 20, 30))):
        img, tgt = _inputs(seed, V, H, W)
        cams = [scenes.camera(width=W, height=H)] * V
        f = B.Frame(ctx, cams, 10, 3, 100)
        ref_loss = torch.full((4,), np.nan, dtype=torch.float64, device="cuda")
        ref_g = _grads(V, H, W) if with_grads else None
        f.object_loss(img, tgt, ref_g, ref_loss, 0.8, 1.2, 0.5)
        loss = torch.full((4,), np.nan, dtype=torch.float64, device="cuda")
        g = _grads(V, H, W) if with_grads else None
        B.object_loss_noalloc(ctx, cams, 3, img, tgt, g, loss, 0.8, 1.2, 0.5)
        torch.cuda.synchronize()
        assert torch.isfinite(ref_loss).all() and float(ref_loss[0]) > 0
        assert torch.equal(loss, ref_loss), (V, H, W, loss, ref_loss)
        if with_grads:
            for k in ref_g:
                assert torch.isfinite(ref_g[k]).all()
                assert torch.equal(g[k], ref_g[k]), (V, H, W, k)


def test_noalloc_loss_validates_on_host():
    ctx = B.Context()
    cams = [scenes.camera(width=20, height=10)]
    img, tgt = _inputs(0, 1, 10, 20)
    loss = torch.zeros(4, dtype=torch.float64, device="cuda")
    bad = dict(img)
    del bad["p_target"]
    with pytest.raises(B.DqoError):
        B.object_loss_noalloc(ctx, cams, 3, bad, tgt, None, loss)
    with pytest.raises(B.DqoError):
        B.object_loss_noalloc(ctx, cams, 3, img, tgt, None, loss, ce_eps=0.0)
