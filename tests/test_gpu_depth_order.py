"""GPU: the two ways of putting each tile's pairs in depth order give the same
pair list.  GLOBAL radix-sorts every item by depth and emits pairs in that
order; TILE emits pairs in item order and sorts each tile's pairs by depth
after the tile sort (in LDS, or through global memory for tiles longer than
the LDS limit).  Both must give the blending order of Sec. III-D (by depth,
ties by item index), hence the same tile ranges and bitwise the same images;
the parameter gradients differ only in the order of the per-item sums."""
import numpy as np
import pytest
import torch

from paper_2503_02223_amd import binding as B
from paper_2503_02223_amd import scenes
from tests.gpu_util import pair_items, to_dev


pytestmark = pytest.mark.gpu


def _run(sc, tile, order, lds=0):
    n = sc["params"].shape[1]
    cam = sc["cams"][0]
    H, W = cam["height"], cam["width"]
    ctx = B.Context(tile_w=tile[0], tile_h=tile[1], depth_order=order, tile_sort_lds=lds)
    r = B.Rasterizer(sc["cams"], n, sc["K"], ctx=ctx)
    p = to_dev(sc["params"])
    ids = torch.tensor(sc["ids"], device="cuda")
    img = r.forward(p, ids)
    torch.cuda.synchronize()
    f = r.frame
    rc, st, P = f.read_status()
    assert rc == 0 and st == 0
    out = dict(P=P, vals=f.buf("pair_vals", torch.int32, P).cpu().numpy().copy(),
               keys=f.buf("pair_keys", torch.int32, P).cpu().numpy().copy(),
               ranges=f.buf("ranges", torch.int32).cpu().numpy().copy(),
               dkeys=f.buf("depth_keys", torch.int32, n).cpu().numpy().view(np.uint32).copy())
    for k in ("color", "depth", "t_final", "last"):
        out[k] = img[k].cpu().numpy()
    up = scenes.random_image_grads(41, (3, H, W))
    grads = dict(d_color=to_dev(up["gC"][None]), d_depth=to_dev(up["gD"][None]), d_t_final=to_dev(up["gT"][None]))
    out["grad"] = r.backward(p, img, grads).cpu().numpy()
    return out


# lds -1: the LDS limit at the median tile length, so both paths of the sort run
@pytest.mark.parametrize("n,tile,lds", [(2000, (8, 8), 0), (2000, (16, 16), 0), (30000, (8, 8), 0),
                                        (30000, (8, 8), 64), (30000, (16, 16), -1)])
def test_tile_depth_order_matches_global(n, tile, lds):
    sc = scenes.single_view_scene(seed=3, n=n)
    g = _run(sc, tile, B.DEPTH_ORDER_GLOBAL)
    if lds < 0:
        rg = g["ranges"].reshape(-1, 2)
        lds = int(np.median(rg[:, 1] - rg[:, 0]))
    t = _run(sc, tile, B.DEPTH_ORDER_TILE, lds)
    assert g["P"] == t["P"] and g["P"] > 1000
    assert (g["keys"] == t["keys"]).all() and (g["ranges"] == t["ranges"]).all()
    assert (g["vals"] == t["vals"]).all()
    rng = t["ranges"].reshape(-1, 2)
    lens = rng[:, 1] - rng[:, 0]
    if lds:
        # both paths of the per-tile sort ran
        assert (lens > lds).sum() > 0 and ((lens > 1) & (lens <= lds)).sum() > 0
    # the order itself: by tile, then the item's depth key, then item index
    item = pair_items(t["vals"]).astype(np.int64)
    order = np.lexsort((item, t["dkeys"][item], t["keys"]))
    assert (order == np.arange(t["P"])).all()
    for k in ("color", "depth", "t_final", "last"):
        assert np.array_equal(g[k], t[k]), k
    np.testing.assert_allclose(t["grad"], g["grad"], rtol=1e-5, atol=1e-6 * np.abs(g["grad"]).max())
