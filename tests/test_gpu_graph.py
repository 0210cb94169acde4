"""GPU: the training step captured in a HIP graph replays exactly like eager
steps (checked after every replay, with unrelated eager work and
synchronisations in between), the device-counted Adam equals the host-step
Adam, mask boxes, and the tile autotuner."""
import numpy as np
import pytest
import torch

from paper_2503_02223_amd import autotune
from paper_2503_02223_amd import binding as B
from paper_2503_02223_amd import scenes
from tests.gpu_util import to_dev

pytestmark = pytest.mark.gpu


def _setup(oracle, tile=(8, 8)):
    sc = scenes.single_view_scene(seed=6, n=2000)
    cam = sc["cams"][0]
    tg = oracle.render(scenes.perturb(sc["params"], 7), sc["ids"], cam, K=3)
    targets = dict(color=to_dev(tg["C"][None]), depth=to_dev(tg["D"][None]),
                   id=torch.tensor(oracle.id_map(tg["P"], tg["Tf"])[None], dtype=torch.int32, device="cuda"))
    ids = torch.tensor(sc["ids"], device="cuda")
    p = to_dev(sc["params"])
    mk = lambda: B.Trainer(p.clone(), ids, sc["cams"], 3, targets, ctx=B.Context(tile_w=tile[0], tile_h=tile[1]))
    return mk


@pytest.mark.parametrize("tile", [(8, 8), (16, 16)])
def test_graph_replays_match_eager_steps(oracle, tile):
    mk = _setup(oracle, tile)
    eager, graphed = mk(), mk()
    g = graphed.capture()          # runs one warm-up step on `graphed`
    eager.step()
    torch.cuda.synchronize()
    assert torch.equal(eager.params, graphed.params)
    for i in range(4):
        eager.step()
        g.replay()
        junk = torch.randn(4096, device="cuda")
        junk = (junk * 2).sum()     # unrelated eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(eager.params, graphed.params), f"replay {i}"
        assert torch.equal(eager.loss, graphed.loss), f"replay {i}"
        assert torch.equal(eager.m, graphed.m) and torch.equal(eager.v, graphed.v)
    assert int(graphed.d_step.item()) == 5 and int(eager.d_step.item()) == 5
    graphed.check()


def test_counted_adam_equals_host_step_adam():
    rng = np.random.default_rng(3)
    ctx = B.Context()
    n = 1000
    p0 = to_dev(rng.normal(size=(14, n)))
    a = [p0.clone(), torch.zeros_like(p0), torch.zeros_like(p0)]
    b = [p0.clone(), torch.zeros_like(p0), torch.zeros_like(p0)]
    d_step = torch.zeros(1, dtype=torch.int64, device="cuda")
    lrs = B.default_lrs(2.0)
    for step in range(1, 6):
        g = to_dev(rng.normal(size=(14, n)))
        B.adam_step(ctx, a[0], g, a[1], a[2], lrs, step)
        B.adam_step_counted(ctx, b[0], g, b[1], b[2], lrs, d_step)
    torch.cuda.synchronize()
    assert int(d_step.item()) == 5
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def test_id_boxes_match_plain_min_max():
    rng = np.random.default_rng(0)
    V, H, W, K = 3, 50, 70, 6
    idm = np.full((V, H, W), -1, np.int32)
    for v in range(V):
        for k in range(K - 1):  # object K-1 never appears
            x0, y0 = rng.integers(0, W - 10), rng.integers(0, H - 10)
            idm[v, y0:y0 + rng.integers(1, 10), x0:x0 + rng.integers(1, 10)] = k
    boxes, bo, bv = B.id_boxes(B.Context(), torch.tensor(idm, device="cuda"), K)
    torch.cuda.synchronize()
    boxes, bo, bv = boxes.cpu().numpy(), bo.cpu().numpy(), bv.cpu().numpy()
    for v in range(V):
        for k in range(K):
            i = v * K + k
            assert bv[i] == v
            ys, xs = np.nonzero(idm[v] == k)
            if xs.size == 0:
                assert bo[i] == -1
            else:
                assert bo[i] == k
                np.testing.assert_array_equal(boxes[i], [xs.min(), ys.min(), xs.max() + 1, ys.max() + 1])


def test_autotune_picks_a_measured_tile(oracle):
    mk = _setup(oracle)
    best, table = autotune.autotune_tile(lambda ctx: B.Trainer(mk().params, mk().ids, mk().r.cams, 3, mk().targets,
                                                               ctx=ctx),
                                         candidates=((8, 8), (16, 16)), warmup=1, reps=2)
    assert best in ((8, 8), (16, 16))
    assert set(table) == {"8x8", "16x16"} and all(v > 0 for v in table.values())
    assert table[f"{best[0]}x{best[1]}"] == min(table.values())


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_fused_backward_adam_equals_separate_calls(oracle, dtype):
    """dqo_project_backward_adam against dqo_project_backward followed by
    dqo_adam_step_counted: bitwise equal parameters, moments and gradients
    over several steps, the step counter advanced once per call."""
    sc = scenes.single_view_scene(seed=6, n=2000)
    cam = sc["cams"][0]
    tg = oracle.render(scenes.perturb(sc["params"], 7), sc["ids"], cam, K=3)
    targets = dict(color=to_dev(tg["C"][None], dtype), depth=to_dev(tg["D"][None], dtype),
                   id=torch.tensor(oracle.id_map(tg["P"], tg["Tf"])[None], dtype=torch.int32, device="cuda"))
    ids = torch.tensor(sc["ids"], device="cuda")
    p = to_dev(sc["params"], dtype)
    sep = B.Trainer(p.clone(), ids, sc["cams"], 3, targets, fused=False)
    fus = B.Trainer(p.clone(), ids, sc["cams"], 3, targets, fused=True)
    grads_f = torch.empty_like(p)
    for i in range(4):
        sep.step()
        f = fus.r.frame
        f.project_cull_bin(fus.params, fus.ids)
        f.sort()
        f.render_forward(fus.img)
        f.object_loss(fus.img, fus.targets, fus.grads_img, fus.loss)
        f.render_backward(fus.img, fus.grads_img)
        f.project_backward_adam(fus.params, fus.m, fus.v, fus.lrs, fus.d_step, grads=grads_f)
        torch.cuda.synchronize()
        assert torch.equal(sep.grads, grads_f), f"gradients, step {i}"
        assert torch.equal(sep.params, fus.params), f"params, step {i}"
        assert torch.equal(sep.m, fus.m) and torch.equal(sep.v, fus.v), f"moments, step {i}"
        assert int(sep.d_step.item()) == i + 1 and int(fus.d_step.item()) == i + 1
