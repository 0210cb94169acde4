"""GPU: the device status word.  A bounded device wait that gives up sets a
status bit; from then on the sort orders its blocks by ticket instead of by
workgroup index (which needs the whole grid resident), and the training loop
reports the bit.  The bit is set from the host here (every kernel runs to
completion normally); the sort must give the same order either way."""
import numpy as np
import pytest
import torch

from paper_2503_02223_amd import binding as B
from paper_2503_02223_amd import scenes
from tests.gpu_util import to_dev

pytestmark = pytest.mark.gpu

# int32 words of the control block: status, epoch, pair count, valid count, counters[16]
STATUS, NPAIRS, COUNTERS = 0, 2, 4
DEPTH_TICKETS = slice(COUNTERS + 0, COUNTERS + 4)
SCAN_TICKET = COUNTERS + 4
PAIR_TICKETS = slice(COUNTERS + 5, COUNTERS + 7)


def _set_timeout_bit(f):
    ctrl = f.buf("control", torch.int32)
    ctrl[STATUS] = ctrl[STATUS] | B.STATUS_TIMEOUT


@pytest.mark.parametrize("view", ["128x96", "640x480"])
def test_timeout_bit_switches_sort_to_ticket_order(view):
    # 128x96: 192 tiles, one 8-bit pair pass; 640x480: 4800 tiles, two
    n = 2000 if view == "128x96" else 20000
    sc = scenes.single_view_scene(seed=1, n=n) if view == "128x96" else scenes.slam_view_scene(seed=1, n=n)
    # the global depth order, whose four depth passes take tickets too
    r = B.Rasterizer(sc["cams"], n, 3 if view == "128x96" else sc["K"],
                     ctx=B.Context(tile_w=8, tile_h=8, depth_order=B.DEPTH_ORDER_GLOBAL))
    p = to_dev(sc["params"])
    ids = torch.tensor(sc["ids"], device="cuda")
    r.bin(p, ids)          # sizes the pair list (grows it on overflow)
    f = r.frame
    f.project_cull_bin(p, ids)
    f.sort()
    torch.cuda.synchronize()
    rc, st, npairs = f.read_status()
    assert rc == 0 and st == 0
    ctrl = f.buf("control", torch.int32)
    assert npairs > 4096   # two pair blocks at least
    ref = {k: f.buf(k, torch.int32)[:npairs].clone() for k in ("pair_keys", "pair_vals")}
    ref["depth_order"] = f.buf("depth_order", torch.int32)[:n].clone()
    ref["ranges"] = f.buf("ranges", torch.int32).clone()
    assert (ctrl[DEPTH_TICKETS] == 0).all() and int(ctrl[SCAN_TICKET]) == 0 and (ctrl[PAIR_TICKETS] == 0).all()

    _set_timeout_bit(f)
    f.project_cull_bin(p, ids)
    f.sort()
    torch.cuda.synchronize()
    rc, st, npairs2 = f.read_status()
    assert rc == B.EINTERNAL and st & B.STATUS_TIMEOUT and npairs2 == npairs
    ctrl = f.buf("control", torch.int32)
    # every block of every pass took a ticket: the depth passes' blocks of
    # 2048 items, the scan's blocks of 512; the emission performs the first
    # pair pass itself (its grid fits on the device), so only a second pair
    # pass runs (its grid is sized by the pair capacity)
    # (the fourth depth pass draws none when three passes suffice for the key range)
    dt = ctrl[DEPTH_TICKETS].cpu().numpy()
    assert (dt[:3] == (n + 2047) // 2048).all() and dt[3] in (0, (n + 2047) // 2048), dt
    assert int(ctrl[SCAN_TICKET]) == (n + 511) // 512
    assert int(ctrl[PAIR_TICKETS][0]) == 0, ctrl[PAIR_TICKETS]
    if view == "640x480":
        assert int(ctrl[PAIR_TICKETS][1]) >= 2, ctrl[PAIR_TICKETS]
    else:
        assert int(ctrl[PAIR_TICKETS][1]) == 0, ctrl[PAIR_TICKETS]
    for k in ("pair_keys", "pair_vals"):
        assert torch.equal(f.buf(k, torch.int32)[:npairs], ref[k]), k
    assert torch.equal(f.buf("depth_order", torch.int32)[:n], ref["depth_order"])
    assert torch.equal(f.buf("ranges", torch.int32), ref["ranges"])

    f.clear_status()
    f.project_cull_bin(p, ids)
    f.sort()
    rc, st, _ = f.read_status()
    assert rc == 0 and st == 0
    ctrl = f.buf("control", torch.int32)
    assert (ctrl[DEPTH_TICKETS] == 0).all() and int(ctrl[SCAN_TICKET]) == 0


def test_trainer_reports_a_timeout():
    sc = scenes.single_view_scene(seed=2, n=2000)
    p = to_dev(sc["params"])
    ids = torch.tensor(sc["ids"], device="cuda")
    r0 = B.Rasterizer(sc["cams"], 2000, 3)
    t0 = r0.forward(to_dev(scenes.perturb(sc["params"], 1)), ids, probs=True, id_map=True)
    targets = dict(color=t0["color"].clone(), depth=t0["depth"].clone(), id=t0["id_map"].clone())
    tr = B.Trainer(p, ids, sc["cams"], 3, targets, ctx=B.Context(tile_w=8, tile_h=8), status_every=3)
    tr.step()
    tr.step()
    _set_timeout_bit(tr.r.frame)
    with pytest.raises(B.DqoError) as e:
        tr.step()       # the third step reads the status
    assert e.value.code == B.EINTERNAL
    tr.r.frame.clear_status()
    for _ in range(3):
        tr.step()
    assert np.isfinite(tr.loss.cpu().numpy()).all()
