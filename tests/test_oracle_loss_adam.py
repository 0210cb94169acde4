"""Pins for the object loss (Eq. (10)-(14) read as L1 colour + L1 depth + object
cross-entropy) and the Adam step: hand-computed values on 2x2 images and the
PyTorch library routines (l1_loss, nll_loss, torch.optim.Adam)."""
import numpy as np
import pytest
import torch


def test_loss_hand_values(oracle):
    C = np.array([[[0.5, 0.0], [1.0, 0.2]]] * 3)
    tC = np.zeros((3, 2, 2))
    D = np.array([[2.0, 1.0], [0.0, 3.0]])
    tD = np.array([[1.5, 0.0], [0.5, 3.0]])        # pixel (0,1) has no valid depth
    p = np.array([[0.5, 1.0], [1e-9, 0.25]])
    out = oracle.object_loss(C, D, p, tC, tD, None)
    assert out["l_rgb"] == pytest.approx((0.5 + 0 + 1.0 + 0.2) / 4)
    assert out["n_valid"] == 3
    assert out["l_depth"] == pytest.approx((0.5 + 0.5 + 0.0) / 3)
    lobj = (-np.log(0.5) - np.log(1.0) - np.log(1e-6) - np.log(0.25)) / 4
    assert out["l_obj"] == pytest.approx(lobj)
    assert out["loss"] == pytest.approx(out["l_rgb"] + out["l_depth"] + lobj)
    assert out["gp"][1, 0] == 0.0                 # clamped at eps: no gradient
    assert out["gp"][0, 0] == pytest.approx(-1 / (4 * 0.5))
    assert out["gD"][0, 1] == 0.0 and out["gD"][1, 1] == 0.0  # invalid / sign(0) = 0


def test_loss_matches_torch(oracle):
    rng = np.random.default_rng(0)
    H, W, K = 5, 7, 4
    C, tC = rng.uniform(size=(3, H, W)), rng.uniform(size=(3, H, W))
    D, tD = rng.uniform(1, 3, size=(H, W)), rng.uniform(-1, 3, size=(H, W))
    probs = rng.dirichlet(np.ones(K + 1), size=(H, W)).transpose(2, 0, 1)
    t = rng.integers(-1, K, size=(H, W))
    p_t = np.where(t >= 0, np.take_along_axis(probs[:K], np.maximum(t, 0)[None], 0)[0], probs[K])
    out = oracle.object_loss(C, D, p_t, tC, tD, t, w_rgb=0.7, w_depth=1.3, lam=0.5)
    l1 = torch.nn.functional.l1_loss(torch.tensor(C), torch.tensor(tC)).item()
    valid = tD > 0
    ld = torch.nn.functional.l1_loss(torch.tensor(D[valid]), torch.tensor(tD[valid])).item()
    logp = torch.log(torch.tensor(probs).clamp_min(1e-6)).permute(1, 2, 0).reshape(-1, K + 1)
    tgt = torch.tensor(np.where(t >= 0, t, K)).reshape(-1)
    ce = torch.nn.functional.nll_loss(logp, tgt).item()
    assert out["l_rgb"] == pytest.approx(l1, rel=1e-12)
    assert out["l_depth"] == pytest.approx(ld, rel=1e-12)
    assert out["l_obj"] == pytest.approx(ce, rel=1e-12)
    assert out["loss"] == pytest.approx(0.7 * l1 + 1.3 * ld + 0.5 * ce, rel=1e-12)
    # gradients against autograd
    tCt = torch.tensor(C, requires_grad=True)
    tDt = torch.tensor(D, requires_grad=True)
    tp = torch.tensor(p_t, requires_grad=True)
    L = (0.7 * torch.nn.functional.l1_loss(tCt, torch.tensor(tC))
         + 1.3 * torch.nn.functional.l1_loss(tDt[torch.tensor(valid)], torch.tensor(tD[valid]))
         + 0.5 * (-torch.log(tp.clamp_min(1e-6))).mean())
    L.backward()
    np.testing.assert_allclose(out["gC"], tCt.grad.numpy(), rtol=1e-12)
    np.testing.assert_allclose(out["gD"], tDt.grad.numpy(), rtol=1e-12)
    np.testing.assert_allclose(out["gp"], tp.grad.numpy(), rtol=1e-12)


def test_adam_matches_torch(oracle):
    rng = np.random.default_rng(1)
    n = 9
    p0 = rng.normal(size=(14, n))
    lrs = np.array([1e-3] * 3 + [5e-3] * 3 + [1e-3] * 4 + [5e-2] + [2.5e-3] * 3)
    tp = torch.tensor(p0.copy(), requires_grad=True)
    groups = [{"params": [], "lr": 0}]
    rows = [torch.nn.Parameter(tp.detach()[r].clone()) for r in range(14)]
    opt = torch.optim.Adam([{"params": [rows[r]], "lr": float(lrs[r])} for r in range(14)],
                           betas=(0.9, 0.999), eps=1e-15)
    p, m, v = p0.copy(), np.zeros_like(p0), np.zeros_like(p0)
    for step in range(1, 6):
        g = rng.normal(size=(14, n))
        for r in range(14):
            rows[r].grad = torch.tensor(g[r])
        opt.step()
        p, m, v = oracle.adam(p, g, m, v, step, lrs)
    got = np.stack([rows[r].detach().numpy() for r in range(14)])
    np.testing.assert_allclose(p, got, rtol=1e-12, atol=1e-14)
    del groups


def test_job_loss_hand_values(oracle):
    """One per-object job (object 1) on a 2x3 image with a window of its
    left 2x2 pixels: the colour and depth terms count the window pixels
    observed as object 1, the cross-entropy term every window pixel, on
    ins_1 = 1 - T_final where observed as 1 and on T_final elsewhere."""
    t_id = np.array([[[1, 0, 1], [-1, 1, 1]]])
    Tf = np.array([[[0.2, 0.6, 0.5], [0.9, 0.5, 0.1]]])
    P = np.zeros((1, 2, 2, 3))
    P[0, 1] = 1 - Tf[0]
    C = np.full((1, 3, 2, 3), 0.5)
    tC = np.zeros((1, 3, 2, 3))
    tC[0, :, 0, 0] = 0.1            # residual 0.4 on the first object pixel
    D = np.array([[[2.0, 9.0, 9.0], [9.0, 1.0, 9.0]]])
    tD = np.array([[[1.5, 0.0, 0.0], [0.0, 0.0, 0.0]]])   # valid depth only at (0, 0)
    out = oracle.object_loss_views(C, D, P, Tf, tC, tD, t_id, jobs=[1], windows=[(0, 0, 2, 2)])
    # window pixels (0,0) (0,1) (1,0) (1,1); observed as 1: (0,0), (1,1)
    assert out["n_colour"] == 2 and out["n_depth"] == 1 and out["n_obj"] == 4
    assert out["l_rgb"] == pytest.approx((3 * 0.4 + 3 * 0.5) / 6)
    assert out["l_depth"] == pytest.approx(0.5)
    ce = -np.log(0.8) - np.log(0.6) - np.log(0.9) - np.log(0.5)
    assert out["l_obj"] == pytest.approx(ce / 4)
    assert out["loss"] == pytest.approx(out["l_rgb"] + 0.5 + ce / 4)
    # gradients: -1/(4 p) on ins_1 at object pixels, on T_final elsewhere, none outside the window
    assert out["gP"][0, 1, 0, 0] == pytest.approx(-1 / (4 * 0.8))
    assert out["gT"][0, 0, 1] == pytest.approx(-1 / (4 * 0.6))
    assert out["gT"][0, 1, 0] == pytest.approx(-1 / (4 * 0.9))
    assert out["gP"][0, 1, 1, 1] == pytest.approx(-1 / (4 * 0.5))
    assert out["gT"][0, 0, 2] == 0 and out["gP"][0, 1, 0, 2] == 0 and out["gC"][0, :, 1, 2].sum() == 0
    assert (out["gC"][0, :, 0, 1] == 0).all()     # not observed as the object: no colour term
    assert out["gC"][0, 0, 0, 0] == pytest.approx(1 / 6)


def test_job_loss_matches_torch(oracle):
    """A whole-scene view and two per-object jobs with windows: the
    cross-entropy term equals torch's binary cross-entropy of ins_k against
    the observed mask over each job's window (and nll over the whole-scene
    window), the colour and depth terms torch's l1 over the counted pixels;
    gradients against autograd of that torch expression."""
    rng = np.random.default_rng(3)
    V, K, H, W = 3, 4, 6, 9
    jobs = [-1, 2, 3]
    windows = [(1, 0, 8, 6), (2, 1, 7, 5), (0, 2, 9, 6)]
    t_id = rng.integers(-1, K, size=(V, H, W))
    Tf = rng.uniform(0.05, 0.95, size=(V, H, W))
    P = np.zeros((V, K, H, W))
    P[0] = rng.dirichlet(np.ones(K), size=(H, W)).transpose(2, 0, 1) * (1 - Tf[0])
    for v in (1, 2):
        P[v, jobs[v]] = 1 - Tf[v]
    C, tC = rng.uniform(size=(V, 3, H, W)), rng.uniform(size=(V, 3, H, W))
    D, tD = rng.uniform(1, 3, size=(V, H, W)), rng.uniform(-1, 3, size=(V, H, W))
    out = oracle.object_loss_views(C, D, P, Tf, tC, tD, t_id, jobs=jobs, windows=windows, w_rgb=0.7,
                                   w_depth=1.3, lam=0.5)
    Ct, Dt, Pt, Tt = (torch.tensor(a, requires_grad=True) for a in (C, D, P, Tf))
    ce_terms, rgb_terms, d_terms = [], [], []
    for v in range(V):
        x0, y0, x1, y1 = windows[v]
        sl = (slice(y0, y1), slice(x0, x1))
        tv = torch.tensor(t_id[v][sl])
        if jobs[v] < 0:
            probs = torch.cat([Pt[v][(slice(None),) + sl], Tt[v][sl][None]], 0).clamp_min(1e-6)
            logp = torch.log(probs).permute(1, 2, 0).reshape(-1, K + 1)
            tgt = torch.where(tv >= 0, tv, torch.full_like(tv, K)).reshape(-1)
            ce_terms.append(torch.nn.functional.nll_loss(logp, tgt, reduction="sum"))
            cmask = torch.ones_like(tv, dtype=torch.bool)
        else:
            ins = Pt[v, jobs[v]][sl]
            m = (tv == jobs[v]).double()
            ce_terms.append(torch.nn.functional.binary_cross_entropy(ins, m, reduction="sum"))
            cmask = tv == jobs[v]
        rgb_terms.append((Ct[v][(slice(None),) + sl] - torch.tensor(tC[v][(slice(None),) + sl]))[:, cmask].abs())
        dm = cmask & (torch.tensor(tD[v][sl]) > 0)
        d_terms.append((Dt[v][sl] - torch.tensor(tD[v][sl]))[dm].abs())
    n_o = sum((y1 - y0) * (x1 - x0) for x0, y0, x1, y1 in windows)
    rgb = torch.cat([r.reshape(-1) for r in rgb_terms])
    dd = torch.cat(d_terms)
    L = 0.7 * rgb.mean() + 1.3 * dd.mean() + 0.5 * sum(ce_terms) / n_o
    assert out["n_obj"] == n_o and out["n_colour"] * 3 == rgb.numel() and out["n_depth"] == dd.numel()
    assert out["loss"] == pytest.approx(L.item(), rel=1e-12)
    L.backward()
    np.testing.assert_allclose(out["gC"], Ct.grad.numpy(), atol=1e-15)
    np.testing.assert_allclose(out["gD"], Dt.grad.numpy(), atol=1e-15)
    # whole-scene view: the probability the CE takes (P_t or T_final) receives the gradient
    np.testing.assert_allclose(out["gP"][0], Pt.grad.numpy()[0], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(out["gT"][0], Tt.grad.numpy()[0], rtol=1e-12, atol=1e-15)
    # jobs: ins_k and T_final are tied (ins_k = 1 - T_final); torch's BCE puts
    # the gradient on ins_k, the oracle on T_final where the mask is 0, so the
    # total derivative along T_final, dL/dT - dL/dins_k, must agree
    for v in (1, 2):
        k = jobs[v]
        ours = out["gT"][v] - out["gP"][v, k]
        theirs = Tt.grad.numpy()[v] - Pt.grad.numpy()[v, k]
        np.testing.assert_allclose(ours, theirs, rtol=1e-12, atol=1e-15)
        others = [j for j in range(K) if j != k]
        assert (out["gP"][v, others] == 0).all()


def test_job_loss_without_jobs_is_the_frame_loss(oracle):
    rng = np.random.default_rng(5)
    V, K, H, W = 2, 3, 4, 5
    t_id = rng.integers(-1, K, size=(V, H, W))
    Tf = rng.uniform(0.05, 0.95, size=(V, H, W))
    P = rng.dirichlet(np.ones(K), size=(V, H, W)).transpose(0, 3, 1, 2) * (1 - Tf)[:, None]
    C, tC = rng.uniform(size=(V, 3, H, W)), rng.uniform(size=(V, 3, H, W))
    D, tD = rng.uniform(1, 3, size=(V, H, W)), rng.uniform(-1, 3, size=(V, H, W))
    out = oracle.object_loss_views(C, D, P, Tf, tC, tD, t_id)
    p_t = np.where(t_id >= 0, np.take_along_axis(P, np.maximum(t_id, 0)[:, None], 1)[:, 0], Tf)
    ref = oracle.object_loss(C, D, p_t, tC, tD, t_id)
    for k in ("loss", "l_rgb", "l_depth", "l_obj"):
        assert out[k] == pytest.approx(ref[k], rel=1e-13)
    np.testing.assert_allclose(out["gC"], ref["gC"], rtol=1e-13)
