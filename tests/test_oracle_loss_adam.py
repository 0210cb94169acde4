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
