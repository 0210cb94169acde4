"""Helpers for the GPU parity tests (no test functions here)."""
import numpy as np
import pytest
import torch

GPU = torch.cuda.is_available()

# Tolerances: colour/depth 1e-4 relative, gradients 1e-3 relative, with the
# floor of 1e-2 * max|oracle| for near-zero entries, plus a normwise bound.
FWD_RTOL = 1e-4
GRAD_RTOL = 1e-3
BAND = 1e-4  # pixels whose oracle threshold margin is below this are ambiguous
DEPTH_BAND = 1e-6  # ... or whose consecutive contributors are closer in depth than this (FP32 z)


def unambiguous(ref, grads=False):
    ok = (ref["margin"] > BAND) & (ref["depth_gap"] > DEPTH_BAND)
    if grads:
        ok &= ref["margin_clamp"] > BAND
    return ok


def skip_no_gpu():
    return pytest.mark.skipif(not GPU, reason="needs a GPU")


def pair_items(vals):
    """Item indices of pair values read after a forward (which marks the
    pairs that cannot contribute in their tile with the top bit)."""
    return np.asarray(vals) & 0x7FFFFFFF


def to_dev(a, dtype=torch.float32):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def close(gpu, ref, rtol, mask=None, what=""):
    """Elementwise |g - o| <= rtol * max(|o|, 1e-2 * max|o|) and normwise
    ||g - o|| / ||o|| <= rtol on the entries selected by mask."""
    g = np.asarray(gpu, np.float64)
    o = np.asarray(ref, np.float64)
    if mask is not None:
        g, o = g[..., mask], o[..., mask]
    g, o = g.ravel(), o.ravel()
    if o.size == 0:
        return
    scale = np.abs(o).max()
    floor = 1e-2 * scale if scale > 0 else 1e-30
    err = np.abs(g - o)
    tol = rtol * np.maximum(np.abs(o), floor)
    bad = err > tol
    nrm = np.linalg.norm(o)
    rel = np.linalg.norm(g - o) / nrm if nrm > 0 else np.linalg.norm(g - o)
    assert not bad.any(), (f"{what}: {bad.sum()} / {bad.size} entries out of tolerance; worst err "
                           f"{err[bad].max():.3e} at ref {o[bad][np.argmax(err[bad])]:.3e}; normwise {rel:.2e}")
    assert rel <= rtol, f"{what}: normwise relative error {rel:.3e} > {rtol}"


def target_images(oracle, scenes, sc, seed=1):
    """Targets from a perturbed copy of the scene, rendered by the oracle."""
    cam = sc["cams"][0]
    tg = oracle.render(scenes.perturb(sc["params"], seed), sc["ids"], cam, K=sc["K"])
    return dict(C=tg["C"], D=tg["D"], id=oracle.id_map(tg["P"], tg["Tf"]))
