"""Measured choice of the pixel-tile shape for a workload.

The render kernels process one tile per workgroup; the LDS batch of splat
records equals the tile's pixel count (one record per pixel thread), so the
tile shape fixes both.  Smaller tiles shorten the longest per-pixel walk (fewer
Gaussians overlap a tile) but emit more (tile, Gaussian) pairs to sort; which
wins depends on the scene, so each candidate is timed on the real workload as a
captured HIP graph of the whole training step, and the fastest is kept.
"""
from __future__ import annotations

from typing import Callable, Dict, Sequence, Tuple

import torch

from . import binding as B

DEFAULT_CANDIDATES = ((8, 8), (16, 8), (16, 16), (32, 8))


def time_graph(g, warmup: int = 2, reps: int = 5) -> float:
    for _ in range(warmup):
        g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def autotune_tile(make_trainer: Callable[[B.Context], "B.Trainer"],
                  candidates: Sequence[Tuple[int, int]] = DEFAULT_CANDIDATES,
                  warmup: int = 2, reps: int = 5) -> Tuple[Tuple[int, int], Dict[str, float]]:
    """make_trainer(ctx) builds a fresh Trainer (from the initial parameters)
    with the given context.  Returns the fastest tile and the ms per step of
    every candidate."""
    results: Dict[str, float] = {}
    best, best_ms = None, float("inf")
    for tw, th in candidates:
        tr = make_trainer(B.Context(tile_w=tw, tile_h=th))
        g = tr.capture()
        ms = time_graph(g, warmup, reps)
        tr.check()
        results[f"{tw}x{th}"] = round(ms, 4)
        if ms < best_ms:
            best, best_ms = (tw, th), ms
        del g, tr
        torch.cuda.empty_cache()
    return best, results
