"""Throughput of the training iteration of the object-aware Gaussian rasterizer.

One step = project/cull/bin + sort + render forward + object loss + render
backward + project backward + Adam, on the 200k-Gaussian room (20 object blobs
plus 30% background, ids 0..20) seen whole by a 640x480 camera (f = 600), all
inputs resident on the GPU.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps 100] [--warmup 10] [--no-cpu]
"""
import argparse
import json
import os
import sys
import tempfile
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2503_02223_amd import binding as B  # noqa: E402
from paper_2503_02223_amd import scenes  # noqa: E402

METRIC = "fwd+bwd iters/s @640x480, 200k Gaussians; time-to-PSNR learned vs plain init"
MI355X_FP32_VECTOR_TFLOPS = 157.3   # published fp32 vector peak (256 CUs, 2.4 GHz)
MI355X_HBM_GBS = 8000.0             # published HBM3E bandwidth
# v_exp_f32 at a quarter of the non-packed FMA rate: 256 CUs x 4 SIMDs x 16 lanes / 4 x 2.4 GHz
MI355X_EXP_PER_S = 256 * 4 * 16 / 4 * 2.4e9
# Algorithmic work of the render backward per launch (the cost model of the
# hot-path plan): 60 FLOP and one exponential per examined (pixel, pair), i.e.
# every pair of the pixel's tile range at or before its last blended one; bytes
# = 44 per pair of the list (pair value + 40-byte record) + 32 per pixel
# (upstream gradients, T_final, last) + 40 per written (tile, Gaussian) pair of
# gradient partials.
FLOP_PER_EXAMINED = 60.0
BYTES_PER_PAIR, BYTES_PER_PIXEL, BYTES_PER_WRITTEN = 44.0, 32.0, 40.0
# HBM bytes per launch of the render backward from rocprofv3 FETCH_SIZE + WRITE_SIZE
# (scaled by a 256 MiB copy: x2.000 and x1.000), valid only for the kernel source
# they were taken with (render.hip and dqo_device.hpp); reported as null otherwise.
MEASURED_TRAFFIC = {"render_src_sha256_16": "5113419c6b02e3c7", "bytes_per_launch": 145690000}


def measured_traffic():
    import hashlib
    h = hashlib.sha256()
    for name in ("render.hip", "dqo_device.hpp"):  # the kernel and its constants
        with open(os.path.join(ROOT, "paper_2503_02223_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    h = h.hexdigest()[:16]
    return MEASURED_TRAFFIC["bytes_per_launch"] if h == MEASURED_TRAFFIC["render_src_sha256_16"] else None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build_workload(seed=0, n=200_000):
    sc = scenes.slam_view_scene(seed=seed, n=n)
    dev = "cuda"
    p = torch.tensor(sc["params"], dtype=torch.float32, device=dev)
    ids = torch.tensor(sc["ids"], device=dev)
    # Targets: the same scene perturbed (means, scales, opacities, colours), rendered once.
    pt = torch.tensor(scenes.perturb(sc["params"], seed + 1), dtype=torch.float32, device=dev)
    r0 = B.Rasterizer(sc["cams"], n, sc["K"])
    t0 = r0.forward(pt, ids, probs=True, id_map=True)
    torch.cuda.synchronize()
    targets = dict(color=t0["color"].clone(), depth=t0["depth"].clone(), id=t0["id_map"].clone())
    del r0, t0
    return sc, p, ids, targets


def backward_work(tr):
    """Examined (pixel, pair) count E and blended count B of the current state."""
    f = tr.r.frame
    img = f.new_images(target=tr.targets["id"], n_blend=True)
    f.project_cull_bin(tr.params, tr.ids)
    f.sort()
    f.render_forward(img)
    torch.cuda.synchronize()
    last = img["last"][0].long()
    tw, th = tr.r.ctx.config.tile_w, tr.r.ctx.config.tile_h
    H, W = last.shape
    tx = (torch.arange(W, device=last.device) // tw)
    ty = (torch.arange(H, device=last.device) // th)
    tile = ty[:, None] * f.layout.tiles_x + tx[None, :]
    ranges = f.buf("ranges", torch.int32).view(-1, 2).long()
    start = ranges[tile, 0]
    E = torch.where(last >= 0, last - start + 1, torch.zeros_like(last)).sum().item()
    Bn = img["n_blend"].long().sum().item()
    return int(E), int(Bn)


def written_pairs(tr):
    """(tile, Gaussian) pairs whose gradient partials the render backward
    writes in the current state: partials zeroed, one backward, records with a
    nonzero entry counted (the loss's sign gradients make every written record
    nonzero)."""
    f = tr.r.frame
    f.project_cull_bin(tr.params, tr.ids)
    f.sort()
    f.render_forward(tr.img)
    f.object_loss(tr.img, tr.targets, tr.grads_img, tr.loss)
    part = f.buf("partials", torch.float32)
    part.zero_()
    f.render_backward(tr.img, tr.grads_img)
    torch.cuda.synchronize()
    return int((part.view(-1, 10) != 0).any(1).sum().item())


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def small_scene_comparison(steps=200):
    """The 2k-Gaussian 128x96 scene: GPU microseconds per training iteration
    (the same step as the headline) against the FP64 oracle's seconds per
    forward + loss + backward + Adam on the whole image."""
    import oracle
    sc = scenes.single_view_scene(seed=0, n=2000)
    cam = sc["cams"][0]
    K = sc["K"]
    tg = oracle.render(scenes.perturb(sc["params"], 1), sc["ids"], cam, K=K)
    t_id = oracle.id_map(tg["P"], tg["Tf"])
    t0 = time.perf_counter()
    out = oracle.render(sc["params"], sc["ids"], cam, K=K)
    p_t = np.where(t_id >= 0, np.take_along_axis(out["P"], np.maximum(t_id, 0)[None], 0)[0], out["Tf"])
    lo = oracle.object_loss(out["C"], out["D"], p_t, tg["C"], tg["D"], t_id)
    gP = np.zeros((K,) + t_id.shape)
    for k in range(K):
        gP[k] = np.where(t_id == k, lo["gp"], 0.0)
    gT = np.where(t_id == -1, lo["gp"], 0.0)
    grads, _ = oracle.render_backward(sc["params"], sc["ids"], cam, K=K, gC=lo["gC"], gD=lo["gD"], gP=gP, gT=gT)
    z = np.zeros_like(sc["params"])
    oracle.adam(sc["params"], grads, z, z, 1, B.default_lrs())
    t_oracle = time.perf_counter() - t0
    dev = "cuda"
    targets = dict(color=torch.tensor(tg["C"][None], dtype=torch.float32, device=dev),
                   depth=torch.tensor(tg["D"][None], dtype=torch.float32, device=dev),
                   id=torch.tensor(t_id[None], dtype=torch.int32, device=dev))
    tr = B.Trainer(torch.tensor(sc["params"], dtype=torch.float32, device=dev),
                   torch.tensor(sc["ids"], device=dev), sc["cams"], K, targets,
                   ctx=B.Context(tile_w=8, tile_h=8), status_every=0)
    for _ in range(10):
        tr.step()
    g = tr.capture()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(steps):
        g.replay()
    torch.cuda.synchronize()
    gpu_us = (time.perf_counter() - t1) * 1e6 / steps
    tr.check()
    return dict(workload="2,000 Gaussians, 128x96, K=3, 8x8 tiles; forward + object loss + backward + Adam "
                         "(the GPU step replayed as one HIP graph)",
                gpu_us_per_iter=round(gpu_us, 2), oracle_s_per_iter=round(t_oracle, 4),
                oracle_cores=oracle.num_threads())


def cpu_baseline(sc, targets_seed=1, n_pix=1024, seed=0):
    """The FP64 oracle (every Gaussian at every sampled pixel) on a bounded
    sample of the same workload: forward + loss + backward over n_pix random
    pixels of the 640x480 frame with all 200k Gaussians, plus Adam over all
    Gaussians; scaled to a full 307,200-pixel iteration."""
    import oracle
    cam = sc["cams"][0]
    HW = cam["width"] * cam["height"]
    rng = np.random.default_rng(seed)
    pix = np.sort(rng.choice(HW, size=n_pix, replace=False)).astype(np.int64)
    K = sc["K"]
    tg = oracle.render(scenes.perturb(sc["params"], targets_seed), sc["ids"], cam, K=K, pix=pix)
    t_id = oracle.id_map(tg["P"], tg["Tf"])
    t0 = time.perf_counter()
    out = oracle.render(sc["params"], sc["ids"], cam, K=K, pix=pix)
    p_t = np.where(t_id >= 0, np.take_along_axis(out["P"], np.maximum(t_id, 0)[None], 0)[0], out["Tf"])
    lo = oracle.object_loss(out["C"], out["D"], p_t, tg["C"], tg["D"], t_id)
    gP = np.zeros((K, n_pix))
    for k in range(K):
        gP[k] = np.where(t_id == k, lo["gp"], 0.0)
    gT = np.where(t_id == -1, lo["gp"], 0.0)
    grads, _ = oracle.render_backward(sc["params"], sc["ids"], cam, K=K, gC=lo["gC"], gD=lo["gD"], gP=gP, gT=gT,
                                      pix=pix)
    t_render = time.perf_counter() - t0
    t1 = time.perf_counter()
    z = np.zeros_like(sc["params"])
    oracle.adam(sc["params"], grads, z, z, 1, B.default_lrs())
    t_adam = time.perf_counter() - t1
    per_iter = t_render * (HW / n_pix) + t_adam
    return dict(value=1.0 / per_iter, unit="iters/s", cores=oracle.num_threads(), cpu_model=cpu_model(),
                kind="oracle",
                sample=f"FP64 forward+object loss+backward over {n_pix} of {HW} pixels with all "
                       f"{sc['params'].shape[1]} Gaussians ({t_render:.1f} s) scaled by the pixel count, "
                       f"plus one Adam step over all Gaussians ({t_adam:.2f} s)")


def bench_keyframes(args):
    """8 ring keyframes at 640x480 over 1.2M Gaussians in 40 objects + background
    (K = 41): every view rendered and back-propagated in one launch per kernel,
    the whole step captured in a HIP graph, the tile shape chosen by measuring
    each candidate; then the per-object quadric fit from the 8 views' mask boxes
    and its refinement by the IoU loss."""
    from paper_2503_02223_amd import autotune
    sc = scenes.keyframe_scene(seed=0)
    n = sc["params"].shape[1]
    V = len(sc["cams"])
    p0 = torch.tensor(sc["params"], dtype=torch.float32, device="cuda")
    ids = torch.tensor(sc["ids"], device="cuda")
    pt = torch.tensor(scenes.perturb(sc["params"], 1), dtype=torch.float32, device="cuda")
    r0 = B.Rasterizer(sc["cams"], n, sc["K"], ctx=B.Context(tile_w=16, tile_h=16))
    t0 = r0.forward(pt, ids, probs=True, id_map=True)
    torch.cuda.synchronize()
    targets = dict(color=t0["color"].clone(), depth=t0["depth"].clone(), id=t0["id_map"].clone())
    del r0, t0
    torch.cuda.empty_cache()
    # Per-object jobs beside the whole-scene views: the objects most visible
    # in some keyframe, each in that keyframe with its own Gaussians (objects
    # are contiguous in the parameters) inside its observed box + 8 px.
    idm = targets["id"].cpu().numpy()
    H, W = idm.shape[1:]
    cnt = np.stack([(idm == k).reshape(V, -1).sum(1) for k in range(sc["K"])])  # [K][V]
    order = [k for k in np.argsort(-cnt.max(1)) if k > 0][:args.jobs]
    jobs_desc = []
    for k in order:
        v = int(np.argmax(cnt[k]))
        ys, xs = np.nonzero(idm[v] == k)
        box = (max(int(xs.min()) - 8, 0), max(int(ys.min()) - 8, 0), min(int(xs.max()) + 9, W),
               min(int(ys.max()) + 9, H))
        g = np.flatnonzero(sc["ids"] == k)
        jobs_desc.append(dict(object=int(k), view=v, window=box, first=int(g[0]), gaussians=int(g.size)))
    cams = list(sc["cams"]) + [sc["cams"][j["view"]] for j in jobs_desc]
    segments = [(0, n)] * V + [(j["first"], j["gaussians"]) for j in jobs_desc]
    windows = [(0, 0, W, H)] * V + [j["window"] for j in jobs_desc]
    jobs = [-1] * V + [j["object"] for j in jobs_desc]
    jv = [j["view"] for j in jobs_desc]
    targets = {key: torch.cat([t, t[jv]]).contiguous() for key, t in targets.items()}

    def make(ctx):
        return B.Trainer(p0.clone(), ids, cams, sc["K"], targets, ctx=ctx, segments=segments, windows=windows,
                         jobs=jobs)

    log("autotuning the tile shape")
    best, table = autotune.autotune_tile(make)
    log(f"tile {best}: {table}")
    tr = make(B.Context(tile_w=best[0], tile_h=best[1]))
    g = tr.capture()
    tr.replay(g, args.warmup)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    tr.replay(g, args.steps)   # reads the device status every 100 replays and after the last
    torch.cuda.synchronize()
    dt = time.perf_counter() - t_start
    npairs = tr.check()
    ms = dt * 1e3 / args.steps
    # per-object dual quadrics from the rendered object masks of the 8 views
    # (the whole-scene views only: the mask boxes of every object)
    r1 = B.Rasterizer(sc["cams"], n, sc["K"], ctx=B.Context(tile_w=16, tile_h=16))
    img = r1.forward(tr.params, ids, probs=True, id_map=True)
    Ps = torch.tensor(np.stack([B.camera_matrix(c).reshape(12) for c in sc["cams"]]), dtype=torch.float64,
                      device="cuda")
    wh = torch.tensor([[c["width"], c["height"]] for c in sc["cams"]], dtype=torch.int32, device="cuda")
    ctx = tr.r.ctx
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    boxes, bo, bv = B.id_boxes(ctx, img["id_map"], sc["K"])
    fit = B.fit_dual_quadric(ctx, boxes, bo, bv, Ps, sc["K"], img_wh=wh)
    e1.record()
    torch.cuda.synchronize()
    st = fit["status"].cpu().numpy()
    mu = fit["mu"].cpu().numpy()
    ok = st[1:] == 0
    centre_err = np.linalg.norm(mu[1:][ok] - sc["centres"][ok], axis=1) if ok.any() else np.array([np.nan])
    # pose refinement of the fitted objects by the IoU loss (Eq. (9)), one launch
    torch.cuda.synchronize()
    e2, e3 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e2.record()
    ref = B.refine_quadrics(ctx, boxes, bo, bv, Ps, fit, img_wh=wh)
    e3.record()
    torch.cuda.synchronize()
    rl = ref["loss"].cpu().numpy()[1:][ok]
    n_box = np.bincount(bo.cpu().numpy()[bo.cpu().numpy() >= 0], minlength=sc["K"])[1:][ok]
    mu_r = ref["mu"].cpu().numpy()
    centre_err_r = np.linalg.norm(mu_r[1:][ok] - sc["centres"][ok], axis=1) if ok.any() else np.array([np.nan])
    iou_before = float(np.mean(1 - rl[:, 0] / np.maximum(n_box, 1))) if ok.any() else float("nan")
    iou_after = float(np.mean(1 - rl[:, 1] / np.maximum(n_box, 1))) if ok.any() else float("nan")
    out = {
        "metric": "keyframe training iters/s (8 views x 640x480 + per-object jobs, 1.2M Gaussians, all per step)",
        "value": round(1e3 / ms, 2), "unit": "iters/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "8 ring keyframes 640x480 (r=2 m), 40 objects with log-uniform [1k, 80k] Gaussians "
                               "plus background to 1.2M, K=41, and per-object jobs (an object's own Gaussians in "
                               "its box of one keyframe, binary instance loss); one HIP-graph replay = project/bin + "
                               "sort + render fwd + object loss + render bwd + project bwd + Adam over all views "
                               "and jobs",
                   "n_gaussians": n, "views": V, "jobs": jobs_desc, "pairs": npairs, "tile": f"{best[0]}x{best[1]}",
                   "autotune_ms_per_step": table},
        "quadric_fit": {"objects": int(sc["K"] - 1), "fitted": int(ok.sum()),
                        "mask_boxes_plus_fit_ms": round(e0.elapsed_time(e1), 4),
                        "median_centre_error_m": round(float(np.median(centre_err)), 4)},
        "quadric_refine": {"iterations": B.REFINE_DEFAULTS["iterations"], "ms": round(e2.elapsed_time(e3), 4),
                           "mean_box_iou_before": round(iou_before, 4), "mean_box_iou_after": round(iou_after, 4),
                           "median_centre_error_m": round(float(np.median(centre_err_r)), 4)},
    }
    print(json.dumps(out), flush=True)


def _left_perturb(cam, w, tau):
    """Camera with R' = exp([w]x) R and t' = exp([w]x) t + tau."""
    from scipy.spatial.transform import Rotation
    E = Rotation.from_rotvec(np.asarray(w, np.float64)).as_matrix()
    out = dict(cam)
    out["R"] = E @ np.asarray(cam["R"], np.float64).reshape(3, 3)
    out["t"] = E @ np.asarray(cam["t"], np.float64).reshape(3) + np.asarray(tau, np.float64)
    return out


def _pose_error(cam, ref):
    """Rotation angle (deg) between the two camera rotations and distance (m)
    between the camera centres -R^T t."""
    R, Rr = np.asarray(cam["R"]).reshape(3, 3), np.asarray(ref["R"]).reshape(3, 3)
    ang = np.degrees(np.arccos(np.clip((np.trace(R @ Rr.T) - 1) / 2, -1, 1)))
    c, cr = -R.T @ np.asarray(cam["t"]), -Rr.T @ np.asarray(ref["t"])
    return float(ang), float(np.linalg.norm(c - cr))


def bench_tracking(args):
    """Camera tracking through the rasterizer: the 200k-Gaussian room seen
    from a displaced camera (0.5 deg, 4 cm), the pose optimised against the
    frame rendered from the true pose.  One iteration = project/bin + sort +
    render fwd (loss mode) + object loss + render bwd + pose gradient
    (dqo_pose_backward) + an Adam step on the 6-vector on the host."""
    sc = scenes.slam_view_scene(seed=0, n=args.n)
    n, K = sc["params"].shape[1], sc["K"]
    true_cam = sc["cams"][0]
    p = torch.tensor(sc["params"], dtype=torch.float32, device="cuda")
    ids = torch.tensor(sc["ids"], device="cuda")
    r0 = B.Rasterizer([true_cam], n, K, ctx=B.Context(tile_w=8, tile_h=8))
    t0 = r0.forward(p, ids, probs=True, id_map=True)
    torch.cuda.synchronize()
    targets = dict(color=t0["color"].clone(), depth=t0["depth"].clone(), id=t0["id_map"].clone())
    del r0, t0
    start = _left_perturb(true_cam, [0.006, -0.005, 0.003], [0.03, -0.025, 0.01])
    r = B.Rasterizer([start], n, K, ctx=B.Context(tile_w=8, tile_h=8))
    img = r.frame.new_images(target=targets["id"])
    gi = dict(d_color=torch.empty_like(img["color"]), d_depth=torch.empty_like(img["depth"]),
              d_p_target=torch.empty_like(img["depth"]))
    loss = torch.zeros(4, dtype=torch.float64, device="cuda")
    pose_g = torch.empty(1, 6, dtype=torch.float64, device="cuda")
    lr = np.array([1e-3] * 3 + [4e-3] * 3)
    iters = args.steps

    def run(n_it):
        cam = dict(start)
        m, v = np.zeros(6), np.zeros(6)
        hist = []
        for it in range(1, n_it + 1):
            r.cams[0] = cam                        # a re-sized frame takes its cameras from here
            r.frame.cams[0] = B.make_cameras([cam])[0]
            r.bin(p, ids, grow=True)
            f = r.frame
            f.render_forward(img)
            f.object_loss(img, targets, gi, loss)
            f.render_backward(img, gi)
            f.pose_backward(p, pose_g)
            g = pose_g.cpu().numpy()[0]          # synchronises: the host takes the pose step
            hist.append(float(loss[0].item()))
            m = 0.9 * m + 0.1 * g
            v = 0.999 * v + 0.001 * g * g
            step = -lr * (m / (1 - 0.9 ** it)) / (np.sqrt(v / (1 - 0.999 ** it)) + 1e-12)
            cam = _left_perturb(cam, step[:3], step[3:])
        return cam, hist

    run(args.warmup)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    cam, hist = run(iters)
    dt = time.perf_counter() - t_start
    ms = dt * 1e3 / iters
    e0, e1 = _pose_error(start, true_cam), _pose_error(cam, true_cam)
    out = {
        "metric": "camera tracking iters/s (640x480, 200k Gaussians, pose gradient through the rasterizer)",
        "value": round(1e3 / ms, 2), "unit": "iters/s", "n_gpus": 1, "steps": iters, "warmup": args.warmup,
        "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "room of 200k Gaussians at 640x480 (8x8 tiles), target rendered from the true pose, "
                               "start displaced by 0.5 deg and 4 cm; iteration = project/bin + sort + render fwd + "
                               "object loss + render bwd + pose gradient + host Adam step on (w, tau)",
                   "n_gaussians": n},
        "tracking": {"start_error_deg_m": [round(e0[0], 4), round(e0[1], 4)],
                     "final_error_deg_m": [round(e1[0], 4), round(e1[1], 4)],
                     "loss_first_last": [round(hist[0], 6), round(hist[-1], 6)]},
    }
    print(json.dumps(out), flush=True)


def bench_large(args):
    """1M Gaussians at 1200x680 through the torch.autograd.Function (forward +
    L1 colour/depth loss + backward, FP32), with peak device memory against the
    memory a store-everything backward would add (alpha, transmittance and
    Gaussian index per blended (pixel, Gaussian): 12 bytes each)."""
    sc = scenes.large_view_scene(seed=0)
    n = sc["params"].shape[1]
    ids = torch.tensor(sc["ids"], device="cuda")
    pt = torch.tensor(scenes.perturb(sc["params"], 1), dtype=torch.float32, device="cuda")
    r = B.Rasterizer(sc["cams"], n, sc["K"], ctx=B.Context(tile_w=8, tile_h=8))
    tg = r.forward(pt, ids, n_blend=True)
    torch.cuda.synchronize()
    tC, tD = tg["color"].clone(), tg["depth"].clone()
    n_blend_total = int(tg["n_blend"].long().sum().item())
    del tg
    p = torch.tensor(sc["params"], dtype=torch.float32, device="cuda").requires_grad_(True)

    def it():
        C, D, T, P = B.rasterize(p, ids, r, want_probs=False)
        loss = (C - tC).abs().mean() + (D - tD).abs().mean()
        loss.backward()
        p.grad = None
        return loss

    for _ in range(args.warmup):
        it()
    torch.cuda.synchronize()
    torch.cuda.reset_peak_memory_stats()
    base = torch.cuda.memory_allocated()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        loss = it()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t_start
    peak = torch.cuda.max_memory_allocated()
    rc, st, npairs = r.frame.read_status()
    HW = 1200 * 680
    store_all = n_blend_total * 12
    out = {
        "metric": "fwd+bwd iters/s through torch.autograd.Function @1200x680, 1M Gaussians",
        "value": round(args.steps / dt, 2), "unit": "iters/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(dt * 1e3 / args.steps, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "room generator at 1M Gaussians, ring pose 0, 1200x680, f=600; autograd forward + "
                               "L1 colour + L1 depth + backward with transmittance recomputed per pixel",
                   "n_gaussians": n, "pairs": npairs, "tile": "8x8", "loss": round(float(loss), 6)},
        "memory": {"peak_allocated_bytes": int(peak), "allocated_before_bytes": int(base),
                   "per_pixel_backward_state_bytes": HW * 8,
                   "blended_pixel_gaussian_pairs": n_blend_total,
                   "store_everything_extra_bytes": store_all},
    }
    print(json.dumps(out), flush=True)


LEARNED_MODEL = os.path.join(ROOT, "paper_2503_02223_amd", "data", "learned_init.npz")
HELD_OUT_SEED, VAL_SEED, TRAIN_SEED = 3, 2, 1


def eval_learned(ctx, model_path, n_objects=20, iters=300):
    """Time-to-PSNR of the learned initialization on held-out crops (seeded
    superquadric objects never used in training)."""
    from paper_2503_02223_amd import learned as L
    crops = L.make_crop_set(HELD_OUT_SEED, n_objects)
    net, chan_w, thr = L.load_model(model_path, ctx=ctx)
    recs, summary = L.time_to_psnr(ctx, net, thr, crops, iters=iters)
    if summary["mean_seconds_learned"]:
        summary["speedup_seconds"] = round(summary["mean_seconds_plain"] / summary["mean_seconds_learned"], 3)
        summary["speedup_iters"] = round(iters / max(summary["mean_iters_learned"], 1e-9), 3)
    summary["model"] = os.path.relpath(model_path, ROOT)
    return {k: (round(v, 5) if isinstance(v, float) else v) for k, v in summary.items()}, recs


def bench_learned(args):
    """Learned initialization end to end: 128x128 object crops, labels from the
    plain optimizer (300 iterations per crop, 16 crops per launch), network
    training with the MFMA kernels, fallback threshold on a validation split,
    then time-to-PSNR on 20 held-out objects."""
    from paper_2503_02223_amd import learned as L
    t0 = time.time()
    crops_tr = L.make_crop_set(TRAIN_SEED, args.n_train, workers=args.workers)
    crops_val = L.make_crop_set(VAL_SEED, args.n_val, workers=args.workers)
    t_data = time.time() - t0
    log(f"crops: {crops_tr.shape[0]} train, {crops_val.shape[0]} validation in {t_data:.1f} s")
    torch.cuda.init()
    ctx = L.crop_context()
    t0 = time.time()
    rg, lab = L.generate_labels(ctx, crops_tr, iters=args.label_iters, log=log)
    t_labels = time.time() - t0
    chan_w = L.channel_weights(crops_tr, lab)
    log(f"labels in {t_labels:.1f} s; channel weights {chan_w}")
    net = L.Net(ctx, seed=0)
    hist, t_train = L.train_net(net, rg, lab, chan_w, steps=args.train_steps, batch=args.batch, lr=args.lr,
                                log=log)
    thr = L.choose_threshold(net, torch.tensor(crops_val, device="cuda"))
    os.makedirs(os.path.dirname(args.save), exist_ok=True)
    L.save_model(args.save, net, chan_w, thr, dict(n_train=args.n_train, label_iters=args.label_iters,
                                                   train_steps=args.train_steps, batch=args.batch, lr=args.lr))
    log(f"model saved to {args.save}; threshold {thr:.4f}")
    del rg, lab
    summary, recs = eval_learned(ctx, args.save, n_objects=args.n_test, iters=args.label_iters)
    for r in recs:
        log(json.dumps(r))
    out = {
        "metric": "time-to-PSNR learned vs plain init", "value": summary.get("mean_seconds_learned"), "unit": "s",
        "n_gpus": 1, "higher_is_better": False, "vs_baseline": None, "dtype": "bf16 net / f32 rasterizer",
        "data": "synthetic",
        "config": {"workload": f"{args.n_train} training + {args.n_val} validation + {args.n_test} held-out "
                               "superquadric crops 128x128 (f=110); labels = Gaussians after "
                               f"{args.label_iters} plain-optimizer iterations; target = plain PSNR after "
                               f"{args.label_iters} iterations",
                   "train_steps": args.train_steps, "batch": args.batch},
        "learned_init": summary,
        "timing_s": {"crops_cpu": round(t_data, 2), "labels_gpu": round(t_labels, 2), "train_gpu": round(t_train, 2)},
        "train_loss": hist,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="slam", choices=["slam", "keyframes", "large", "learned-init", "tracking"],
                    help="slam: 200k Gaussians at 640x480 (default, the headline line); keyframes: 8 views over "
                         "1.2M Gaussians in a HIP graph; large: 1M at 1200x680 through autograd; learned-init: "
                         "train the initialization network and measure time-to-PSNR; tracking: camera pose "
                         "optimisation through the rasterizer on the 200k view")
    ap.add_argument("--n-train", type=int, default=16000)
    ap.add_argument("--n-val", type=int, default=256)
    ap.add_argument("--n-test", type=int, default=20)
    ap.add_argument("--label-iters", type=int, default=300)
    ap.add_argument("--train-steps", type=int, default=12000)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--save", default=os.path.join(tempfile.gettempdir(), "dqo_learned_init.npz"),
                    help="where the learned-init workload saves the trained model")
    ap.add_argument("--no-learned", action="store_true", help="skip the time-to-PSNR part of the default run")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=200_000)
    ap.add_argument("--jobs", type=int, default=8, help="per-object jobs beside the 8 keyframes (at most 8)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--event-every", type=int, default=25,
                    help="time the render backward with HIP events on every N-th timed step (default 25)")
    ap.add_argument("--no-graph", action="store_true",
                    help="issue every timed step eagerly instead of replaying the captured step")
    ap.add_argument("--cpu-pixels", type=int, default=49152)
    ap.add_argument("--tile", default="8x8", help="pixel tile WxH (8x8, 16x8, 16x16, 32x8, 8x32)")
    ap.add_argument("--depth-order", default="auto", choices=["auto", "global", "tile"],
                    help="how each tile's pairs are put in depth order (dqo_depth_order)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 256 MiB device-to-device copy (scale for the HBM byte counters)")
    args = ap.parse_args()
    tw, th = (int(x) for x in args.tile.split("x"))
    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 4, "copy_bytes_written": dst.numel() * 4}))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the multi-GPU (view-sharded) path is designed but not built; "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.workload == "learned-init":
        return bench_learned(args)  # generates its crops before the GPU is touched
    torch.cuda.init()
    if args.workload == "keyframes":
        return bench_keyframes(args)
    if args.workload == "large":
        return bench_large(args)
    if args.workload == "tracking":
        return bench_tracking(args)
    log("building workload")
    sc, p, ids, targets = build_workload(n=args.n)
    order = {"auto": B.DEPTH_ORDER_AUTO, "global": B.DEPTH_ORDER_GLOBAL, "tile": B.DEPTH_ORDER_TILE}[args.depth_order]
    tr = B.Trainer(p, ids, sc["cams"], sc["K"], targets, ctx=B.Context(tile_w=tw, tile_h=th, depth_order=order))
    log(f"pair capacity {tr.r.frame.capacity}")
    for _ in range(args.warmup):
        tr.step()
    torch.cuda.synchronize()
    tr.check()
    # The step is captured once in a HIP graph (every kernel of it, on one
    # stream): replaying it costs one launch instead of the ~20 kernel
    # launches and 6 library calls that the host otherwise issues per step
    # (about 0.4 ms of host time, as long as the step itself).  The capture
    # runs no step.  Timed region: K whole steps; every --event-every-th one
    # runs eagerly with HIP events around the render backward on the stream it
    # is launched on (torch's current stream), the others replay the graph.
    graph = tr.capture() if not args.no_graph else None
    stream = torch.cuda.current_stream()
    every = max(1, args.event_every)
    sampled = list(range(0, args.steps, every))
    ev = {k: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for k in sampled}
    f = tr.r.frame
    orig = f.render_backward
    state = {"k": None}

    def timed_bwd(img, grads, s=None):
        a, b = ev[state["k"]]
        a.record(stream)
        orig(img, grads, s)
        b.record(stream)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        if k in ev or graph is None:
            state["k"] = k
            f.render_backward = timed_bwd if k in ev else orig
            tr.step()
            f.render_backward = orig
        else:
            graph.replay()
            tr.step_count += 1
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    npairs = tr.check()
    bwd_ms = float(np.mean([a.elapsed_time(b) for a, b in ev.values()]))
    ms = dt * 1e3 / args.steps
    loss = tr.loss.cpu().numpy().tolist()
    E, Bn = backward_work(tr)
    Wp = written_pairs(tr)
    t = bwd_ms * 1e-3
    alg_bytes = BYTES_PER_PAIR * npairs + BYTES_PER_PIXEL * 640 * 480 + BYTES_PER_WRITTEN * Wp
    flops = FLOP_PER_EXAMINED * E
    # roofline fraction = max(bytes / BW, flops / F, exps / E) / measured time
    t_hbm = alg_bytes / (MI355X_HBM_GBS * 1e9)
    t_flop = flops / (MI355X_FP32_VECTOR_TFLOPS * 1e12)
    t_exp = E / MI355X_EXP_PER_S
    # 64-pixel tiles: the segmented instantiation (no instance channels) up to 8192 tiles
    seg = -(-640 // tw) * -(-480 // th) <= 8192
    kernel = (f"render_backward_wave_kernel<float,{tw},{th},false,{'true' if seg else 'false'}>" if tw * th == 64
              else f"render_backward_kernel<float,{tw},{th}>")
    if t_hbm >= max(t_flop, t_exp):
        roof = dict(bound="hbm", achieved=round(alg_bytes / t / 1e9, 1), peak=MI355X_HBM_GBS, unit="GB/s")
    else:
        roof = dict(bound="alu", achieved=round(flops / t / 1e12, 3), peak=MI355X_FP32_VECTOR_TFLOPS,
                    unit="TFLOP/s")
    roof.update(frac=round(max(t_hbm, t_flop, t_exp) / t, 4), traffic=measured_traffic(), kernel=kernel,
                avg_ms=round(bwd_ms, 4), alg_bytes=int(alg_bytes), flops=int(flops),
                bytes_frac=round(t_hbm / t, 4), flop_frac=round(t_flop / t, 4), exp_frac=round(t_exp / t, 4),
                pairs=npairs, examined_pixel_pairs=E, blended_pixel_pairs=Bn, written_pairs=Wp,
                flop_per_examined=FLOP_PER_EXAMINED)
    cpu = None
    if not args.no_cpu:
        log("timing the CPU oracle on a bounded sample")
        cpu = cpu_baseline(sc, n_pix=args.cpu_pixels)
        log("timing the 2k-Gaussian scene on the GPU and the oracle")
        cpu["small_scene"] = small_scene_comparison()
    learned = None
    if not args.no_learned and os.path.exists(LEARNED_MODEL):
        log("time-to-PSNR of the learned initialization on 20 held-out objects")
        from paper_2503_02223_amd import learned as L
        learned, _ = eval_learned(L.crop_context(), LEARNED_MODEL)
    out = {
        "metric": METRIC, "value": round(1e3 / ms, 2), "unit": "iters/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "room of 200k Gaussians (20 object blobs + 30% background, K=21) at 640x480, "
                               "f=600; step = project/bin + sort + render fwd + object loss (L1 rgb + L1 depth + "
                               "object CE) + render bwd + project bwd + Adam, replayed as one HIP graph",
                   "n_gaussians": args.n, "width": 640, "height": 480, "K": sc["K"], "pairs": npairs,
                   "tile": args.tile, "graph": graph is not None, "loss": [round(x, 6) for x in loss]},
        "roofline": roof, "cpu_baseline": cpu, "learned_init": learned,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
