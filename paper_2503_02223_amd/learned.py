"""Learned initialization: the network, crop initialization, label generation
by the plain optimizer, training and the time-to-PSNR comparison.

Every step runs in libdqo's kernels (include/dqo_learned.h and dqo.h); this
module marshals arguments, owns device buffers and sequences the calls.
"""
from __future__ import annotations

import ctypes
import math
import time
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

from . import binding as B
from . import crops as CR

NET_OUT = 6
NET_CHANNELS = (5, 32, 64, 64, 6)


def net_layout() -> B.NetLayout:
    lay = B.NetLayout()
    rc = B.lib().dqo_net_layout_get(ctypes.byref(lay))
    if rc != B.OK:
        raise B.DqoError(rc, "dqo_net_layout_get failed")
    return lay


def pack_layers(layers, lay: Optional[B.NetLayout] = None) -> np.ndarray:
    """[(w (cout, cin, 3, 3), b (cout,))] -> flat theta (float32) in the
    library's [cout_pad][9][cin_pad] + bias layout, zero padded."""
    lay = lay or net_layout()
    theta = np.zeros(int(lay.n_params), np.float32)
    for l, (w, b) in enumerate(layers):
        co, ci = w.shape[0], w.shape[1]
        cop, cip = lay.cout_pad[l], lay.cin_pad[l]
        blk = np.zeros((cop, 9, cip), np.float32)
        blk[:co, :, :ci] = np.asarray(w, np.float32).reshape(co, ci, 9).transpose(0, 2, 1)
        theta[lay.w_offset[l]:lay.w_offset[l] + blk.size] = blk.ravel()
        theta[lay.b_offset[l]:lay.b_offset[l] + co] = np.asarray(b, np.float32)
    return theta


def unpack_theta(theta, lay: Optional[B.NetLayout] = None):
    """Inverse of pack_layers (the logical channels only)."""
    lay = lay or net_layout()
    th = np.asarray(theta, np.float64)
    layers = []
    for l in range(B.NET_LAYERS):
        co, ci, cop, cip = lay.cout[l], lay.cin[l], lay.cout_pad[l], lay.cin_pad[l]
        blk = th[lay.w_offset[l]:lay.w_offset[l] + cop * 9 * cip].reshape(cop, 9, cip)
        w = blk[:co, :, :ci].transpose(0, 2, 1).reshape(co, ci, 3, 3)
        layers.append((w, th[lay.b_offset[l]:lay.b_offset[l] + co].copy()))
    return layers


def he_init(seed):
    """He-normal weights (std sqrt(2 / (9 cin))) and zero biases, seeded."""
    rng = np.random.default_rng(seed)
    return [(rng.normal(0.0, np.sqrt(2.0 / (9 * ci)), size=(co, ci, 3, 3)), np.zeros(co))
            for ci, co in zip(NET_CHANNELS[:-1], NET_CHANNELS[1:])]


def crop_context() -> B.Context:
    """Rasterizer context of the 128x128 crops: 8x8 tiles (256 single-wave
    workgroups per crop instead of 64 four-wave ones at 16x16; the plain
    optimizer's 300 iterations on a held-out crop measured 0.101 -> 0.068 s)."""
    return B.Context(tile_w=8, tile_h=8)


class Net:
    """The network's parameters (FP32 master copy + BF16 packed copies), Adam
    state and per-batch-shape workspaces, all in device memory."""

    def __init__(self, ctx: Optional[B.Context] = None, theta: Optional[np.ndarray] = None, seed=0, device="cuda"):
        self.ctx = ctx or crop_context()
        self.lay = net_layout()
        self.device = torch.device(device)
        th = pack_layers(he_init(seed), self.lay) if theta is None else np.asarray(theta, np.float32)
        assert th.size == self.lay.n_params
        self.theta = torch.tensor(th, device=self.device)
        self.grad = torch.zeros_like(self.theta)
        self.m = torch.zeros_like(self.theta)
        self.v = torch.zeros_like(self.theta)
        self.d_step = torch.zeros(1, dtype=torch.int64, device=self.device)
        self.wf = torch.empty(int(self.lay.w_elems), dtype=torch.int16, device=self.device)
        self.wt = torch.empty_like(self.wf)
        self.loss = torch.zeros(2, dtype=torch.float64, device=self.device)
        self._ws: Dict[tuple, torch.Tensor] = {}
        self.pack()

    def workspace(self, Bn, H, W):
        key = (Bn, H, W)
        if key not in self._ws:
            nb = ctypes.c_int64()
            rc = B.lib().dqo_net_workspace_size(Bn, H, W, ctypes.byref(nb))
            if rc != B.OK:
                raise B.DqoError(rc, f"dqo_net_workspace_size({Bn}, {H}, {W}) rejected")
            self._ws[key] = torch.empty(int(nb.value), dtype=torch.uint8, device=self.device)
        return self._ws[key]

    def pack(self, stream=None):
        self.ctx.check(B.lib().dqo_net_pack(self.ctx.h, B._ptr(self.theta), B._ptr(self.wf), B._ptr(self.wt),
                                            B._stream(stream)))

    def forward(self, rgbdm: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        Bn, _, H, W = rgbdm.shape
        if out is None:
            out = torch.empty(Bn, NET_OUT, H, W, dtype=torch.float32, device=self.device)
        self.ctx.check(B.lib().dqo_net_forward(self.ctx.h, Bn, H, W, B._ptr(rgbdm), B._ptr(self.wf),
                                               B._ptr(self.theta), B._ptr(self.workspace(Bn, H, W)), B._ptr(out),
                                               B._stream(stream)))
        return out

    def loss_backward(self, rgbdm, out, labels, chan_w, stream=None):
        """Loss of the last forward (into self.loss) and dL/dtheta (into self.grad)."""
        Bn, _, H, W = rgbdm.shape
        ws = self.workspace(Bn, H, W)
        cw = (ctypes.c_double * 5)(*[float(x) for x in chan_w])
        self.ctx.check(B.lib().dqo_net_loss(self.ctx.h, Bn, H, W, B._ptr(rgbdm), B._ptr(out), B._ptr(labels), cw,
                                            B._ptr(self.loss), B._ptr(ws), B._stream(stream)))
        self.ctx.check(B.lib().dqo_net_backward(self.ctx.h, Bn, H, W, B._ptr(self.wt), B._ptr(ws),
                                                B._ptr(self.grad), B._stream(stream)))

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        self.ctx.check(B.lib().dqo_adam_flat(self.ctx.h, B._ptr(self.theta), B._ptr(self.grad), B._ptr(self.m),
                                             B._ptr(self.v), int(self.theta.numel()), float(lr), beta1, beta2, eps,
                                             B._ptr(self.d_step), B._stream(stream)))
        self.pack(stream)

    def train_step(self, rgbdm, labels, chan_w, lr, out=None, stream=None):
        out = self.forward(rgbdm, out, stream)
        self.loss_backward(rgbdm, out, labels, chan_w, stream)
        self.adam(lr, stream=stream)
        return out

    def fallback(self, rgbdm, out, threshold, stream=None):
        Bn, _, H, W = rgbdm.shape
        use = torch.empty(Bn, dtype=torch.int32, device=self.device)
        mean = torch.empty(Bn, dtype=torch.float32, device=self.device)
        self.ctx.check(B.lib().dqo_net_fallback(self.ctx.h, Bn, H, W, B._ptr(rgbdm), B._ptr(out), float(threshold),
                                                B._ptr(use), B._ptr(mean), B._stream(stream)))
        return use, mean


# ---------------------------------------------------------------- crops
def valid_counts(rgbdm_np: np.ndarray) -> np.ndarray:
    """Valid pixels per crop (mask > 1/2 and depth > 0), counted on the host
    with the rule the kernels use."""
    r = np.asarray(rgbdm_np)
    return ((r[:, 4] > 0.5) & (r[:, 3] > 0)).reshape(r.shape[0], -1).sum(1).astype(np.int64)


def init_gaussians(ctx, rgbdm: torch.Tensor, cams: Sequence[dict], offsets: np.ndarray,
                   pred: Optional[torch.Tensor] = None, use_pred: Optional[torch.Tensor] = None,
                   params: Optional[torch.Tensor] = None, ids: Optional[torch.Tensor] = None, obj_id=0,
                   stream=None):
    """Gaussians of the crops (one per valid pixel), plain or learned; see
    dqo_init_gaussians.  offsets: host int64 [B + 1]."""
    Bn, _, H, W = rgbdm.shape
    n = int(offsets[-1])
    dev = rgbdm.device
    if params is None:
        params = torch.empty(B.NUM_PARAMS, n, dtype=torch.float32, device=dev)
    if ids is None:
        ids = torch.empty(n, dtype=torch.int32, device=dev)
    off = torch.tensor(np.asarray(offsets, np.int64), device=dev)
    ctx.check(B.lib().dqo_init_gaussians(ctx.h, Bn, H, W, B._ptr(rgbdm), B.make_cameras(cams), B._ptr(off),
                                         B._ptr(pred), B._ptr(use_pred), n, B._ptr(params), B._ptr(ids), obj_id,
                                         B._stream(stream)))
    return params, ids, off


def init_labels(ctx, rgbdm, cams, offsets_dev, params, labels=None, stream=None):
    Bn, _, H, W = rgbdm.shape
    if labels is None:
        labels = torch.empty(Bn, 5, H, W, dtype=torch.float32, device=rgbdm.device)
    ctx.check(B.lib().dqo_init_labels(ctx.h, Bn, H, W, B._ptr(rgbdm), B.make_cameras(cams), B._ptr(offsets_dev),
                                      B._ptr(params), int(params.shape[1]), B._ptr(labels), B._stream(stream)))
    return labels


def masked_psnr(ctx, color, rgbdm, out=None, stream=None):
    V, _, H, W = color.shape
    if out is None:
        out = torch.empty(V, dtype=torch.float64, device=color.device)
    ctx.check(B.lib().dqo_masked_psnr(ctx.h, V, H, W, B._ptr(color), B._ptr(rgbdm), B._ptr(out), B._stream(stream)))
    return out


def crop_targets(rgbdm: torch.Tensor) -> Dict[str, torch.Tensor]:
    """Targets of the plain optimizer: the crop's colour (black background),
    its depth (0 = no depth) and object id 0 at valid pixels, empty (-1)
    elsewhere."""
    valid = (rgbdm[:, 4] > 0.5) & (rgbdm[:, 3] > 0)
    return dict(color=rgbdm[:, 0:3].contiguous(), depth=rgbdm[:, 3].contiguous(),
                id=torch.where(valid, 0, -1).to(torch.int32).contiguous())


def crop_lrs(extent=0.3):
    return B.default_lrs(extent)


class CropOptimizer:
    """The plain optimizer over a batch of crops (at most 16): one view per
    crop with its own Gaussian segment, the whole iteration captured in a HIP
    graph.  Re-initialise with reset() to rerun on new initial Gaussians of
    the same crops."""

    def __init__(self, ctx, rgbdm: torch.Tensor, rgbdm_np: np.ndarray, pred=None, use_pred=None):
        self.ctx = ctx
        self.rgbdm = rgbdm
        Bn = rgbdm.shape[0]
        assert Bn <= B.MAX_VIEWS
        self.cams = [CR.crop_camera(size=rgbdm.shape[3])] * Bn
        counts = valid_counts(rgbdm_np)
        self.offsets = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
        self.n = int(self.offsets[-1])
        params, ids, self.off_dev = init_gaussians(ctx, rgbdm, self.cams, self.offsets, pred, use_pred)
        seg = np.stack([self.offsets[:-1], counts], 1)
        self.tr = B.Trainer(params, ids, self.cams, 1, crop_targets(rgbdm), lrs=crop_lrs(),
                            capacity=max(4096, 48 * self.n), ctx=ctx, segments=seg)
        self.psnr_hist = None
        self.graph = self.tr.capture()  # its warm-up step changes the state: reset below
        self.reset(pred, use_pred)

    def reset(self, pred=None, use_pred=None, stream=None):
        init_gaussians(self.ctx, self.rgbdm, self.cams, self.offsets, pred, use_pred, params=self.tr.params,
                       ids=self.tr.ids, stream=stream)
        self.tr.m.zero_()
        self.tr.v.zero_()
        self.tr.d_step.zero_()

    def run(self, iters, record_psnr=False):
        """iters graph replays; with record_psnr, the masked PSNR of each
        iteration's forward (the state before that iteration's update) goes to
        psnr_hist[k] (device, no synchronisation)."""
        V = self.rgbdm.shape[0]
        if record_psnr:
            self.psnr_hist = torch.zeros(iters + 1, V, dtype=torch.float64, device=self.rgbdm.device)
        for k in range(iters):
            self.graph.replay()
            if record_psnr:
                masked_psnr(self.ctx, self.tr.img["color"], self.rgbdm, out=self.psnr_hist[k])
        return self.psnr_hist

    def final_psnr(self):
        """PSNR of the current Gaussians (one more forward)."""
        r = self.tr.r
        img = r.frame.new_images()
        r.bin(self.tr.params, self.tr.ids, grow=False)
        r.frame.render_forward(img)
        return masked_psnr(self.ctx, img["color"], self.rgbdm)


def label_batch(ctx, rgbdm_np: np.ndarray, iters=300, device="cuda"):
    """Labels of up to 16 crops: plain init, `iters` plain-optimizer
    iterations, then the converged Gaussians read back per pixel."""
    rgbdm = torch.tensor(rgbdm_np, device=device)
    opt = CropOptimizer(ctx, rgbdm, rgbdm_np)
    opt.run(iters)
    labels = init_labels(ctx, rgbdm, opt.cams, opt.off_dev, opt.tr.params)
    return rgbdm, labels, opt


# ---------------------------------------------------------------- pipeline
def make_crop_set(seed, count, workers=1):
    """count crops (numpy, (count, 5, 128, 128) float32), generated in chunks of
    16 with seeds seed * 100003 + chunk, optionally by a pool of processes
    (call it before the GPU is touched: the workers only run numpy)."""
    chunks = [(seed * 100003 + c, min(16, count - 16 * c)) for c in range((count + 15) // 16)]
    if workers > 1 and len(chunks) > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(workers) as pool:
            parts = pool.starmap(CR.make_crops, chunks)
    else:
        parts = [CR.make_crops(s, c) for s, c in chunks]
    return np.concatenate(parts, 0)


def generate_labels(ctx, crops_np: np.ndarray, iters=300, device="cuda", log=None):
    """Labels of every crop from `iters` plain-optimizer iterations, 16 crops
    per launch.  Returns (rgbdm, labels) as device tensors."""
    n = crops_np.shape[0]
    rgbdm = torch.tensor(crops_np, device=device)
    labels = torch.empty(n, 5, crops_np.shape[2], crops_np.shape[3], dtype=torch.float32, device=device)
    t0 = time.time()
    for s in range(0, n, B.MAX_VIEWS):
        e = min(n, s + B.MAX_VIEWS)
        rg = rgbdm[s:e]
        opt = CropOptimizer(ctx, rg, crops_np[s:e])
        opt.run(iters)
        init_labels(ctx, rg, opt.cams, opt.off_dev, opt.tr.params, labels=labels[s:e])
        opt.tr.check()
        if log and (s // B.MAX_VIEWS) % 50 == 0:
            torch.cuda.synchronize()
            log(f"labels {e}/{n} ({time.time() - t0:.1f} s)")
    torch.cuda.synchronize()
    return rgbdm, labels


def channel_weights(crops_np, labels: torch.Tensor):
    """1 / variance of each label channel over the valid pixels."""
    ok = torch.tensor((crops_np[:, 4] > 0.5) & (crops_np[:, 3] > 0), device=labels.device)
    w = []
    for c in range(5):
        v = labels[:, c][ok]
        w.append(float(1.0 / max(v.var().item(), 1e-6)))
    return w


def train_net(net: Net, rgbdm, labels, chan_w, steps=3000, batch=32, lr=2e-3, seed=0, log=None):
    """Adam on random batches; the learning rate decays by cosine to 5% of lr."""
    rng = np.random.default_rng(seed)
    n = rgbdm.shape[0]
    xb = torch.empty((batch,) + tuple(rgbdm.shape[1:]), dtype=torch.float32, device=rgbdm.device)
    lb = torch.empty((batch,) + tuple(labels.shape[1:]), dtype=torch.float32, device=rgbdm.device)
    out = torch.empty(batch, NET_OUT, rgbdm.shape[2], rgbdm.shape[3], dtype=torch.float32, device=rgbdm.device)
    hist = []
    t0 = time.time()
    for it in range(steps):
        idx = torch.tensor(rng.choice(n, batch, replace=False), device=rgbdm.device)
        torch.index_select(rgbdm, 0, idx, out=xb)
        torch.index_select(labels, 0, idx, out=lb)
        cur = lr * (0.05 + 0.95 * 0.5 * (1 + math.cos(math.pi * it / max(1, steps))))
        net.train_step(xb, lb, chan_w, cur, out=out)
        if it % 250 == 0 or it == steps - 1:
            hist.append((it, float(net.loss[0].item()), float(net.loss[1].item())))
            if log:
                log(f"train step {it}: loss {hist[-1][1]:.4f} fit {hist[-1][2]:.4f} ({time.time() - t0:.1f} s)")
    torch.cuda.synchronize()
    return hist, time.time() - t0


def predict(net: Net, rgbdm, batch=32):
    outs = []
    for s in range(0, rgbdm.shape[0], batch):
        outs.append(net.forward(rgbdm[s:s + batch].contiguous()))
    return torch.cat(outs, 0)


def choose_threshold(net: Net, rgbdm_val, quantile=0.95):
    """Fallback threshold: the given quantile of the validation crops' mean
    predicted log-error."""
    out = predict(net, rgbdm_val)
    _, mean = net.fallback(rgbdm_val, out, float("inf"))
    return float(np.quantile(mean.cpu().numpy(), quantile))


def save_model(path, net: Net, chan_w, threshold, meta: dict):
    np.savez(path, theta=net.theta.cpu().numpy(), chan_w=np.asarray(chan_w, np.float64),
             threshold=np.float64(threshold), meta=np.array(repr(meta)))


def load_model(path, ctx=None, device="cuda"):
    z = np.load(path, allow_pickle=False)
    net = Net(ctx=ctx, theta=z["theta"], device=device)
    return net, [float(x) for x in z["chan_w"]], float(z["threshold"])


def _elapsed(fn):
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s.record()
    fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) * 1e-3


def time_to_psnr(ctx, net: Net, threshold, crops_np: np.ndarray, iters=300, device="cuda", max_factor=2):
    """Per held-out crop: the plain method's PSNR after `iters` iterations is
    the target; the learned initialization (network inference, fallback
    decision, Gaussian initialization) then runs the same optimizer until it
    reaches that PSNR, for at most max_factor * iters iterations.  Returns
    per-crop records and the means over all crops (a crop that never reaches
    the target counts with max_factor * iters iterations and their time)."""
    recs = []
    for i in range(crops_np.shape[0]):
        c_np = crops_np[i:i + 1]
        rg = torch.tensor(c_np, device=device)
        opt = CropOptimizer(ctx, rg, c_np)
        # plain: target PSNR and its time
        t_plain = _elapsed(lambda: (opt.reset(), opt.run(iters)))
        target = float(opt.final_psnr().item())
        # learned: inference + decision + init, then iterations until the target
        pred = torch.empty(1, NET_OUT, rg.shape[2], rg.shape[3], dtype=torch.float32, device=device)
        use = torch.empty(1, dtype=torch.int32, device=device)

        def start():
            net.forward(rg, out=pred)
            u, _ = net.fallback(rg, pred, threshold)
            use.copy_(u)
            opt.reset(pred, use)

        start()
        cap = max_factor * iters
        hist = opt.run(cap, record_psnr=True).cpu().numpy()[:, 0]
        fin = float(opt.final_psnr().item())
        psnr = np.concatenate([hist[:cap], [fin]])  # psnr[k] = PSNR after k updates
        hit = np.nonzero(psnr >= target)[0]
        reached = bool(hit.size)
        k = int(hit[0]) if reached else cap
        init_psnr = float(hist[0])
        t_learned = _elapsed(lambda: (start(), opt.run(k)))
        opt.reset()
        plain_init_psnr = float(opt.final_psnr().item())
        recs.append(dict(target_psnr=target, plain_init_psnr=plain_init_psnr, learned_init_psnr=init_psnr,
                         used_prediction=int(use.item()), reached=reached, iters_learned=k,
                         seconds_learned=t_learned, iters_plain=iters, seconds_plain=t_plain))
    summary = dict(objects=len(recs), reached=int(sum(r["reached"] for r in recs)),
                   reached_within_plain_iters=int(sum(r["reached"] and r["iters_learned"] <= iters for r in recs)),
                   fallback_rate=float(np.mean([1 - r["used_prediction"] for r in recs])),
                   mean_iters_learned=float(np.mean([r["iters_learned"] for r in recs])),
                   median_iters_learned=float(np.median([r["iters_learned"] for r in recs])),
                   mean_seconds_learned=float(np.mean([r["seconds_learned"] for r in recs])),
                   mean_seconds_plain=float(np.mean([r["seconds_plain"] for r in recs])),
                   iters_plain=iters,
                   mean_target_psnr=float(np.mean([r["target_psnr"] for r in recs])),
                   mean_plain_init_psnr=float(np.mean([r["plain_init_psnr"] for r in recs])),
                   mean_learned_init_psnr=float(np.mean([r["learned_init_psnr"] for r in recs])))
    return recs, summary
