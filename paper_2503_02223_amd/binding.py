"""Thin ctypes binding of libdqo (include/dqo.h).

Argument marshalling only: every step of the path runs in the HIP kernels of
libdqo.so; torch supplies device memory and the current stream.  Loading
fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libdqo.so")

MAX_VIEWS = 16
MAX_K = 64
NUM_PARAMS = 14
SPLAT_WORDS = 16  # values per splat record in the state buffer (dqo_buf DQO_BUF_SPLATS)
OK, EINVAL, ECAPACITY, ENONFINITE, EDEGENERATE, EHIP, EINTERNAL = 0, -1, -2, -3, -4, -5, -6
F32, F64 = 0, 1
STATUS_OVERFLOW, STATUS_NONFINITE, STATUS_TIMEOUT = 1, 2, 4
BUF_NAMES = ["splats", "rects", "counts", "offsets", "depth_keys", "depth_order", "pair_keys", "pair_vals",
             "ranges", "partials", "control", "scratch"]

EXPORTED = ["dqo_config_default", "dqo_ctx_create", "dqo_ctx_destroy", "dqo_last_error", "dqo_status_string",
            "dqo_version", "dqo_state_layout", "dqo_state_init", "dqo_read_status", "dqo_clear_status",
            "dqo_project_cull_bin", "dqo_sort", "dqo_render_forward", "dqo_object_loss", "dqo_render_backward",
            "dqo_project_backward", "dqo_project_backward_adam", "dqo_pose_backward", "dqo_adam_step", "dqo_adam_step_counted", "dqo_fit_dual_quadric",
            "dqo_id_boxes", "dqo_incremental_masks", "dqo_densify", "dqo_quadric_iou_grad",
            "dqo_refine_quadrics", "dqo_associate", "dqo_quadric_distance", "dqo_associate_decide",
            "dqo_object_loss_noalloc"]
# include/dqo_learned.h
EXPORTED_LEARNED = ["dqo_net_layout_get", "dqo_net_workspace_size", "dqo_net_pack", "dqo_net_forward", "dqo_net_loss",
                    "dqo_net_backward", "dqo_adam_flat", "dqo_init_gaussians", "dqo_init_labels", "dqo_net_fallback",
                    "dqo_masked_psnr"]
NET_LAYERS = 4


class NetLayout(ctypes.Structure):
    _fields_ = [("cin", ctypes.c_int32 * NET_LAYERS), ("cout", ctypes.c_int32 * NET_LAYERS),
                ("cin_pad", ctypes.c_int32 * NET_LAYERS), ("cout_pad", ctypes.c_int32 * NET_LAYERS),
                ("w_offset", ctypes.c_int64 * NET_LAYERS), ("b_offset", ctypes.c_int64 * NET_LAYERS),
                ("wk_offset", ctypes.c_int64 * NET_LAYERS), ("n_params", ctypes.c_int64), ("w_elems", ctypes.c_int64)]


class Config(ctypes.Structure):
    _fields_ = [("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32), ("z_near", ctypes.c_double),
                ("dilation", ctypes.c_double), ("q_max", ctypes.c_double), ("alpha_min", ctypes.c_double),
                ("alpha_max", ctypes.c_double), ("t_min", ctypes.c_double), ("bg", ctypes.c_double * 3),
                ("depth_order", ctypes.c_int32), ("tile_sort_lds", ctypes.c_int32)]

DEPTH_ORDER_AUTO, DEPTH_ORDER_GLOBAL, DEPTH_ORDER_TILE = 0, 1, 2


class Camera(ctypes.Structure):
    _fields_ = [("R", ctypes.c_double * 9), ("t", ctypes.c_double * 3), ("fx", ctypes.c_double),
                ("fy", ctypes.c_double), ("cx", ctypes.c_double), ("cy", ctypes.c_double),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


class FrameDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("n_views", ctypes.c_int32), ("K", ctypes.c_int32),
                ("pair_capacity", ctypes.c_int64), ("dtype", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("segments", ctypes.POINTER(ctypes.c_int64)), ("windows", ctypes.POINTER(ctypes.c_int32)),
                ("jobs", ctypes.POINTER(ctypes.c_int32))]


class Layout(ctypes.Structure):
    _fields_ = [("offset", ctypes.c_int64 * 12), ("bytes", ctypes.c_int64 * 12), ("total", ctypes.c_int64),
                ("tiles_x", ctypes.c_int32), ("tiles_y", ctypes.c_int32), ("pair_key_bits", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class Images(ctypes.Structure):
    _fields_ = [("color", ctypes.c_void_p), ("depth", ctypes.c_void_p), ("t_final", ctypes.c_void_p),
                ("last", ctypes.c_void_p), ("probs", ctypes.c_void_p), ("id_map", ctypes.c_void_p),
                ("target", ctypes.c_void_p), ("p_target", ctypes.c_void_p), ("n_blend", ctypes.c_void_p)]


class ImageGrads(ctypes.Structure):
    _fields_ = [("d_color", ctypes.c_void_p), ("d_depth", ctypes.c_void_p), ("d_t_final", ctypes.c_void_p),
                ("d_probs", ctypes.c_void_p), ("d_p_target", ctypes.c_void_p)]


class Targets(ctypes.Structure):
    _fields_ = [("color", ctypes.c_void_p), ("depth", ctypes.c_void_p), ("id", ctypes.c_void_p)]


class LossWeights(ctypes.Structure):
    _fields_ = [("w_rgb", ctypes.c_double), ("w_depth", ctypes.c_double), ("lam", ctypes.c_double),
                ("ce_eps", ctypes.c_double)]


class IncrementCfg(ctypes.Structure):
    _fields_ = [("theta_alpha", ctypes.c_double), ("theta_d", ctypes.c_double), ("theta_c", ctypes.c_double),
                ("og_opacity", ctypes.c_double), ("tg_opacity", ctypes.c_double)]


# thresholds of Eq. (7) (theta_alpha is not stated in the paper) and the OG / TG opacities
INCREMENT_DEFAULTS = dict(theta_alpha=0.5, theta_d=0.1, theta_c=0.1, og_opacity=0.9, tg_opacity=0.1)


class RefineCfg(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("lr_mu", ctypes.c_double), ("lr_rot", ctypes.c_double),
                ("lr_axes", ctypes.c_double), ("beta1", ctypes.c_double), ("beta2", ctypes.c_double),
                ("eps", ctypes.c_double)]


# Adam on the quadric pose (the paper does not state its optimiser settings)
REFINE_DEFAULTS = dict(iterations=100, lr_mu=0.01, lr_rot=0.01, lr_axes=0.01, beta1=0.9, beta2=0.999, eps=1e-15)


class AdamParams(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_double * NUM_PARAMS), ("beta1", ctypes.c_double), ("beta2", ctypes.c_double),
                ("eps", ctypes.c_double)]


class DqoError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libdqo error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """The loaded libdqo.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBPATH):
        raise RuntimeError(f"{LIBPATH} is missing: build it with paper_2503_02223_amd/build.py "
                           "(or __graft_entry__.build()); there is no fallback path")
    L = ctypes.CDLL(LIBPATH)
    P, vp, i32, i64, d = ctypes.POINTER, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    ctx = vp
    L.dqo_config_default.argtypes = [P(Config)]
    L.dqo_config_default.restype = None
    L.dqo_ctx_create.argtypes = [P(vp), P(Config)]
    L.dqo_ctx_destroy.argtypes = [ctx]
    L.dqo_last_error.argtypes = [ctx]
    L.dqo_last_error.restype = ctypes.c_char_p
    L.dqo_status_string.argtypes = [ctypes.c_int]
    L.dqo_status_string.restype = ctypes.c_char_p
    L.dqo_version.restype = ctypes.c_char_p
    fr = [ctx, P(FrameDesc), P(Camera)]
    L.dqo_state_layout.argtypes = fr + [P(Layout)]
    L.dqo_state_init.argtypes = fr + [vp, vp]
    L.dqo_read_status.argtypes = fr + [vp, P(ctypes.c_uint32), P(i64), vp]
    L.dqo_clear_status.argtypes = fr + [vp, vp]
    L.dqo_project_cull_bin.argtypes = fr + [vp, vp, vp, vp]
    L.dqo_sort.argtypes = fr + [vp, vp]
    L.dqo_render_forward.argtypes = fr + [vp, P(Images), vp]
    L.dqo_object_loss.argtypes = fr + [P(Images), P(Targets), P(LossWeights), vp, P(ImageGrads), vp, vp]
    L.dqo_object_loss_noalloc.argtypes = fr + [P(Images), P(Targets), P(LossWeights), vp, P(ImageGrads), vp]
    L.dqo_render_backward.argtypes = fr + [vp, P(Images), P(ImageGrads), vp]
    L.dqo_project_backward.argtypes = fr + [vp, vp, vp, vp]
    L.dqo_project_backward_adam.argtypes = fr + [vp, vp, vp, vp, P(AdamParams), vp, vp, vp]
    L.dqo_pose_backward.argtypes = fr + [vp, vp, vp, vp]
    L.dqo_adam_step.argtypes = [ctx, i32, vp, vp, vp, vp, i64, P(AdamParams), i64, vp]
    L.dqo_incremental_masks.argtypes = fr + [P(Images), P(Targets), P(IncrementCfg), vp, vp, vp]
    L.dqo_densify.argtypes = fr + [P(Targets), vp, P(IncrementCfg), i64, i64, vp, vp, vp, vp]
    L.dqo_adam_step_counted.argtypes = [ctx, i32, vp, vp, vp, vp, i64, P(AdamParams), vp, vp]
    L.dqo_fit_dual_quadric.argtypes = [ctx, i32, i64, vp, vp, vp, i32, vp, vp, d, vp, vp, vp, vp, vp, vp]
    L.dqo_id_boxes.argtypes = [ctx, vp, i32, i32, i32, i32, vp, vp, vp, vp]
    L.dqo_associate.argtypes = [ctx, i32, vp, vp, vp, i64, vp, vp, i32, vp, vp, d, vp, vp, vp, vp]
    L.dqo_quadric_distance.argtypes = [ctx, i32, vp, vp, vp, i32, vp, vp, vp, d, vp, vp]
    L.dqo_associate_decide.argtypes = [ctx, i64, i32, vp, vp, vp, vp, vp, d, d, d, vp, vp, vp, vp, vp]
    L.dqo_quadric_iou_grad.argtypes = [ctx, i32, i64, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp, vp]
    L.dqo_refine_quadrics.argtypes = [ctx, i32, i64, vp, vp, vp, i32, vp, vp, vp, P(RefineCfg), vp, vp, vp, vp, vp,
                                      vp, vp]
    L.dqo_net_layout_get.argtypes = [P(NetLayout)]
    L.dqo_net_workspace_size.argtypes = [i32, i32, i32, P(i64)]
    L.dqo_net_pack.argtypes = [ctx, vp, vp, vp, vp]
    L.dqo_net_forward.argtypes = [ctx, i32, i32, i32, vp, vp, vp, vp, vp, vp]
    L.dqo_net_loss.argtypes = [ctx, i32, i32, i32, vp, vp, vp, P(d), vp, vp, vp]
    L.dqo_net_backward.argtypes = [ctx, i32, i32, i32, vp, vp, vp, vp]
    L.dqo_adam_flat.argtypes = [ctx, vp, vp, vp, vp, i64, d, d, d, d, vp, vp]
    L.dqo_init_gaussians.argtypes = [ctx, i32, i32, i32, vp, P(Camera), vp, vp, vp, i64, vp, vp, i32, vp]
    L.dqo_init_labels.argtypes = [ctx, i32, i32, i32, vp, P(Camera), vp, vp, i64, vp, vp]
    L.dqo_net_fallback.argtypes = [ctx, i32, i32, i32, vp, vp, d, vp, vp, vp]
    L.dqo_masked_psnr.argtypes = [ctx, i32, i32, i32, vp, vp, vp, vp]
    for f in EXPORTED + EXPORTED_LEARNED:
        if f not in ("dqo_config_default", "dqo_last_error", "dqo_status_string", "dqo_version"):
            getattr(L, f).restype = ctypes.c_int
    _lib = L
    return L


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def default_config(**kw) -> Config:
    c = Config()
    lib().dqo_config_default(ctypes.byref(c))
    for k, v in kw.items():
        if k == "bg":
            for i in range(3):
                c.bg[i] = float(v[i])
        else:
            setattr(c, k, v)
    return c


class Context:
    """A libdqo context (host-side configuration and error text)."""

    def __init__(self, config: Optional[Config] = None, **kw):
        cfg = config if config is not None else default_config(**kw)
        h = ctypes.c_void_p()
        rc = lib().dqo_ctx_create(ctypes.byref(h), ctypes.byref(cfg))
        if rc != OK:
            raise DqoError(rc, "dqo_ctx_create rejected the configuration")
        self.h = h
        self.config = cfg

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.dqo_ctx_destroy(self.h)
            self.h = None

    def check(self, rc):
        if rc != OK:
            raise DqoError(rc, lib().dqo_last_error(self.h).decode())
        return rc


def make_cameras(cams: Sequence[dict]):
    arr = (Camera * len(cams))()
    for i, c in enumerate(cams):
        R = np.asarray(c["R"], np.float64).reshape(9)
        t = np.asarray(c["t"], np.float64).reshape(3)
        for k in range(9):
            arr[i].R[k] = float(R[k])
        for k in range(3):
            arr[i].t[k] = float(t[k])
        arr[i].fx, arr[i].fy, arr[i].cx, arr[i].cy = (float(c[k]) for k in ("fx", "fy", "cx", "cy"))
        arr[i].width, arr[i].height = int(c["width"]), int(c["height"])
    return arr


_TORCH_DT = {F32: torch.float32, F64: torch.float64}


class Frame:
    """Caller-owned device state of one frame of work (n Gaussians, V views)."""

    def __init__(self, ctx: Context, cams: Sequence[dict], n: int, K: int, capacity: int,
                 dtype=torch.float32, device="cuda", segments=None, windows=None, jobs=None):
        self.ctx = ctx
        self.cam_dicts = list(cams)
        self.cams = make_cameras(cams)
        self.dt = F64 if dtype == torch.float64 else F32
        self.tdtype = dtype
        self.device = torch.device(device)
        self.desc = FrameDesc(n=int(n), n_views=len(cams), K=int(K), pair_capacity=int(capacity), dtype=self.dt)
        self.segments = None
        if segments is not None:   # [V][2] (first, count); kept alive with the descriptor
            seg = np.ascontiguousarray(np.asarray(segments, dtype=np.int64).reshape(len(cams), 2))
            self.segments = (ctypes.c_int64 * seg.size)(*seg.ravel().tolist())
            self.desc.segments = ctypes.cast(self.segments, ctypes.POINTER(ctypes.c_int64))
        self.windows = self.jobs = None
        if windows is not None:    # [V][4] (x0, y0, x1, y1) pixel windows
            win = np.ascontiguousarray(np.asarray(windows, dtype=np.int32).reshape(len(cams), 4))
            self.windows = (ctypes.c_int32 * win.size)(*win.ravel().tolist())
            self.desc.windows = ctypes.cast(self.windows, ctypes.POINTER(ctypes.c_int32))
        if jobs is not None:       # [V] object of each per-object job, -1 = whole scene
            jb = np.ascontiguousarray(np.asarray(jobs, dtype=np.int32).reshape(len(cams)))
            self.jobs = (ctypes.c_int32 * jb.size)(*jb.tolist())
            self.desc.jobs = ctypes.cast(self.jobs, ctypes.POINTER(ctypes.c_int32))
        self.layout = Layout()
        ctx.check(lib().dqo_state_layout(ctx.h, ctypes.byref(self.desc), self.cams, ctypes.byref(self.layout)))
        self.state = torch.empty(int(self.layout.total), dtype=torch.uint8, device=self.device)
        ctx.check(lib().dqo_state_init(ctx.h, ctypes.byref(self.desc), self.cams, _ptr(self.state), _stream()))
        self.W, self.H = int(cams[0]["width"]), int(cams[0]["height"])
        self.V = len(cams)
        self.n, self.K, self.capacity = int(n), int(K), int(capacity)

    # -- views on the state buffer (for tests and diagnostics) --
    def buf(self, name: str, dtype=torch.int32, count: Optional[int] = None) -> torch.Tensor:
        i = BUF_NAMES.index(name)
        off, nb = int(self.layout.offset[i]), int(self.layout.bytes[i])
        item = torch.empty((), dtype=dtype).element_size()
        cnt = nb // item if count is None else count
        return self.state[off:off + cnt * item].view(dtype)

    def _fr(self):
        return (self.ctx.h, ctypes.byref(self.desc), self.cams)

    def project_cull_bin(self, params: torch.Tensor, ids: torch.Tensor, stream=None):
        assert params.dtype == self.tdtype and params.shape == (NUM_PARAMS, self.n)
        assert ids.dtype == torch.int32 and ids.shape == (self.n,)
        self.ctx.check(lib().dqo_project_cull_bin(*self._fr(), _ptr(params), _ptr(ids), _ptr(self.state),
                                                  _stream(stream)))

    def sort(self, stream=None):
        self.ctx.check(lib().dqo_sort(*self._fr(), _ptr(self.state), _stream(stream)))

    def read_status(self, stream=None):
        st = ctypes.c_uint32()
        npairs = ctypes.c_int64()
        rc = lib().dqo_read_status(*self._fr(), _ptr(self.state), ctypes.byref(st), ctypes.byref(npairs),
                                   _stream(stream))
        return rc, int(st.value), int(npairs.value)

    def clear_status(self, stream=None):
        self.ctx.check(lib().dqo_clear_status(*self._fr(), _ptr(self.state), _stream(stream)))

    def new_images(self, probs=False, id_map=False, target: Optional[torch.Tensor] = None,
                   n_blend=False) -> Dict[str, torch.Tensor]:
        V, H, W, dt, dev = self.V, self.H, self.W, self.tdtype, self.device
        img = dict(color=torch.empty(V, 3, H, W, dtype=dt, device=dev), depth=torch.empty(V, H, W, dtype=dt, device=dev),
                   t_final=torch.empty(V, H, W, dtype=dt, device=dev),
                   last=torch.empty(V, H, W, dtype=torch.int32, device=dev))
        if probs:
            img["probs"] = torch.empty(V, self.K, H, W, dtype=dt, device=dev)
        if id_map:
            img["id_map"] = torch.empty(V, H, W, dtype=torch.int32, device=dev)
        if target is not None:
            img["target"] = target
            img["p_target"] = torch.empty(V, H, W, dtype=dt, device=dev)
        if n_blend:
            img["n_blend"] = torch.empty(V, H, W, dtype=torch.int32, device=dev)
        return img

    @staticmethod
    def _images(img: Dict[str, torch.Tensor]) -> Images:
        return Images(*(_ptr(img.get(k)) for k in ("color", "depth", "t_final", "last", "probs", "id_map",
                                                   "target", "p_target", "n_blend")))

    def render_forward(self, img: Dict[str, torch.Tensor], stream=None):
        s = Frame._images(img)
        self.ctx.check(lib().dqo_render_forward(*self._fr(), _ptr(self.state), ctypes.byref(s), _stream(stream)))

    def object_loss(self, img, tgt: Dict[str, torch.Tensor], grads: Optional[Dict[str, torch.Tensor]], loss: torch.Tensor,
                    w_rgb=1.0, w_depth=1.0, lam=1.0, ce_eps=1e-6, stream=None):
        s = Frame._images(img)
        t = Targets(_ptr(tgt["color"]), _ptr(tgt["depth"]), _ptr(tgt.get("id")))
        w = LossWeights(w_rgb, w_depth, lam, ce_eps)
        g = None
        if grads is not None:
            g = ctypes.byref(ImageGrads(*(_ptr(grads.get(k)) for k in ("d_color", "d_depth", "d_t_final", "d_probs",
                                                                      "d_p_target"))))
        self.ctx.check(lib().dqo_object_loss(*self._fr(), ctypes.byref(s), ctypes.byref(t), ctypes.byref(w),
                                             _ptr(loss), g, _ptr(self.state), _stream(stream)))

    def render_backward(self, img, grads: Dict[str, torch.Tensor], stream=None):
        s = Frame._images(img)
        g = ImageGrads(*(_ptr(grads.get(k)) for k in ("d_color", "d_depth", "d_t_final", "d_probs", "d_p_target")))
        self.ctx.check(lib().dqo_render_backward(*self._fr(), _ptr(self.state), ctypes.byref(s), ctypes.byref(g),
                                                 _stream(stream)))

    def project_backward(self, params: torch.Tensor, grads: torch.Tensor, stream=None):
        self.ctx.check(lib().dqo_project_backward(*self._fr(), _ptr(params), _ptr(self.state), _ptr(grads),
                                                  _stream(stream)))

    def project_backward_adam(self, params: torch.Tensor, m: torch.Tensor, v: torch.Tensor, lrs, d_step: torch.Tensor,
                              grads: Optional[torch.Tensor] = None, beta1=0.9, beta2=0.999, eps=1e-15, stream=None):
        """project_backward + adam_step_counted in one pass (params, m, v updated in place)."""
        assert d_step.dtype == torch.int64 and d_step.numel() == 1
        hp = _adam_hp(lrs, beta1, beta2, eps)
        self.ctx.check(lib().dqo_project_backward_adam(*self._fr(), _ptr(params), _ptr(self.state), _ptr(m), _ptr(v),
                                                       ctypes.byref(hp), _ptr(d_step), _ptr(grads), _stream(stream)))

    def pose_backward(self, params: torch.Tensor, pose_grads: Optional[torch.Tensor] = None, stream=None):
        """(dL/dw, dL/dtau) per view, [V][6] float64 on the device (left
        perturbation of each camera: R' = exp([w]x) R, t' = exp([w]x) t + tau)."""
        if pose_grads is None:
            pose_grads = torch.empty(self.V, 6, dtype=torch.float64, device=self.device)
        assert pose_grads.dtype == torch.float64 and pose_grads.numel() >= 6 * self.V
        self.ctx.check(lib().dqo_pose_backward(*self._fr(), _ptr(params), _ptr(self.state), _ptr(pose_grads),
                                               _stream(stream)))
        return pose_grads

    # -- incremental update (Eq. (7)-(8)) --
    def incremental_masks(self, img, tgt: Dict[str, torch.Tensor], masks: torch.Tensor, obj_counts: torch.Tensor,
                          stream=None, **cfg):
        """img: a loss-mode forward's images (p_target rendered with target = tgt["id"])."""
        assert masks.dtype == torch.uint8 and masks.shape == (self.V, self.H, self.W)
        assert obj_counts.dtype == torch.int32 and obj_counts.numel() >= 2 * self.K
        s = Frame._images(img)
        t = Targets(_ptr(tgt["color"]), _ptr(tgt["depth"]), _ptr(tgt["id"]))
        c = IncrementCfg(**{**INCREMENT_DEFAULTS, **cfg})
        self.ctx.check(lib().dqo_incremental_masks(*self._fr(), ctypes.byref(s), ctypes.byref(t), ctypes.byref(c),
                                                   _ptr(masks), _ptr(obj_counts), _stream(stream)))

    def densify(self, tgt: Dict[str, torch.Tensor], masks: torch.Tensor, params: torch.Tensor, ids: torch.Tensor,
                n_old: int, counts: torch.Tensor, stream=None, **cfg):
        """Writes the new Gaussians into columns [n_old, params.shape[1]) of params / ids; counts int64[V + 1]."""
        assert masks.dtype == torch.uint8 and masks.shape == (self.V, self.H, self.W)
        assert params.dtype == self.tdtype and params.shape[0] == NUM_PARAMS and ids.shape == (params.shape[1],)
        assert counts.dtype == torch.int64 and counts.numel() >= self.V + 1
        t = Targets(_ptr(tgt["color"]), _ptr(tgt["depth"]), _ptr(tgt["id"]))
        c = IncrementCfg(**{**INCREMENT_DEFAULTS, **cfg})
        self.ctx.check(lib().dqo_densify(*self._fr(), ctypes.byref(t), _ptr(masks), ctypes.byref(c), int(n_old),
                                         int(params.shape[1]), _ptr(params), _ptr(ids), _ptr(counts),
                                         _stream(stream)))


def object_loss_noalloc(ctx: Context, cams: Sequence[dict], K: int, img: Dict[str, torch.Tensor],
                        tgt: Dict[str, torch.Tensor], grads: Optional[Dict[str, torch.Tensor]], loss: torch.Tensor,
                        w_rgb=1.0, w_depth=1.0, lam=1.0, ce_eps=1e-6, stream=None):
    """The object loss of Frame.object_loss without a state buffer: its
    partial sums live in the library's per-device scratch, so the call
    allocates nothing (calls that overlap on one GPU race)."""
    dt = F64 if img["color"].dtype == torch.float64 else F32
    desc = FrameDesc(n=0, n_views=len(cams), K=int(K), pair_capacity=0, dtype=dt)
    s = Frame._images(img)
    t = Targets(_ptr(tgt["color"]), _ptr(tgt["depth"]), _ptr(tgt.get("id")))
    w = LossWeights(w_rgb, w_depth, lam, ce_eps)
    g = None
    if grads is not None:
        g = ctypes.byref(ImageGrads(*(_ptr(grads.get(k)) for k in ("d_color", "d_depth", "d_t_final", "d_probs",
                                                                  "d_p_target"))))
    ctx.check(lib().dqo_object_loss_noalloc(ctx.h, ctypes.byref(desc), make_cameras(cams), ctypes.byref(s),
                                            ctypes.byref(t), ctypes.byref(w), _ptr(loss), g, _stream(stream)))


def adam_step(ctx: Context, params, grads, m, v, lrs, step, beta1=0.9, beta2=0.999, eps=1e-15, stream=None):
    hp = AdamParams()
    for k in range(NUM_PARAMS):
        hp.lr[k] = float(lrs[k])
    hp.beta1, hp.beta2, hp.eps = beta1, beta2, eps
    dt = F64 if params.dtype == torch.float64 else F32
    ctx.check(lib().dqo_adam_step(ctx.h, dt, _ptr(params), _ptr(grads), _ptr(m), _ptr(v), params.shape[-1],
                                  ctypes.byref(hp), int(step), _stream(stream)))


def _adam_hp(lrs, beta1, beta2, eps):
    hp = AdamParams()
    for k in range(NUM_PARAMS):
        hp.lr[k] = float(lrs[k])
    hp.beta1, hp.beta2, hp.eps = beta1, beta2, eps
    return hp


def adam_step_counted(ctx: Context, params, grads, m, v, lrs, d_step, beta1=0.9, beta2=0.999, eps=1e-15,
                      stream=None):
    """Adam with the step count in device memory (graph-capturable)."""
    hp = _adam_hp(lrs, beta1, beta2, eps)
    dt = F64 if params.dtype == torch.float64 else F32
    assert d_step.dtype == torch.int64 and d_step.numel() == 1
    ctx.check(lib().dqo_adam_step_counted(ctx.h, dt, _ptr(params), _ptr(grads), _ptr(m), _ptr(v), params.shape[-1],
                                          ctypes.byref(hp), _ptr(d_step), _stream(stream)))


def camera_matrix(cam) -> np.ndarray:
    """3x4 projection P = K [R | t] of a camera dict (the P of the quadric fit)."""
    Kc = np.array([[cam["fx"], 0.0, cam["cx"]], [0.0, cam["fy"], cam["cy"]], [0.0, 0.0, 1.0]])
    Rt = np.concatenate([np.asarray(cam["R"], np.float64).reshape(3, 3),
                         np.asarray(cam["t"], np.float64).reshape(3, 1)], axis=1)
    return Kc @ Rt


def id_boxes(ctx: Context, id_map: torch.Tensor, K: int, stream=None):
    """Per (view, object) pixel-edge boxes of the rendered id maps [V][H][W]."""
    V, H, W = id_map.shape
    boxes = torch.empty(V * K, 4, dtype=torch.float64, device=id_map.device)
    box_obj = torch.empty(V * K, dtype=torch.int32, device=id_map.device)
    box_view = torch.empty(V * K, dtype=torch.int32, device=id_map.device)
    ctx.check(lib().dqo_id_boxes(ctx.h, _ptr(id_map), V, W, H, K, _ptr(boxes), _ptr(box_obj), _ptr(box_view),
                                 _stream(stream)))
    return boxes, box_obj, box_view


def fit_dual_quadric(ctx: Context, boxes, box_obj, box_view, Ps, n_obj, img_wh=None, border=1.0, stream=None):
    """Device tensors in, device tensors out (see dqo_fit_dual_quadric)."""
    dev = boxes.device
    Q = torch.empty(n_obj, 4, 4, dtype=torch.float64, device=dev)
    mu = torch.empty(n_obj, 3, dtype=torch.float64, device=dev)
    R = torch.empty(n_obj, 3, 3, dtype=torch.float64, device=dev)
    axes = torch.empty(n_obj, 3, dtype=torch.float64, device=dev)
    status = torch.empty(n_obj, dtype=torch.int32, device=dev)
    ctx.check(lib().dqo_fit_dual_quadric(ctx.h, int(n_obj), int(boxes.shape[0]), _ptr(boxes), _ptr(box_obj),
                                         _ptr(box_view), int(Ps.shape[0]), _ptr(Ps), _ptr(img_wh), float(border),
                                         _ptr(Q), _ptr(mu), _ptr(R), _ptr(axes), _ptr(status), _stream(stream)))
    return dict(Q=Q, mu=mu, R=R, axes=axes, status=status)


# association thresholds (the paper leaves tau and the IoU threshold unstated)
ASSOC_DEFAULTS = dict(iou_min=0.3, tau=1.0, qd_min=0.5, t_occ=0.85, qd_occ=0.1)


def associate(ctx: Context, mu, R, axes, boxes, det_frame, Ps, img_wh, iou_min=ASSOC_DEFAULTS["iou_min"],
              occlusion=True, stream=None):
    """Association scores of detections against object quadrics (device tensors)."""
    n_obj, n_det = int(mu.shape[0]), int(boxes.shape[0])
    dev = boxes.device
    iou = torch.empty(n_obj, n_det, dtype=torch.float64, device=dev)
    match = torch.empty(n_det, dtype=torch.int32, device=dev)
    occ = torch.empty(n_det, n_det, dtype=torch.float64, device=dev) if occlusion else None
    ctx.check(lib().dqo_associate(ctx.h, n_obj, _ptr(mu), _ptr(R), _ptr(axes), n_det, _ptr(boxes), _ptr(det_frame),
                                  int(Ps.shape[0]), _ptr(Ps), _ptr(img_wh), float(iou_min), _ptr(iou), _ptr(match),
                                  _ptr(occ), _stream(stream)))
    return dict(iou=iou, match=match, occ=occ)


def quadric_distance(ctx: Context, a, b, tau=ASSOC_DEFAULTS["tau"], stream=None):
    """Eq. (5) between quadric sets a and b (dicts of mu, R, axes device tensors)."""
    na, nb = int(a["mu"].shape[0]), int(b["mu"].shape[0])
    qd = torch.empty(na, nb, dtype=torch.float64, device=a["mu"].device)
    ctx.check(lib().dqo_quadric_distance(ctx.h, na, _ptr(a["mu"]), _ptr(a["R"]), _ptr(a["axes"]), nb, _ptr(b["mu"]),
                                         _ptr(b["R"]), _ptr(b["axes"]), float(tau), _ptr(qd), _stream(stream)))
    return qd


def associate_decide(ctx: Context, match, qd_obs, occ, qd_det, label, qd_min=ASSOC_DEFAULTS["qd_min"],
                     t_occ=ASSOC_DEFAULTS["t_occ"], qd_occ=ASSOC_DEFAULTS["qd_occ"], stream=None):
    """QD filter of the coarse matches and occlusion merge (device tensors):
    returns fine, parent, root and obj, one int32 per detection."""
    n_det = int(match.shape[0])
    n_obj = int(qd_obs.shape[1]) if qd_obs is not None and qd_obs.dim() == 2 else 0
    out = {k: torch.empty(n_det, dtype=torch.int32, device=match.device) for k in ("fine", "parent", "root", "obj")}
    ctx.check(lib().dqo_associate_decide(ctx.h, n_det, n_obj, _ptr(match), _ptr(qd_obs), _ptr(occ), _ptr(qd_det),
                                         _ptr(label), float(qd_min), float(t_occ), float(qd_occ), _ptr(out["fine"]),
                                         _ptr(out["parent"]), _ptr(out["root"]), _ptr(out["obj"]), _stream(stream)))
    return out


def quadric_iou_grad(ctx: Context, boxes, box_obj, box_view, Ps, theta, img_wh=None, stream=None):
    """J_k and dJ_k/dtheta_k of Eq. (9) at theta[n_obj][10] (device tensors)."""
    n_obj = int(theta.shape[0])
    dev = theta.device
    loss = torch.empty(n_obj, dtype=torch.float64, device=dev)
    grad = torch.empty(n_obj, 10, dtype=torch.float64, device=dev)
    iou = torch.full((boxes.shape[0],), float("nan"), dtype=torch.float64, device=dev)
    ctx.check(lib().dqo_quadric_iou_grad(ctx.h, n_obj, int(boxes.shape[0]), _ptr(boxes), _ptr(box_obj),
                                         _ptr(box_view), int(Ps.shape[0]), _ptr(Ps), _ptr(img_wh), _ptr(theta),
                                         _ptr(loss), _ptr(grad), _ptr(iou), _stream(stream)))
    return dict(loss=loss, grad=grad, iou=iou)


def refine_quadrics(ctx: Context, boxes, box_obj, box_view, Ps, fit, img_wh=None, stream=None, **cfg):
    """Refines fit = dict(mu, R, axes[, status]) in place by Adam on the IoU
    loss; returns fit with Q, loss (n_obj, 2) and the final per-box IoU."""
    c = RefineCfg(**{**REFINE_DEFAULTS, **cfg})
    n_obj = int(fit["mu"].shape[0])
    dev = fit["mu"].device
    Q = fit.get("Q")
    if Q is None:
        Q = torch.empty(n_obj, 4, 4, dtype=torch.float64, device=dev)
    loss = torch.empty(n_obj, 2, dtype=torch.float64, device=dev)
    iou = torch.full((boxes.shape[0],), float("nan"), dtype=torch.float64, device=dev)
    ctx.check(lib().dqo_refine_quadrics(ctx.h, n_obj, int(boxes.shape[0]), _ptr(boxes), _ptr(box_obj),
                                        _ptr(box_view), int(Ps.shape[0]), _ptr(Ps), _ptr(img_wh),
                                        _ptr(fit.get("status")), ctypes.byref(c), _ptr(fit["mu"]), _ptr(fit["R"]),
                                        _ptr(fit["axes"]), _ptr(Q), _ptr(loss), _ptr(iou), _stream(stream)))
    return dict(fit, Q=Q, loss=loss, iou=iou)


# ------------------------------------------------------------------ helpers
def default_lrs(scene_extent: float = 1.0):
    """Per-row learning rates: mean 1.6e-4 * extent, log-scale 5e-3, quaternion
    1e-3, opacity logit 5e-2, colour 2.5e-3."""
    return [1.6e-4 * scene_extent] * 3 + [5e-3] * 3 + [1e-3] * 4 + [5e-2] + [2.5e-3] * 3


class Rasterizer:
    """Frame + image buffers for a fixed camera set, with capacity management."""

    def __init__(self, cams: Sequence[dict], n: int, K: int, capacity: Optional[int] = None,
                 dtype=torch.float32, ctx: Optional[Context] = None, device="cuda", segments=None, windows=None,
                 jobs=None):
        self.ctx = ctx if ctx is not None else Context()
        self.cams, self.n, self.K, self.dtype, self.device = list(cams), int(n), int(K), dtype, device
        self.segments, self.windows, self.jobs = segments, windows, jobs
        cap = capacity if capacity is not None else max(1024, 4 * n * (len(cams) if segments is None else 1))
        self.frame = self._new_frame(min(cap, 1 << 30))
        self.generation = 0   # bumped by every bin(): identifies the pair list in the state

    def _new_frame(self, capacity):
        return Frame(self.ctx, self.cams, self.n, self.K, capacity, self.dtype, self.device, segments=self.segments,
                     windows=self.windows, jobs=self.jobs)

    def bin(self, params, ids, grow=True, stream=None):
        """project_cull_bin + sort; when grow is set, checks the pair count (a
        host synchronisation) and re-runs with a larger pair list on overflow."""
        self.generation += 1
        f = self.frame
        f.project_cull_bin(params, ids, stream)
        if grow:
            rc, st, npairs = f.read_status(stream)
            if st & STATUS_OVERFLOW:
                cap = min(1 << 30, int(math.ceil(npairs * 1.25)) + 1024)
                self.frame = f = self._new_frame(cap)
                f.project_cull_bin(params, ids, stream)
                rc, st, npairs = f.read_status(stream)
            if st & STATUS_TIMEOUT:
                raise DqoError(EINTERNAL, "device wait bound exceeded")
        f.sort(stream)

    def forward(self, params, ids, probs=False, id_map=False, target=None, stream=None, grow=True, n_blend=False):
        self.bin(params, ids, grow=grow, stream=stream)
        img = self.frame.new_images(probs=probs, id_map=id_map, target=target, n_blend=n_blend)
        self.frame.render_forward(img, stream)
        return img

    def backward(self, params, img, grads, stream=None):
        f = self.frame
        f.render_backward(img, grads, stream)
        out = torch.empty_like(params)
        f.project_backward(params, out, stream)
        return out


class RasterizeFunction(torch.autograd.Function):
    """Differentiable render of (colour, depth, T_final, instance channels)
    with respect to the Gaussian parameters [14][n].  Backward recomputes the
    transmittance per pixel from T_final instead of storing per-pixel lists."""

    @staticmethod
    def forward(ctx, params, ids, rasterizer: Rasterizer, want_probs: bool = True):
        p = params.detach().contiguous()
        img = rasterizer.forward(p, ids, probs=want_probs and rasterizer.K > 0)
        ctx.rasterizer = rasterizer
        ctx.generation = rasterizer.generation
        ctx.ids = ids
        ctx.want_probs = want_probs and rasterizer.K > 0
        probs = img["probs"] if ctx.want_probs else img["color"].new_zeros(0)
        # Outputs are saved through save_for_backward: holding them on ctx would
        # make a reference cycle (output -> grad_fn -> ctx -> output) that keeps
        # every iteration's images alive until a cyclic garbage collection.
        ctx.save_for_backward(p, img["color"], img["depth"], img["t_final"])
        ctx.last = img["last"]   # not an output
        return img["color"], img["depth"], img["t_final"], probs

    @staticmethod
    def backward(ctx, d_color, d_depth, d_t_final, d_probs):
        p, color, depth, t_final = ctx.saved_tensors
        img = dict(color=color, depth=depth, t_final=t_final, last=ctx.last)
        r: Rasterizer = ctx.rasterizer
        if r.generation != ctx.generation:
            # Another forward reused the pair list since: rebuild it from the saved
            # parameters (binning and sorting are deterministic, so the positions
            # stored in `last` refer to the same list again).
            r.bin(p, ctx.ids)
            ctx.generation = r.generation
        z = lambda t, like: (t.contiguous() if t is not None else torch.zeros_like(like))
        grads = dict(d_color=z(d_color, color), d_depth=z(d_depth, depth), d_t_final=z(d_t_final, t_final))
        if ctx.want_probs and d_probs is not None:
            grads["d_probs"] = d_probs.contiguous()
        g = r.backward(p, img, grads)
        return g, None, None, None


def rasterize(params, ids, rasterizer: Rasterizer, want_probs=True):
    return RasterizeFunction.apply(params, ids, rasterizer, want_probs)


class Trainer:
    """The timed training iteration: project/bin, sort, render forward (loss
    mode: probability of each pixel's target object), object loss, render
    backward, project backward and Adam, all as libdqo calls on one stream
    with preallocated buffers and no host synchronisation.  With fused set,
    project backward and Adam are one call (same results, one pass over the
    parameters); self.grads is then not written."""

    def __init__(self, params: torch.Tensor, ids: torch.Tensor, cams, K, targets: Dict[str, torch.Tensor],
                 lrs=None, capacity=None, loss_weights=(1.0, 1.0, 1.0), ctx=None, segments=None, fused=True,
                 status_every=100, windows=None, jobs=None):
        self.params = params.contiguous()
        self.ids = ids
        self.n = params.shape[1]
        self.dtype = params.dtype
        self.r = Rasterizer(cams, self.n, K, capacity=capacity, dtype=self.dtype, ctx=ctx, segments=segments,
                            device=params.device, windows=windows, jobs=jobs)
        self.r.bin(self.params, ids, grow=True)  # sizes the pair list once
        if self.r.frame.capacity < (1 << 30):   # headroom for pairs added while training
            cap = min(1 << 30, int(self.r.frame.read_status()[2] * 1.5) + 4096)
            if cap > self.r.frame.capacity:
                self.r.frame = self.r._new_frame(cap)
                self.r.bin(self.params, ids, grow=True)
        f = self.r.frame
        self.targets = targets
        self.img = f.new_images(target=targets["id"])
        dev = params.device
        V, H, W = f.V, f.H, f.W
        self.grads_img = dict(d_color=torch.empty(V, 3, H, W, dtype=self.dtype, device=dev),
                              d_depth=torch.empty(V, H, W, dtype=self.dtype, device=dev),
                              d_p_target=torch.empty(V, H, W, dtype=self.dtype, device=dev))
        self.grads = torch.empty_like(self.params)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.loss = torch.zeros(4, dtype=torch.float64, device=dev)
        self.lrs = lrs if lrs is not None else default_lrs()
        self.lw = loss_weights
        self.step_count = 0
        self.d_step = torch.zeros(1, dtype=torch.int64, device=dev)  # Adam step count on the device
        self.fused = fused   # project backward and Adam in one pass (bitwise the same as the two calls)
        # Every status_every steps (0: never) the device status word is read
        # (a host synchronisation): pair-list overflow or a device wait that
        # gave up raise DqoError.  After a timeout the library orders the
        # sort's blocks by ticket until the status is cleared.
        self.status_every = int(status_every)

    def step(self, stream=None):
        f = self.r.frame
        f.project_cull_bin(self.params, self.ids, stream)
        f.sort(stream)
        f.render_forward(self.img, stream)
        f.object_loss(self.img, self.targets, self.grads_img, self.loss, *self.lw, stream=stream)
        f.render_backward(self.img, self.grads_img, stream)
        self.step_count += 1
        if self.fused:
            f.project_backward_adam(self.params, self.m, self.v, self.lrs, self.d_step, stream=stream)
        else:
            f.project_backward(self.params, self.grads, stream)
            adam_step_counted(self.r.ctx, self.params, self.grads, self.m, self.v, self.lrs, self.d_step,
                              stream=stream)
        if self.status_every and self.step_count % self.status_every == 0:
            self.check(stream)

    def replay(self, graph, steps: int):
        """Replays a captured step `steps` times, reading the device status
        every status_every replays and after the last."""
        for i in range(1, steps + 1):
            graph.replay()
            self.step_count += 1
            if self.status_every and (i % self.status_every == 0 or i == steps):
                self.check()

    def capture(self):
        """Records one training step (every kernel of it, on one stream) in a
        HIP graph; replaying the graph performs one more step."""
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            self.step()  # warm-up outside the capture
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        every, self.status_every = self.status_every, 0   # no synchronisation inside the capture
        try:
            with torch.cuda.graph(g):
                self.step()
        finally:
            self.status_every = every
        self.step_count -= 1  # the capture itself does not run
        return g

    def check(self, stream=None):
        """Reads the device status (synchronises): raises DqoError on pair-list
        overflow or a device wait that gave up; returns the pair count."""
        rc, st, npairs = self.r.frame.read_status(stream)
        if st & (STATUS_OVERFLOW | STATUS_TIMEOUT):
            raise DqoError(ECAPACITY if st & STATUS_OVERFLOW else EINTERNAL,
                           f"status {st}, pairs {npairs}, capacity {self.r.frame.capacity}")
        return npairs
