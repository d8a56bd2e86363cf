"""PyTorch binding of the C ABI: device tensors in, device tensors out.

PyTorch supplies device memory and the current HIP stream; every step of rendering
runs in the library's HIP kernels.  Cameras are the plain dictionaries of
``paper_2609_13397_amd.synth`` (or anything with the same keys).
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

from . import _lib

FILTER_CENTER_RAY, FILTER_ANISOTROPIC, FILTER_ISOTROPIC = 0, 1, 2
COMPOSE_MARGINAL, COMPOSE_ADDITIVE = 0, 1
ORDER_KEY, ORDER_RAY = 0, 1
BACKBONE_MAX_RESPONSE, BACKBONE_RAY_INTEGRAL = 0, 1

PARAM_NAMES = ("means", "log_scales", "quats", "opacity_logits", "color")


@dataclass
class RenderOpts:
    filter_mode: int = FILTER_ANISOTROPIC
    use_floor: bool = False
    composition: int = COMPOSE_MARGINAL
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    T_min: float = 1e-4
    t_near: float = 0.2
    bg: tuple = (0.0, 0.0, 0.0)
    footprint_scale: float = 1.0
    count_pairs: bool = False
    order_mode: int = ORDER_KEY
    backbone: int = BACKBONE_MAX_RESPONSE

    def to_c(self) -> _lib.CgOpts:
        o = _lib.CgOpts()
        o.filter_mode = int(self.filter_mode)
        o.use_floor = 1 if self.use_floor else 0
        o.composition = int(self.composition)
        o.alpha_min = self.alpha_min
        o.alpha_max = self.alpha_max
        o.T_min = self.T_min
        o.t_near = self.t_near
        o.bg[:] = list(self.bg)
        o.footprint_scale = self.footprint_scale
        o.count_pairs = 1 if self.count_pairs else 0
        o.order_mode = int(self.order_mode)
        o.backbone = int(self.backbone)
        return o


def camera_struct(cam: dict) -> _lib.CgCamera:
    c = _lib.CgCamera()
    c.model = cam["model"]
    c.full_w, c.full_h = cam["full_w"], cam["full_h"]
    c.crop_x0, c.crop_y0, c.crop_w, c.crop_h = cam["crop"]
    c.fx, c.fy, c.cx, c.cy = cam["fx"], cam["fy"], cam["cx"], cam["cy"]
    c.k[:] = list(cam["k"])
    c.R_c2w[:] = [float(v) for row in cam["R_c2w"] for v in row]
    c.origin[:] = list(cam["origin"])
    c.theta_max = cam["theta_max"]
    return c


def cameras_array(cams: Sequence[dict]):
    arr = (_lib.CgCamera * len(cams))(*[camera_struct(c) for c in cams])
    return arr


def view_pixels(cams: Sequence[dict]) -> List[int]:
    return [c["crop"][2] * c["crop"][3] for c in cams]


def _stream_handle(device) -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


class TorchAllocator:
    """A cg_allocator whose scratch comes from PyTorch's caching allocator, on the
    stream the library passes (the call's stream), so scratch memory is counted and
    reused by torch like any tensor's.  A failed allocation returns NULL, which the
    library turns into CG_ERR_OUT_OF_MEMORY after freeing what the call already held."""

    def __init__(self):
        self._alloc = _lib.ALLOC_FN(self._on_alloc)
        self._free = _lib.FREE_FN(self._on_free)
        self.struct = _lib.CgAllocator(None, self._alloc, self._free)

    def allocate(self, nbytes: int, stream: int) -> int:
        return torch._C._cuda_cudaCachingAllocator_raw_alloc(int(nbytes), int(stream))

    def release(self, ptr: int) -> None:
        torch._C._cuda_cudaCachingAllocator_raw_delete(int(ptr))

    def _on_alloc(self, ctx, nbytes, stream):
        try:
            return self.allocate(nbytes, stream or 0)
        except Exception:  # out of memory (or any failure): NULL
            return None

    def _on_free(self, ctx, ptr, stream):
        if ptr:
            self.release(ptr)


_TORCH_ALLOCATOR: Optional[TorchAllocator] = None


def torch_allocator() -> TorchAllocator:
    global _TORCH_ALLOCATOR
    if _TORCH_ALLOCATOR is None:
        _TORCH_ALLOCATOR = TorchAllocator()
    return _TORCH_ALLOCATOR


@dataclass
class Scene:
    """Gaussian parameters as float32 device tensors, component-major ([C][N])."""
    means: torch.Tensor
    log_scales: torch.Tensor
    quats: torch.Tensor
    opacity_logits: torch.Tensor
    color: torch.Tensor
    rho2: Optional[torch.Tensor] = None
    color_mode: int = 0

    @property
    def n(self) -> int:
        return int(self.opacity_logits.shape[0])

    @staticmethod
    def from_numpy(scene: dict, device="cuda") -> "Scene":
        t = {k: torch.from_numpy(np.ascontiguousarray(scene[k], dtype=np.float32)).to(device)
             for k in PARAM_NAMES}
        rho2 = scene.get("rho2")
        r = None if rho2 is None else torch.from_numpy(np.ascontiguousarray(rho2, dtype=np.float32)).to(device)
        return Scene(t["means"], t["log_scales"], t["quats"], t["opacity_logits"], t["color"], r,
                     int(scene["color_mode"]))

    def check(self):
        n = self.n
        ncol = 3 if self.color_mode == 0 else 48
        shapes = {"means": (3, n), "log_scales": (3, n), "quats": (4, n), "opacity_logits": (n,),
                  "color": (ncol, n)}
        for k, shp in shapes.items():
            t = getattr(self, k)
            if tuple(t.shape) != shp or t.dtype != torch.float32 or not t.is_contiguous() or not t.is_cuda:
                raise ValueError(f"{k}: expected contiguous float32 cuda tensor of shape {shp}, "
                                 f"got {tuple(t.shape)} {t.dtype} cuda={t.is_cuda}")
        if self.rho2 is not None and (tuple(self.rho2.shape) != (n,) or self.rho2.dtype != torch.float32
                                      or not self.rho2.is_contiguous()):
            raise ValueError("rho2: expected contiguous float32 tensor of shape (n,)")

    def to_c(self) -> _lib.CgGaussians:
        self.check()
        g = _lib.CgGaussians()
        g.n = self.n
        g.color_mode = self.color_mode
        g.means = _ptr(self.means)
        g.log_scales = _ptr(self.log_scales)
        g.quats = _ptr(self.quats)
        g.opacity_logits = _ptr(self.opacity_logits)
        g.color = _ptr(self.color)
        g.rho2 = _ptr(self.rho2)
        return g


class ForwardState:
    """Owns a cg_fwd_state; released when garbage-collected or by release()."""

    def __init__(self, handle: C.c_void_p, keep: tuple):
        self.handle = handle
        self.keep = keep  # tensors the state points into, and the allocator of its scratch

    def release(self):
        if self.handle:
            _lib.lib().cg_fwd_state_release(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


def render_forward(scene: Scene, cams: Sequence[dict], opts: RenderOpts = None, need_state: bool = False,
                   out: Optional[torch.Tensor] = None, allocator: Optional[TorchAllocator] = None):
    """Renders ``cams`` (one batched call).  Returns (rgba [sum px, 4] float32 tensor,
    stats dict, ForwardState or None).  Scratch memory comes from ``allocator``
    (default: PyTorch's caching allocator on the current stream)."""
    opts = opts or RenderOpts()
    allocator = allocator or torch_allocator()
    L = _lib.lib()
    device = scene.means.device
    npx = sum(view_pixels(cams))
    if out is None:
        out = torch.empty((npx, 4), dtype=torch.float32, device=device)
    elif tuple(out.shape) != (npx, 4) or out.dtype != torch.float32 or not out.is_contiguous():
        raise ValueError("out must be a contiguous float32 tensor of shape (pixels, 4)")
    g = scene.to_c()
    carr = cameras_array(cams)
    o = opts.to_c()
    stats = _lib.CgStats()
    state = C.c_void_p(0)
    with torch.cuda.device(device):
        st = L.cg_render_forward(_lib.byref(g), C.cast(carr, C.c_void_p), len(cams), _lib.byref(o),
                                 _lib.byref(allocator.struct), C.c_void_p(out.data_ptr()),
                                 C.byref(state) if need_state else None, _lib.byref(stats), _stream_handle(device))
    _lib.check(st)
    fs = ForwardState(state, (scene, out, allocator)) if need_state else None
    info = {"n_pairs": stats.n_pairs, "n_tiles": stats.n_tiles, "n_pixels": stats.n_pixels,
            "sort_bits": stats.sort_bits, "n_evaluated": stats.n_evaluated, "n_full": stats.n_full,
            "n_contrib": stats.n_contrib, "n_order_overflow": stats.n_order_overflow,
            "n_segments": stats.n_segments, "max_tile_pairs": stats.max_tile_pairs}
    return out, info, fs


def render_forward_noalloc(scene: Scene, cams: Sequence[dict], opts: RenderOpts = None,
                           out: Optional[torch.Tensor] = None):
    """cg_render_forward_noalloc: the inference forward with its scratch in the library's
    fixed per-GPU device array (no allocation inside the call).  ``out`` (or a new tensor)
    receives rgba [sum px, 4].  Returns (rgba, stats dict)."""
    opts = opts or RenderOpts()
    L = _lib.lib()
    device = scene.means.device
    npx = sum(view_pixels(cams))
    if out is None:
        out = torch.empty((npx, 4), dtype=torch.float32, device=device)
    elif tuple(out.shape) != (npx, 4) or out.dtype != torch.float32 or not out.is_contiguous():
        raise ValueError("out must be a contiguous float32 tensor of shape (pixels, 4)")
    g = scene.to_c()
    carr = cameras_array(cams)
    o = opts.to_c()
    stats = _lib.CgStats()
    with torch.cuda.device(device):
        st = L.cg_render_forward_noalloc(_lib.byref(g), C.cast(carr, C.c_void_p), len(cams), _lib.byref(o),
                                         C.c_void_p(out.data_ptr()), _lib.byref(stats), _stream_handle(device))
    _lib.check(st)
    return out, {"n_pairs": stats.n_pairs, "n_tiles": stats.n_tiles, "n_segments": stats.n_segments}


def set_tile_split(max_tiles: int = 0, min_longest: int = 0, seg_len: int = 0) -> None:
    """Thresholds of the split tile render (cg_set_tile_split); zeros restore the defaults."""
    _lib.lib().cg_set_tile_split(int(max_tiles), int(min_longest), int(seg_len))


def set_scratch_guards(mode: int) -> None:
    """Scratch guard bands (cg_debug_set_scratch_guards): 0 off, 1 on, 2 on with one
    band overwritten from the host before the check."""
    _lib.lib().cg_debug_set_scratch_guards(int(mode))


def guard_violations() -> int:
    """Changed guard words found since the library was loaded (cg_debug_guard_violations)."""
    return int(_lib.lib().cg_debug_guard_violations())


def split_views(rgba: torch.Tensor, cams: Sequence[dict]) -> List[torch.Tensor]:
    """Per-view [h, w, 4] views of a flat forward output."""
    outs = []
    off = 0
    for c in cams:
        w, h = c["crop"][2], c["crop"][3]
        outs.append(rgba[off:off + w * h].view(h, w, 4))
        off += w * h
    return outs


def render_backward(state: ForwardState, grad_rgba: torch.Tensor, scene: Scene) -> Dict[str, torch.Tensor]:
    """Gradients of sum(grad_rgba * rgba) w.r.t. the raw parameters of ``scene``.
    grad_rgba: float32 tensor of the forward output's shape, on the scene's device."""
    L = _lib.lib()
    if not state.handle:
        raise ValueError("the forward state was already released")
    out = state.keep[1]
    if (tuple(grad_rgba.shape) != tuple(out.shape) or grad_rgba.dtype != torch.float32
            or grad_rgba.device != out.device):
        raise ValueError(f"grad_rgba: expected float32 {tuple(out.shape)} on {out.device}, got "
                         f"{grad_rgba.dtype} {tuple(grad_rgba.shape)} on {grad_rgba.device}")
    grads = {k: torch.empty_like(getattr(scene, k)) for k in PARAM_NAMES}
    g = grad_rgba.contiguous()
    with torch.cuda.device(scene.means.device):
        st = L.cg_render_backward(state.handle, C.c_void_p(g.data_ptr()),
                                  *[C.c_void_p(grads[k].data_ptr()) for k in PARAM_NAMES],
                                  _stream_handle(scene.means.device))
    _lib.check(st)
    return grads


def replay_mismatches(state: ForwardState) -> int:
    """Pixels whose backward replay did not reproduce the forward transmittance."""
    return int(_lib.lib().cg_bwd_replay_mismatches(state.handle))


def camera_unproject(cam: dict, pix_xy: torch.Tensor):
    """Pi^{-1} of continuous full-image coordinates pix_xy [2, n] (float32 cuda).
    Returns (dirs [3, n], valid [n] bool)."""
    L = _lib.lib()
    pix_xy = pix_xy.contiguous()
    n = pix_xy.shape[1]
    dirs = torch.empty((3, n), dtype=torch.float32, device=pix_xy.device)
    valid = torch.empty((n,), dtype=torch.uint8, device=pix_xy.device)
    c = camera_struct(cam)
    _lib.check(L.cg_camera_unproject(_lib.byref(c), n, C.c_void_p(pix_xy.data_ptr()), C.c_void_p(dirs.data_ptr()),
                                     C.c_void_p(valid.data_ptr()), _stream_handle(pix_xy.device)))
    return dirs, valid.bool()


def bake_rho2(scene: Scene, cams: Sequence[dict], t_near: float = 0.2) -> torch.Tensor:
    """Eq. 11 floor variance per Gaussian over ``cams`` (float32 cuda [n])."""
    L = _lib.lib()
    out = torch.empty((scene.n,), dtype=torch.float32, device=scene.means.device)
    g = scene.to_c()
    carr = cameras_array(cams)
    _lib.check(L.cg_bake_rho2(_lib.byref(g), C.cast(carr, C.c_void_p), len(cams), float(t_near),
                              C.c_void_p(out.data_ptr()), _stream_handle(scene.means.device)))
    return out


class ConeGaussRender(torch.autograd.Function):
    """Differentiable render of a batch of views; gradients flow to the raw
    parameters (means, log-scales, quaternions, opacity logits, colour)."""

    @staticmethod
    def forward(ctx, means, log_scales, quats, opacity_logits, color, rho2, cams, opts, color_mode):
        scene = Scene(means.contiguous(), log_scales.contiguous(), quats.contiguous(),
                      opacity_logits.contiguous(), color.contiguous(),
                      None if rho2 is None else rho2.contiguous(), color_mode)
        rgba, _, state = render_forward(scene, cams, opts, need_state=True)
        ctx.state = state
        ctx.scene = scene
        # The backward reads the forward image (the colour behind each pair comes from it)
        # and the parameters: saved here, autograd refuses a backward after any of them
        # was modified in place.
        ctx.save_for_backward(means, log_scales, quats, opacity_logits, color, rho2, rgba)
        return rgba

    @staticmethod
    def backward(ctx, grad_rgba):
        ctx.saved_tensors  # raises if a saved tensor was modified in place since the forward
        grads = render_backward(ctx.state, grad_rgba, ctx.scene)
        ctx.state.release()
        return (grads["means"], grads["log_scales"], grads["quats"], grads["opacity_logits"], grads["color"],
                None, None, None, None)


def render(scene: Scene, cams: Sequence[dict], opts: RenderOpts = None) -> torch.Tensor:
    """Differentiable batched render; returns rgba [sum px, 4]."""
    return ConeGaussRender.apply(scene.means, scene.log_scales, scene.quats, scene.opacity_logits, scene.color,
                                 scene.rho2, list(cams), opts or RenderOpts(), scene.color_mode)


class Profiler:
    """Per-stage GPU time of the library's kernels (HIP events on their streams).
    ``stages``: names of the stages to bracket (None: all)."""

    def __init__(self, stages: Optional[Sequence[str]] = None):
        L = _lib.lib()
        self.names = [L.cg_profile_stage_name(i).decode() for i in range(L.cg_profile_num_stages())]
        unknown = set(stages or []) - set(self.names)
        if unknown:
            raise ValueError(f"unknown profiling stages {sorted(unknown)}")
        self.mask = 0xFFFFFFFF if stages is None else sum(1 << self.names.index(n) for n in stages)

    def __enter__(self):
        L = _lib.lib()
        L.cg_profile_read(None, None)
        L.cg_profile_enable_stages(self.mask)
        return self

    def __exit__(self, *exc):
        L = _lib.lib()
        L.cg_profile_enable(0)
        return False

    def read(self) -> Dict[str, dict]:
        L = _lib.lib()
        _lib.check(L.cg_profile_collect())
        n = len(self.names)
        ms = (C.c_double * n)()
        cnt = (C.c_int64 * n)()
        L.cg_profile_read(C.cast(ms, C.c_void_p), C.cast(cnt, C.c_void_p))
        return {self.names[i]: {"ms": ms[i], "launches": cnt[i]} for i in range(n)}
