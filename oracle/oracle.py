"""ctypes wrapper around the FP64 CPU oracle (test infrastructure only).

All functions take the plain scene / camera dictionaries produced by the seeded
generators and return numpy float64 arrays.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build_oracle

__all__ = [
    "Opts", "lib", "render", "render_supersampled", "unproject", "project", "pixel_rays",
    "pair_batch", "preprocess", "sh_basis", "bake_rho2", "grad", "N_ALT",
]

N_ALT = 4  # alternatives stored per pixel (one per flipped near-threshold decision)


class _Camera(C.Structure):
    _fields_ = [
        ("model", C.c_int32), ("full_w", C.c_int32), ("full_h", C.c_int32),
        ("crop_x0", C.c_int32), ("crop_y0", C.c_int32), ("crop_w", C.c_int32), ("crop_h", C.c_int32),
        ("fx", C.c_float), ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float),
        ("k", C.c_float * 4), ("R_c2w", C.c_float * 9), ("origin", C.c_float * 3),
        ("theta_max", C.c_float),
    ]


class _Gaussians(C.Structure):
    _fields_ = [
        ("n", C.c_int64), ("color_mode", C.c_int32),
        ("means", C.c_void_p), ("log_scales", C.c_void_p), ("quats", C.c_void_p),
        ("opacity_logits", C.c_void_p), ("color", C.c_void_p), ("rho2", C.c_void_p),
    ]


class _Opts(C.Structure):
    _fields_ = [
        ("filter_mode", C.c_int32), ("use_floor", C.c_int32), ("composition", C.c_int32),
        ("alpha_min", C.c_float), ("alpha_max", C.c_float), ("T_min", C.c_float), ("t_near", C.c_float),
        ("bg", C.c_float * 3), ("footprint_scale", C.c_float), ("order_mode", C.c_int32),
        ("backbone", C.c_int32),
    ]


class Opts:
    """Render options (same meaning as the library's): filter_mode 0 centre ray,
    1 anisotropic footprint, 2 isotropic; use_floor applies Eq. 10 with rho^2;
    composition 0 marginal (Eq. 12), 1 additive; order_mode 0 composites by the
    per-Gaussian key |mu - o|, 1 by each ray's own max-response depth t*; backbone 0 is
    the max response (C = 1), 1 the ray integral (w = 1, with the Z_G reading)."""

    def __init__(self, filter_mode=1, use_floor=0, composition=0, alpha_min=1.0 / 255.0,
                 alpha_max=0.99, T_min=1e-4, t_near=0.2, bg=(0.0, 0.0, 0.0), footprint_scale=1.0,
                 order_mode=0, backbone=0):
        self.filter_mode = filter_mode
        self.use_floor = use_floor
        self.composition = composition
        self.alpha_min = alpha_min
        self.alpha_max = alpha_max
        self.T_min = T_min
        self.t_near = t_near
        self.bg = tuple(bg)
        self.footprint_scale = footprint_scale
        self.order_mode = order_mode
        self.backbone = backbone

    @staticmethod
    def smooth(**kw):
        """No cut-offs (alpha_min = 0, alpha_max = 1, T_min = 0): a smooth function of
        the parameters, for finite differences."""
        base = dict(alpha_min=0.0, alpha_max=1.0, T_min=0.0)
        base.update(kw)
        return Opts(**base)

    def _c(self):
        o = _Opts()
        o.filter_mode = self.filter_mode
        o.use_floor = self.use_floor
        o.composition = self.composition
        o.alpha_min = self.alpha_min
        o.alpha_max = self.alpha_max
        o.T_min = self.T_min
        o.t_near = self.t_near
        o.bg[:] = list(self.bg)
        o.footprint_scale = self.footprint_scale
        o.order_mode = self.order_mode
        o.backbone = self.backbone
        return o


_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        path = build_oracle.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(build_oracle.SRC):
            build_oracle.build()
        L = C.CDLL(path)
        vp = C.c_void_p
        L.orc_unproject.argtypes = [vp, C.c_int64, vp, vp, vp, vp]
        L.orc_project.argtypes = [vp, C.c_int64, vp, vp, vp, vp]
        L.orc_pixel_rays.argtypes = [vp, vp, vp]
        L.orc_sh_basis.argtypes = [vp, vp]
        L.orc_preprocess.argtypes = [vp, vp, vp, vp, vp]
        L.orc_pair_batch.argtypes = [vp, C.c_int64, vp, C.c_int64, vp, vp, vp]
        L.orc_render.argtypes = [vp, vp, vp, C.c_int, C.c_int, vp, vp, vp, vp, vp]
        L.orc_render.restype = C.c_int
        L.orc_render_supersampled.argtypes = [vp, vp, vp, C.c_int64, vp, C.c_int, vp]
        L.orc_bake_rho2.argtypes = [vp, vp, C.c_int32, C.c_float, C.c_int, vp]
        L.orc_grad.argtypes = [vp, vp, vp, vp, vp, C.c_int, vp, vp, vp, vp, vp]
        _LIB = L
    return _LIB


def _ptr(a):
    return C.c_void_p(a.ctypes.data) if a is not None else C.c_void_p(0)


def _cam(cam: dict) -> _Camera:
    c = _Camera()
    c.model = cam["model"]
    c.full_w, c.full_h = cam["full_w"], cam["full_h"]
    c.crop_x0, c.crop_y0, c.crop_w, c.crop_h = cam["crop"]
    c.fx, c.fy, c.cx, c.cy = cam["fx"], cam["fy"], cam["cx"], cam["cy"]
    c.k[:] = list(cam["k"])
    c.R_c2w[:] = [float(v) for row in cam["R_c2w"] for v in row]
    c.origin[:] = list(cam["origin"])
    c.theta_max = cam["theta_max"]
    return c


class _Scene:
    """Keeps float32 contiguous copies alive while the C struct points at them."""

    def __init__(self, scene: dict):
        self.arrays = {k: np.ascontiguousarray(scene[k], dtype=np.float32)
                       for k in ("means", "log_scales", "quats", "opacity_logits", "color")}
        rho2 = scene.get("rho2")
        self.arrays["rho2"] = None if rho2 is None else np.ascontiguousarray(rho2, dtype=np.float32)
        g = _Gaussians()
        g.n = int(scene["n"])
        g.color_mode = int(scene["color_mode"])
        for k, v in self.arrays.items():
            setattr(g, k, v.ctypes.data if v is not None else None)
        self.c = g


def _byref(x):
    return C.cast(C.pointer(x), C.c_void_p)


def render(scene: dict, cam: dict, opts: Opts = None, mode: str = "brute", n_threads: int = 0,
           with_alt: bool = False):
    """Render one view.  Returns dict(rgba [h, w, 4], n_dec [h, w], alt [h, w, N_ALT, 4]
    (if with_alt), n_contrib [h, w], skip [h, w])."""
    opts = opts or Opts()
    s = _Scene(scene)
    c = _cam(cam)
    o = opts._c()
    h, w = cam["crop"][3], cam["crop"][2]
    rgba = np.zeros((h, w, 4), np.float64)
    n_dec = np.zeros((h, w), np.int32)
    n_contrib = np.zeros((h, w), np.int64)
    skip = np.zeros((h, w), np.uint8)
    alt = np.zeros((h, w, N_ALT, 4), np.float64) if with_alt else None
    rc = lib().orc_render(_byref(s.c), _byref(c), _byref(o), 0 if mode == "brute" else 1, int(n_threads),
                          _ptr(rgba), _ptr(n_dec), _ptr(alt), _ptr(n_contrib), _ptr(skip))
    assert rc == 0
    out = {"rgba": rgba, "n_dec": n_dec, "n_contrib": n_contrib, "skip": skip.astype(bool)}
    if with_alt:
        out["alt"] = alt
    return out


def render_supersampled(scene: dict, cam: dict, jitter: np.ndarray, opts: Opts = None, n_threads: int = 0):
    """Eq. 5 reference: mean of centre-ray renders over the sub-pixel offsets ``jitter``."""
    opts = opts or Opts()
    s = _Scene(scene)
    c = _cam(cam)
    o = opts._c()
    j = np.ascontiguousarray(jitter, dtype=np.float64)
    h, w = cam["crop"][3], cam["crop"][2]
    rgba = np.zeros((h, w, 4), np.float64)
    lib().orc_render_supersampled(_byref(s.c), _byref(c), _byref(o), j.shape[0], _ptr(j), int(n_threads),
                                  _ptr(rgba))
    return rgba


def unproject(cam: dict, px, py):
    px = np.ascontiguousarray(px, dtype=np.float64).ravel()
    py = np.ascontiguousarray(py, dtype=np.float64).ravel()
    n = px.size
    d = np.zeros((n, 3), np.float64)
    v = np.zeros(n, np.uint8)
    c = _cam(cam)
    lib().orc_unproject(_byref(c), n, _ptr(px), _ptr(py), _ptr(d), _ptr(v))
    return d, v.astype(bool)


def project(cam: dict, dirs):
    dirs = np.ascontiguousarray(dirs, dtype=np.float64).reshape(-1, 3)
    n = dirs.shape[0]
    px = np.zeros(n, np.float64)
    py = np.zeros(n, np.float64)
    v = np.zeros(n, np.uint8)
    c = _cam(cam)
    lib().orc_project(_byref(c), n, _ptr(dirs), _ptr(px), _ptr(py), _ptr(v))
    return px, py, v.astype(bool)


def pixel_rays(cam: dict):
    """(rays [h, w, 9] = d, d_x, d_y, valid [h, w]) for the crop window."""
    h, w = cam["crop"][3], cam["crop"][2]
    out = np.zeros((h, w, 9), np.float64)
    v = np.zeros((h, w), np.uint8)
    c = _cam(cam)
    lib().orc_pixel_rays(_byref(c), _ptr(out), _ptr(v))
    return out, v.astype(bool)


def pair_batch(scene: dict, gi: int, origin, rays, opts: Opts = None):
    """Response of Gaussian ``gi`` to rays [n, 9] = (d, d_x, d_y) from ``origin``.
    Returns [n, 4] = (T, T ignoring t_near, t*, D^2)."""
    opts = opts or Opts()
    s = _Scene(scene)
    o = opts._c()
    rays = np.ascontiguousarray(rays, dtype=np.float64).reshape(-1, 9)
    org = np.ascontiguousarray(origin, dtype=np.float64)
    out = np.zeros((rays.shape[0], 4), np.float64)
    lib().orc_pair_batch(_byref(s.c), int(gi), _ptr(org), rays.shape[0], _ptr(rays), _byref(o), _ptr(out))
    return out


def preprocess(scene: dict, origin, opts: Opts = None):
    """Per Gaussian: (s'[3], sigma_eff, rgb[3], depth key) [n, 8] and W [n, 3, 3]."""
    opts = opts or Opts()
    s = _Scene(scene)
    o = opts._c()
    org = np.ascontiguousarray(origin, dtype=np.float32)
    n = int(scene["n"])
    out = np.zeros((n, 8), np.float64)
    W = np.zeros((n, 3, 3), np.float64)
    lib().orc_preprocess(_byref(s.c), _ptr(org), _byref(o), _ptr(out), _ptr(W))
    return out, W


def sh_basis(direction):
    d = np.ascontiguousarray(direction, dtype=np.float64)
    Y = np.zeros(16, np.float64)
    lib().orc_sh_basis(_ptr(d), _ptr(Y))
    return Y


def bake_rho2(scene: dict, cams, t_near: float = 0.2, n_threads: int = 0):
    """Eq. 11 floor variance per Gaussian over the views ``cams`` (float64 [n])."""
    s = _Scene(scene)
    arr = (_Camera * len(cams))(*[_cam(c) for c in cams])
    out = np.zeros(int(scene["n"]), np.float64)
    lib().orc_bake_rho2(_byref(s.c), C.cast(arr, C.c_void_p), len(cams), float(t_near), int(n_threads), _ptr(out))
    return out


def grad(scene: dict, cams, grad_rgba, opts: Opts = None, skip=None, n_threads: int = 0):
    """Gradients of sum(grad_rgba * render) w.r.t. the raw parameters, summed over
    views.  ``grad_rgba`` / ``skip`` are lists (one [h, w, 4] / [h, w] per view)."""
    opts = opts or Opts()
    if isinstance(cams, dict):
        cams, grad_rgba, skip = [cams], [grad_rgba], [skip]
    if skip is None:
        skip = [None] * len(cams)
    s = _Scene(scene)
    o = opts._c()
    n = int(scene["n"])
    ncol = 3 if scene["color_mode"] == 0 else 48
    out = {"means": np.zeros((3, n)), "log_scales": np.zeros((3, n)), "quats": np.zeros((4, n)),
           "opacity_logits": np.zeros(n), "color": np.zeros((ncol, n))}
    for cam, g, sk in zip(cams, grad_rgba, skip):
        c = _cam(cam)
        g = np.ascontiguousarray(g, dtype=np.float32)
        skc = None if sk is None else np.ascontiguousarray(sk, dtype=np.uint8)
        rc = lib().orc_grad(_byref(s.c), _byref(c), _byref(o), _ptr(g), _ptr(skc), int(n_threads),
                            _ptr(out["means"]), _ptr(out["log_scales"]), _ptr(out["quats"]),
                            _ptr(out["opacity_logits"]), _ptr(out["color"]))
        if rc != 0:
            raise ValueError("the gradient oracle follows the per-Gaussian key order only (order_mode 0)")
    return out
