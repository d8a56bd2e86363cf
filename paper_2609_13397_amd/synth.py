"""Seeded synthetic scenes, cameras and request traces.

This module only draws inputs: Gaussian parameters in their raw (pre-activation)
form and camera descriptions. It holds none of the rendering arithmetic, so the
FP64 oracle and the HIP path can both consume its output without sharing any
computation. Every draw goes through ``numpy.random.Generator(PCG64(seed))`` so a
seed always gives identical bytes.

Scene parameters follow the paper's Gaussian (Sec. 3): a mean, a rotation (unit
quaternion w,x,y,z), three scales (stored as log-scales), an opacity (stored as a
logit), a colour (RGB, or degree-3 spherical-harmonic coefficients) and the
per-Gaussian floor variance rho^2 of Eq. 10 (zero until baked).

Arrays are component-major (``[C][N]`` contiguous float32), the layout the C ABI
takes.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

PINHOLE = 0
FISHEYE_KB = 1
EQUIRECT = 2

MODEL_NAMES = {PINHOLE: "pinhole", FISHEYE_KB: "fisheye_kb", EQUIRECT: "equirect"}

SH_COEFFS = 16  # degree 3: (l, m) for l = 0..3, m = -l..l


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# --------------------------------------------------------------------------- scenes

def _random_quats(rng: np.random.Generator, n: int) -> np.ndarray:
    """Uniform rotations: a normalised 4-D standard normal is uniform on S^3."""
    q = rng.standard_normal((4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    return q.astype(np.float32)


def _cluster_means(rng: np.random.Generator, n: int, n_clusters: int = 32,
                   half_box: float = 5.0) -> np.ndarray:
    """Means drawn from anisotropic Gaussian clusters inside a cube of side 2*half_box.

    Cluster centres ~ U[-half_box, half_box]^3; per-axis cluster std ~ U[0.2, 1.5];
    cluster orientation uniform; membership uniform; points that fall outside the
    box are redrawn from their cluster.
    """
    centres = rng.uniform(-half_box, half_box, size=(n_clusters, 3))
    stds = rng.uniform(0.2, 1.5, size=(n_clusters, 3))
    rots = []
    for _ in range(n_clusters):
        m = rng.standard_normal((3, 3))
        qm, rm = np.linalg.qr(m)
        qm = qm * np.sign(np.diag(rm))[None, :]
        if np.linalg.det(qm) < 0:
            qm[:, 0] = -qm[:, 0]
        rots.append(qm)
    rots = np.stack(rots)
    member = rng.integers(0, n_clusters, size=n)
    out = np.empty((n, 3))
    todo = np.arange(n)
    while todo.size:
        z = rng.standard_normal((todo.size, 3))
        c = member[todo]
        pts = centres[c] + np.einsum("nij,nj->ni", rots[c], z * stds[c])
        inside = np.all(np.abs(pts) <= half_box, axis=1)
        out[todo[inside]] = pts[inside]
        todo = todo[~inside]
    return out.T.astype(np.float32)


def make_scene(n: int, seed: int, layout: str = "uniform", color: str = "rgb",
               log_scale_mean: float = -3.0, log_scale_std: float = 0.5,
               sh_std: float = 0.3) -> dict:
    """A seeded scene of ``n`` Gaussians.

    layout "uniform": means ~ U[-1,1]^3.  layout "clusters": 32 anisotropic clusters
    in a 10 m box.  color "rgb": RGB ~ U[0,1]; "sh3": 48 SH coefficients ~ N(0, sh_std)
    (16 coefficients x 3 channels, coefficient-major: index = 3*coef + channel).
    """
    rng = _rng(seed)
    if layout == "uniform":
        means = rng.uniform(-1.0, 1.0, size=(3, n)).astype(np.float32)
    elif layout == "clusters":
        means = _cluster_means(rng, n)
    else:
        raise ValueError(f"unknown layout {layout!r}")
    log_scales = rng.normal(log_scale_mean, log_scale_std, size=(3, n)).astype(np.float32)
    quats = _random_quats(rng, n)
    opacity_logits = rng.standard_normal(n).astype(np.float32)
    if color == "rgb":
        col = rng.uniform(0.0, 1.0, size=(3, n)).astype(np.float32)
        color_mode = 0
    elif color == "sh3":
        col = rng.normal(0.0, sh_std, size=(3 * SH_COEFFS, n)).astype(np.float32)
        color_mode = 3
    else:
        raise ValueError(f"unknown color {color!r}")
    return {
        "n": n,
        "color_mode": color_mode,
        "means": np.ascontiguousarray(means),
        "log_scales": np.ascontiguousarray(log_scales),
        "quats": np.ascontiguousarray(quats),
        "opacity_logits": np.ascontiguousarray(opacity_logits),
        "color": np.ascontiguousarray(col),
        "rho2": np.zeros(n, dtype=np.float32),
    }


def perturb_scene(scene: dict, seed: int, mean_std: float = 0.01, color_std: float = 0.1) -> dict:
    """A copy of ``scene`` with N(0, mean_std) added to the means and N(0, color_std)
    to the colour coefficients (the training-step target scene)."""
    rng = _rng(seed)
    out = dict(scene)
    out["means"] = (scene["means"] + rng.normal(0, mean_std, scene["means"].shape)).astype(np.float32)
    out["color"] = (scene["color"] + rng.normal(0, color_std, scene["color"].shape)).astype(np.float32)
    return out


def subset_scene(scene: dict, idx: np.ndarray) -> dict:
    out = {"n": int(len(idx)), "color_mode": scene["color_mode"]}
    for k in ("means", "log_scales", "quats", "color"):
        out[k] = np.ascontiguousarray(scene[k][:, idx])
    for k in ("opacity_logits", "rho2"):
        out[k] = np.ascontiguousarray(scene[k][idx])
    return out


# --------------------------------------------------------------------------- cameras

def look_at(origin, target, up=(0.0, 0.0, 1.0)) -> np.ndarray:
    """Camera-to-world rotation with OpenCV camera axes (x right, y down, z forward).

    z_c = normalise(target - origin); x_c = normalise(z_c x up); y_c = z_c x x_c.
    Returned row-major 3x3 with the camera axes as columns.
    """
    o = np.asarray(origin, dtype=np.float64)
    t = np.asarray(target, dtype=np.float64)
    u = np.asarray(up, dtype=np.float64)
    z = t - o
    z /= np.linalg.norm(z)
    x = np.cross(z, u)
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    return np.stack([x, y, z], axis=1)


def camera(model: int, full_w: int, full_h: int, *, fx=0.0, fy=0.0, cx=0.0, cy=0.0,
           k=(0.0, 0.0, 0.0, 0.0), R_c2w=None, origin=(0.0, 0.0, 0.0), theta_max=0.0,
           crop=None) -> dict:
    """A camera description (plain values; both renderers build their own struct).

    ``crop`` = (x0, y0, w, h) selects the rendered window of the full virtual image.
    """
    if R_c2w is None:
        R_c2w = np.eye(3)
    if crop is None:
        crop = (0, 0, full_w, full_h)
    return {
        "model": int(model), "full_w": int(full_w), "full_h": int(full_h),
        "crop": tuple(int(c) for c in crop),
        "fx": float(fx), "fy": float(fy), "cx": float(cx), "cy": float(cy),
        "k": tuple(float(v) for v in k),
        "R_c2w": np.asarray(R_c2w, dtype=np.float64).reshape(3, 3).tolist(),
        "origin": tuple(float(v) for v in origin),
        "theta_max": float(theta_max),
    }


def scale_camera(cam: dict, s: float) -> dict:
    """Calibration scaled with resolution (the paper's zoom convention, Sec. 5):
    the full virtual image becomes round(s*W) x round(s*H) and fx, fy, cx, cy scale by s.
    The crop becomes the whole scaled image."""
    w = int(round(cam["full_w"] * s))
    h = int(round(cam["full_h"] * s))
    out = dict(cam)
    out.update(full_w=w, full_h=h, crop=(0, 0, w, h), fx=cam["fx"] * s, fy=cam["fy"] * s,
               cx=cam["cx"] * s, cy=cam["cy"] * s)
    return out


def with_crop(cam: dict, x0: int, y0: int, w: int, h: int) -> dict:
    out = dict(cam)
    out["crop"] = (int(x0), int(y0), int(w), int(h))
    return out


def _kb_poly_np(k, th):
    t2 = th * th
    return th * (1 + k[0] * t2 + k[1] * t2 ** 2 + k[2] * t2 ** 3 + k[3] * t2 ** 4)


def draw_kb_coeffs(seed: int, theta_max: float, lo: float = -0.05, hi: float = 0.05):
    """k1..k4 ~ U[lo, hi], redrawn until theta_d(theta) is strictly increasing on
    [0, theta_max] (checked on a dense grid with a positive-slope margin)."""
    rng = _rng(seed)
    th = np.linspace(0.0, theta_max, 20001)
    tries = 0
    while True:
        tries += 1
        k = rng.uniform(lo, hi, size=4)
        t2 = th * th
        slope = 1 + 3 * k[0] * t2 + 5 * k[1] * t2 ** 2 + 7 * k[2] * t2 ** 3 + 9 * k[3] * t2 ** 4
        if np.all(slope > 1e-3):
            return tuple(float(np.float32(v)) for v in k), tries


def kb_camera(full_w, full_h, theta_max_deg, k, radius_px, R_c2w, origin, crop=None) -> dict:
    """Equidistant Kannala-Brandt fisheye whose image circle (theta = theta_max) has
    the given pixel radius, centred in the image."""
    tm = math.radians(theta_max_deg)
    f = radius_px / float(_kb_poly_np(k, tm))
    return camera(FISHEYE_KB, full_w, full_h, fx=f, fy=f, cx=full_w / 2.0, cy=full_h / 2.0,
                  k=k, R_c2w=R_c2w, origin=origin, theta_max=tm, crop=crop)


# --------------------------------------------------------------------------- workloads

def orbit_views(n_views=8, radius=12.0, height=3.0, w=1920, h=1080, f=1371.0):
    """Pinhole views on a circular orbit looking at the origin (world up +z)."""
    cams = []
    for i in range(n_views):
        phi = 2 * math.pi * i / n_views
        o = (radius * math.cos(phi), radius * math.sin(phi), height)
        cams.append(camera(PINHOLE, w, h, fx=f, fy=f, cx=w / 2.0, cy=h / 2.0,
                           R_c2w=look_at(o, (0, 0, 0)), origin=o))
    return cams


def tiny_config():
    """256 Gaussians in U[-1,1]^3, RGB, one 64x48 pinhole (f = 60) at z = -3 looking +z."""
    scene = make_scene(256, seed=1, layout="uniform", color="rgb",
                       log_scale_mean=-3.0, log_scale_std=0.5)
    cam = camera(PINHOLE, 64, 48, fx=60.0, fy=60.0, cx=32.0, cy=24.0,
                 R_c2w=np.eye(3), origin=(0.0, 0.0, -3.0))
    return scene, cam


def pinhole_config(n=100_000, seed=2):
    """Cluster scene with SH colour; 8 orbit views at 1920x1080 (plus scaled copies)."""
    scene = make_scene(n, seed=seed, layout="clusters", color="sh3",
                       log_scale_mean=-4.0, log_scale_std=0.7)
    return scene, orbit_views()


def fisheye_cameras():
    """190-degree KB fisheye 1600x1600 and a 2048x1024 equirectangular view, both at
    the origin looking along +x."""
    k, _ = draw_kb_coeffs(31, math.radians(95.0))
    R = look_at((0, 0, 0), (1, 0, 0))
    kb = kb_camera(1600, 1600, 95.0, k, 800.0, R, (0.0, 0.0, 0.0))
    eq = camera(EQUIRECT, 2048, 1024, R_c2w=R, origin=(0.0, 0.0, 0.0))
    return [kb, eq]


def fisheye_config(n=1_000_000, seed=3):
    scene = make_scene(n, seed=seed, layout="clusters", color="sh3",
                       log_scale_mean=-4.0, log_scale_std=0.7)
    return scene, fisheye_cameras()


def training_cameras(scale: float = 1.0):
    """Two orbit pinholes (phi = 0, pi/2; f = 914) and two centre KB fisheyes looking
    along +x and -x, all 1280x720 (times ``scale``)."""
    cams = []
    for phi in (0.0, math.pi / 2):
        o = (12 * math.cos(phi), 12 * math.sin(phi), 3.0)
        cams.append(camera(PINHOLE, 1280, 720, fx=914.0, fy=914.0, cx=640.0, cy=360.0,
                           R_c2w=look_at(o, (0, 0, 0)), origin=o))
    k, _ = draw_kb_coeffs(31, math.radians(95.0))
    for tgt in ((1, 0, 0), (-1, 0, 0)):
        cams.append(kb_camera(1280, 720, 95.0, k, 640.0, look_at((0, 0, 0), tgt), (0.0, 0.0, 0.0)))
    if scale != 1.0:
        cams = [scale_camera(c, scale) for c in cams]
    return cams


def training_config(n=1_000_000, seed=4):
    scene = make_scene(n, seed=seed, layout="clusters", color="sh3",
                       log_scale_mean=-4.0, log_scale_std=0.7)
    target_scene = perturb_scene(scene, seed=41)
    return scene, target_scene, training_cameras()


@dataclass
class Request:
    rid: int
    arrival_s: float
    scene: int
    camera: dict
    pixels: int = field(init=False)

    def __post_init__(self):
        self.pixels = self.camera["crop"][2] * self.camera["crop"][3]


def serving_base_cameras():
    """The three base cameras of the serving mix: an orbit pinhole 1920x1080, the
    centre KB fisheye 1600x1600 and the centre equirect 2048x1024."""
    pin = orbit_views(1)[0]
    kb, eq = fisheye_cameras()
    return [pin, kb, eq]


def serving_trace(n_requests: int, qps: float, seed: int, n_scenes: int = 3,
                  scales=(0.125, 0.25, 0.5, 1.0, 2.0, 4.0, 8.0)):
    """Poisson arrivals at ``qps``; scene uniform; camera model uniform over the three
    base cameras (each with a random orbit angle / yaw); scale uniform over
    ``scales``.  For scale > 1 the request renders a random crop of the base size out
    of the scaled virtual image."""
    rng = _rng(seed)
    base = serving_base_cameras()
    t = 0.0
    reqs = []
    for rid in range(n_requests):
        t += rng.exponential(1.0 / qps)
        sc = int(rng.integers(0, n_scenes))
        m = int(rng.integers(0, 3))
        s = float(scales[int(rng.integers(0, len(scales)))])
        yaw = float(rng.uniform(0, 2 * math.pi))
        cam = dict(base[m])
        if m == 0:
            o = (12 * math.cos(yaw), 12 * math.sin(yaw), 3.0)
            cam = camera(PINHOLE, 1920, 1080, fx=1371.0, fy=1371.0, cx=960.0, cy=540.0,
                         R_c2w=look_at(o, (0, 0, 0)), origin=o)
        else:
            tgt = (math.cos(yaw), math.sin(yaw), 0.0)
            R = look_at((0, 0, 0), tgt)
            cam = dict(cam)
            cam["R_c2w"] = R.tolist()
        bw, bh = cam["full_w"], cam["full_h"]
        cam = scale_camera(cam, s)
        if s > 1.0:
            x0 = int(rng.integers(0, cam["full_w"] - bw + 1))
            y0 = int(rng.integers(0, cam["full_h"] - bh + 1))
            cam = with_crop(cam, x0, y0, bw, bh)
        reqs.append(Request(rid, t, sc, cam))
    return reqs


def mc_jitter(k: int, seed: int) -> np.ndarray:
    """k x k stratified-jittered offsets in [-1/2, 1/2]^2, shape (k*k, 2)."""
    rng = _rng(seed)
    ii, jj = np.meshgrid(np.arange(k), np.arange(k), indexing="ij")
    u = rng.uniform(0, 1, size=(2, k, k))
    x = (ii + u[0]) / k - 0.5
    y = (jj + u[1]) / k - 0.5
    return np.stack([x.ravel(), y.ravel()], axis=1)


def seeded_image(shape, seed: int, lo=-1.0, hi=1.0) -> np.ndarray:
    """A seeded random float32 array (upstream gradients, targets)."""
    return _rng(seed).uniform(lo, hi, size=shape).astype(np.float32)
