"""GPU parity of the per-ray compositing order (order_mode RAY: each pixel composites
its pairs by their own t* along its ray) against the FP64 oracle's order_mode 1.

The kernel's order is exact whatever the density: a pixel whose pending buffer fills
defers the pairs with the largest keys and walks its tile list again for them.  Every
case is held to the 2e-4 bar against the oracle, with its near-tie order decisions as
alternatives, sparse scenes (nothing deferred) and dense ones (many deferrals) alike.
"""
import math
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2609_13397_amd import synth
from parity import compare_image

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _render(scene, cams, **kw):
    import torch
    from paper_2609_13397_amd import render as R
    sc = R.Scene.from_numpy(scene)
    rgba, info, _ = R.render_forward(sc, cams, R.RenderOpts(**kw))
    torch.cuda.synchronize()
    return [v.cpu().numpy().astype(np.float64) for v in R.split_views(rgba, cams)], info


def _check(img, scene, cam, mode="brute", **kw):
    ref = O.render(scene, cam, O.Opts(**kw), mode=mode, with_alt=True)
    nfail, worst, det = compare_image(img, ref)
    _say(f"   parity: fail={nfail} worst={worst:.3e} {det}")
    assert nfail == 0, (worst, det)


@pytest.mark.parametrize("kw", [dict(filter_mode=1), dict(filter_mode=0), dict(filter_mode=2),
                                dict(filter_mode=1, use_floor=1)],
                         ids=["aniso", "centre", "iso", "aniso_floor"])
def test_tiny_ray_order_parity(kw):
    """256 Gaussians in the unit cube (config 1 scene) seen by the config-1 pinhole and a
    ragged crop: many overlapping Gaussians, so key and ray order differ often."""
    scene, cam = synth.tiny_config()
    scene = dict(scene)
    if kw.get("use_floor"):
        scene["rho2"] = O.bake_rho2(scene, [synth.scale_camera(cam, 2.0)]).astype(np.float32)
    ragged = synth.camera(synth.PINHOLE, 90, 60, fx=45.0, fy=45.0, cx=44.0, cy=31.0,
                          origin=(0.1, -0.1, -3.0), crop=(7, 11, 70, 37))
    _say(f"tiny ray order {kw}")
    imgs, info = _render(scene, [cam, ragged], order_mode=1, **kw)
    _say(f"   pairs {info['n_pairs']} overflow {info['n_order_overflow']}")
    assert info["n_order_overflow"] == 0
    key, _ = _render(scene, [cam], order_mode=0, **kw)
    assert np.abs(key[0] - imgs[0]).max() > 1e-4  # the two orders really differ here
    for img, c in zip(imgs, [cam, ragged]):
        _check(img, scene, c, order_mode=1, **kw)


def _wide_scene(n, spread):
    scene = synth.make_scene(n, seed=22, layout="clusters", color="sh3", log_scale_mean=-3.0, log_scale_std=0.6)
    scene["means"] *= spread
    kb, eq = synth.fisheye_cameras()
    cams = [synth.scale_camera(kb, 1 / 16), synth.scale_camera(eq, 1 / 16)]
    for c in cams:
        c["origin"] = (0.0, -1.0, 0.3)
    scene["rho2"] = O.bake_rho2(scene, [synth.scale_camera(c, 2.0) for c in cams]).astype(np.float32)
    return scene, cams


def test_fisheye_equirect_ray_order_parity():
    """Wide cameras (190-degree KB fisheye, equirect) around 1000 clustered Gaussians,
    floor on; sparse enough that no pixel's pending buffer overflows."""
    scene, cams = _wide_scene(1000, 0.6)
    _say("fisheye + equirect ray order")
    imgs, info = _render(scene, cams, order_mode=1, use_floor=True)
    _say(f"   pairs {info['n_pairs']} overflow {info['n_order_overflow']}")
    assert info["n_order_overflow"] == 0
    for img, c in zip(imgs, cams):
        _check(img, scene, c, order_mode=1, use_floor=1)


@pytest.mark.parametrize("kw", [dict(use_floor=True), dict(filter_mode=0), dict(filter_mode=2, use_floor=True)],
                         ids=["aniso_floor", "centre", "iso_floor"])
def test_dense_scene_ray_order_parity(kw):
    """Dense clusters (2000 Gaussians in 0.3x the volume) fill the 16-entry pending
    buffer of many pixels: the deferred pairs are composited by further walks, and the
    image matches the oracle's exact per-ray order at the 2e-4 bar."""
    scene, cams = _wide_scene(2000, 0.3)
    ray, info = _render(scene, cams, order_mode=1, **kw)
    key, _ = _render(scene, cams, order_mode=0, **kw)
    _say(f"   dense {kw}: deferred {info['n_order_overflow']}")
    assert info["n_order_overflow"] > 0
    okw = {k: int(v) if isinstance(v, bool) else v for k, v in kw.items()}
    for r, k, c in zip(ray, key, cams):
        assert np.abs(r - k).max() > 1e-3  # the two orders differ visibly here
        _check(r, scene, c, order_mode=1, **okw)


def test_two_gaussian_closed_form_on_gpu():
    """The closed-form case of the oracle's pins: A at (0, 0, 5), B at (0.25, 0, 4.995),
    isotropic s = 0.1, centre-ray filter; key order A, B and ray order B, A."""
    s = 0.1
    la, lb = 0.4, 1.4
    scene = {
        "n": 2, "color_mode": 0,
        "means": np.array([[0.0, 0.25], [0.0, 0.0], [5.0, 4.995]], np.float32),
        "log_scales": np.full((3, 2), math.log(s), np.float32),
        "quats": np.array([[1.0, 1.0], [0.0, 0.0], [0.0, 0.0], [0.0, 0.0]], np.float32),
        "opacity_logits": np.array([la, lb], np.float32),
        "color": np.array([[1.0, 0.0], [0.0, 1.0], [0.0, 0.0]], np.float32),
        "rho2": np.zeros(2, np.float32),
    }
    cam = synth.camera(synth.PINHOLE, 65, 49, fx=60.0, fy=60.0, cx=32.5, cy=24.5)
    sig = lambda x: 1.0 / (1.0 + math.exp(-float(np.float32(x))))
    s32 = math.exp(float(np.float32(math.log(s))))
    aA = sig(la)
    aB = sig(lb) * math.exp(-0.5 * (float(np.float32(0.25)) / s32) ** 2)
    (key,), _ = _render(scene, [cam], filter_mode=0, order_mode=0)
    (ray,), info = _render(scene, [cam], filter_mode=0, order_mode=1)
    assert info["n_order_overflow"] == 0
    np.testing.assert_allclose(key[24, 32, :3], [aA, aB * (1 - aA), 0.0], atol=2e-6)
    np.testing.assert_allclose(ray[24, 32, :3], [aA * (1 - aB), aB, 0.0], atol=2e-6)


def test_deep_stack_defers_and_stays_exact():
    """A deep stack of 40 nearly coplanar wide Gaussians on one ray fills the 16-entry
    pending buffer: pairs are deferred (counted) and composited by later walks, and the
    image equals the oracle's exact per-ray order."""
    n = 40
    rng = np.random.default_rng(3)
    scene = {
        "n": n, "color_mode": 0,
        "means": np.stack([rng.normal(0, 0.01, n), rng.normal(0, 0.01, n), 5.0 + rng.normal(0, 0.002, n)]).astype(
            np.float32),
        "log_scales": np.tile(np.array([[-1.0], [-1.0], [-6.0]], np.float32), (1, n)),
        "quats": rng.normal(0, 1, (4, n)).astype(np.float32),
        "opacity_logits": np.full(n, -3.0, np.float32),
        "color": rng.uniform(0, 1, (3, n)).astype(np.float32),
        "rho2": np.zeros(n, np.float32),
    }
    cam = synth.camera(synth.PINHOLE, 32, 32, fx=40.0, fy=40.0, cx=16.0, cy=16.0)
    (img,), info = _render(scene, [cam], filter_mode=1, order_mode=1)
    _say(f"   deferred {info['n_order_overflow']}")
    assert info["n_order_overflow"] > 0
    _check(img, scene, cam, filter_mode=1, order_mode=1)


@pytest.mark.parametrize("case", ["camera_away_from_origin", "near_tied_keys", "separated_keys"])
@pytest.mark.parametrize("filter_mode", [0, 1])
def test_key_order_two_gaussians_against_oracle(case, filter_mode):
    """The per-Gaussian key order (order_mode KEY) on the two-Gaussian scenes of the
    oracle's order pins: a turned camera away from the world origin (the key is |mu - o|,
    not |mu|), two Gaussians whose keys agree within float32 rounding (either order is
    accepted; the oracle offers the swapped composite), and the same pair well apart."""
    from test_oracle_order import _two_gaussian_frame
    if case == "camera_away_from_origin":
        R = synth.look_at((0, 0, 0), (0.3, -1.0, 0.4))
        o = -10.0 * R[:, 0] + np.array([0.7, -0.4, 1.1])
        b_cam = (0.25, 0, 4.995)
    else:
        R = synth.look_at((0, 0, 0), (-0.6, 0.2, 1.0))
        o = np.array([1.25, -3.5, 2.0])
        b_cam = (3.2e-3 if case == "near_tied_keys" else 0.05, 0, 5.0)
    scene, cam, *_ = _two_gaussian_frame(o, R, (0, 0, 5.0), b_cam, 0.4, 1.4)
    _say(f"two-Gaussian key order {case} filter {filter_mode}")
    imgs, _ = _render(scene, [cam], order_mode=0, filter_mode=filter_mode)
    _check(imgs[0], scene, cam, order_mode=0, filter_mode=filter_mode)
