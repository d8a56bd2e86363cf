"""Pins of the oracle's per-ray compositing order (order_mode 1): Gaussians composited
front to back by each pair's own max-response depth t* along the pixel's ray (Sec. 3,
Eq. 4), instead of one per-Gaussian key |mu - o| per view.

The expected values are written out from the closed forms of the centre-ray response
(Eq. 3 with C = 1: T = sigma exp(-D^2 / 2)) and of front-to-back compositing; they do
not call the oracle's pair arithmetic.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2609_13397_amd import synth


def _scene(mus, log_s, logits, rgbs):
    n = len(mus)
    return {
        "n": n, "color_mode": 0,
        "means": np.array(mus, np.float32).T.copy(),
        "log_scales": np.array(log_s, np.float32).T.copy(),
        "quats": np.tile(np.array([[1.0], [0.0], [0.0], [0.0]], np.float32), (1, n)),
        "opacity_logits": np.array(logits, np.float32),
        "color": np.array(rgbs, np.float32).T.copy(),
        "rho2": np.zeros(n, np.float32),
    }


def _sig(x):
    return 1.0 / (1.0 + math.exp(-float(np.float32(x))))


def _axis_camera():
    # the ray through the centre of pixel (32, 24) is exactly +z
    return synth.camera(synth.PINHOLE, 65, 49, fx=60.0, fy=60.0, cx=32.5, cy=24.5, origin=(0.0, 0.0, 0.0))


def test_key_order_and_ray_order_differ_closed_form():
    """Two isotropic Gaussians on and near the +z ray.  A at (0, 0, 5) has |mu - o| = 5
    and t* = 5; B at (0.25, 0, 4.995) has |mu - o| = 5.00125 > 5 but t* = 4.995 < 5 (for
    an isotropic Gaussian t* is the projection of mu - o on the ray).  The key order is
    A, B and the ray order B, A; D_A = 0, D_B = 0.25 / s."""
    s = 0.1
    la, lb = 0.4, 1.4
    scene = _scene([(0.0, 0.0, 5.0), (0.25, 0.0, 4.995)], [(math.log(s),) * 3] * 2, [la, lb],
                   [(1.0, 0.0, 0.0), (0.0, 1.0, 0.0)])
    cam = _axis_camera()
    s32 = math.exp(float(np.float32(math.log(s))))
    # centre-ray response (Eq. 3, C = 1): D is the whitened perpendicular distance
    aA = _sig(la)
    aB = _sig(lb) * math.exp(-0.5 * (float(np.float32(0.25)) / s32) ** 2)
    for mode, first, second in ((0, ("A", aA), ("B", aB)), (1, ("B", aB), ("A", aA))):
        ref = O.render(scene, cam, O.Opts(filter_mode=0, order_mode=mode), with_alt=True)
        px = ref["rgba"][24, 32]
        col = {"A": np.array([1.0, 0.0, 0.0]), "B": np.array([0.0, 1.0, 0.0])}
        expect_rgb = col[first[0]] * first[1] + col[second[0]] * second[1] * (1.0 - first[1])
        expect_a = 1.0 - (1.0 - aA) * (1.0 - aB)
        np.testing.assert_allclose(px[:3], expect_rgb, rtol=0, atol=1e-12)
        assert px[3] == pytest.approx(expect_a, abs=1e-12)
        assert ref["n_dec"][24, 32] == 0
    # the two orders give visibly different colours
    assert abs(aA * (1 - aB) - aA) > 1e-3


def test_orders_agree_when_depths_are_separated():
    """Gaussians whose depths are spaced far beyond their extent: every ray meets them in
    the key order, so both orders composite identically (bitwise)."""
    rng = np.random.default_rng(5)
    n = 24
    # spacing 1.0 against |t* - |mu - o|| <= s'_max D_max ~ 0.1 * 3.4 for these scales
    z = 2.0 + 1.0 * np.arange(n)
    mus = np.stack([rng.uniform(-0.1, 0.1, n) * z, rng.uniform(-0.1, 0.1, n) * z, z], 1)
    log_s = np.clip(rng.normal(-3.0, 0.3, (n, 3)), -3.6, -2.4)
    rgbs = rng.uniform(0, 1, (n, 3))
    scene = _scene(mus.tolist(), log_s.tolist(), rng.normal(0, 1, n).tolist(), rgbs.tolist())
    scene["quats"] = rng.normal(0, 1, (4, n)).astype(np.float32)
    cam = synth.camera(synth.PINHOLE, 48, 40, fx=40.0, fy=40.0, cx=24.0, cy=20.0)
    a = O.render(scene, cam, O.Opts(filter_mode=1, order_mode=0))
    b = O.render(scene, cam, O.Opts(filter_mode=1, order_mode=1))
    assert (a["rgba"][..., 3] > 0.05).sum() > 20  # the scene is visible
    assert np.array_equal(a["rgba"], b["rgba"])


def test_order_effect_is_second_order_in_opacity():
    """Reordering changes C by terms in alpha_i alpha_j only: with every opacity scaled
    down to ~1e-3, both orders agree to O(alpha^2) while C itself is O(alpha)."""
    sc, cam = synth.tiny_config()
    sc = dict(sc)
    sc["opacity_logits"] = np.full(sc["n"], -7.0, np.float32)  # sigma ~ 9e-4
    op = dict(filter_mode=1, alpha_min=1e-6)
    a = O.render(sc, cam, O.Opts(order_mode=0, **op))["rgba"]
    b = O.render(sc, cam, O.Opts(order_mode=1, **op))["rgba"]
    assert a[..., :3].max() > 1e-4
    assert np.abs(a - b).max() < 5e-6


def test_gradient_oracle_refuses_ray_order():
    sc = _scene([(0.0, 0.0, 5.0)], [(-2.0,) * 3], [0.0], [(1.0, 1.0, 1.0)])
    cam = _axis_camera()
    g = np.zeros((49, 65, 4), np.float32)
    with pytest.raises(ValueError):
        O.grad(sc, [cam], [g], O.Opts(filter_mode=0, order_mode=1))


# ----------------------------------------------------------------------------- the key's origin

def _rotated_camera(o, R):
    """A 65x49 pinhole (f = 60) at ``o`` whose centre pixel (32, 24) looks along R's third
    column (the ray through that pixel centre is exactly R e_z)."""
    return synth.camera(synth.PINHOLE, 65, 49, fx=60.0, fy=60.0, cx=32.5, cy=24.5,
                        R_c2w=R, origin=tuple(o))


def _centre_ray_alpha(logit, mu32, o32, d32, s32):
    """Eq. 3 with C = 1 for an isotropic Gaussian: sigma exp(-D^2 / 2), D the perpendicular
    distance of the mean from the ray (o, d) divided by the scale."""
    v = np.asarray(mu32, np.float64) - np.asarray(o32, np.float64)
    d = np.asarray(d32, np.float64)
    perp = np.linalg.norm(np.cross(v, d)) / np.linalg.norm(d)
    return _sig(logit) * math.exp(-0.5 * (perp / s32) ** 2)


def _two_gaussian_frame(o, R, a_cam, b_cam, la, lb, s=0.1):
    """Gaussians A and B at camera-frame offsets a_cam, b_cam from o (world = o + R x),
    float32 as stored; returns the scene, the camera and the closed-form alphas."""
    o = np.asarray(o, np.float64)
    A = (o + R @ np.asarray(a_cam, np.float64)).astype(np.float32)
    B = (o + R @ np.asarray(b_cam, np.float64)).astype(np.float32)
    scene = _scene([tuple(A), tuple(B)], [(math.log(s),) * 3] * 2, [la, lb], [(1.0, 0.0, 0.0), (0.0, 1.0, 0.0)])
    cam = _rotated_camera(o, R)
    o32 = np.array(cam["origin"], np.float32)
    R32 = np.array(cam["R_c2w"], np.float32)
    d32 = R32[:, 2]
    s32 = math.exp(float(np.float32(math.log(s))))
    aA = _centre_ray_alpha(la, A, o32, d32, s32)
    aB = _centre_ray_alpha(lb, B, o32, d32, s32)
    keys = [float(np.sum((np.float64(P) - o32.astype(np.float64)) ** 2)) for P in (A, B)]
    return scene, cam, aA, aB, A, B, keys


def _composite(first, second):
    """Front-to-back composite of two (colour, alpha) pairs (Eq. 4, black background)."""
    (c1, a1), (c2, a2) = first, second
    return np.asarray(c1) * a1 + np.asarray(c2) * a2 * (1.0 - a1), 1.0 - (1.0 - a1) * (1.0 - a2)


RED, GREEN = (1.0, 0.0, 0.0), (0.0, 1.0, 0.0)


def test_key_is_distance_from_the_camera_centre():
    """The per-Gaussian key is |mu - o| for the view's own centre o, not |mu|.  A camera
    away from the world origin, turned, sees A on its centre ray at distance 5 and B
    0.25 m off it at depth 4.995 (|B - o| = 5.00125).  The key order is A, B and the
    per-ray order B, A, while the world distances |mu| order B before A: a key taken
    from |mu| (or from a camera at the origin) composites the wrong colour first."""
    R = synth.look_at((0, 0, 0), (0.3, -1.0, 0.4))
    o = -10.0 * R[:, 0] + np.array([0.7, -0.4, 1.1])
    scene, cam, aA, aB, A, B, keys = _two_gaussian_frame(o, R, (0, 0, 5.0), (0.25, 0, 4.995), 0.4, 1.4)
    assert keys[0] < keys[1]
    assert np.linalg.norm(np.float64(B)) < np.linalg.norm(np.float64(A)) - 0.1  # |mu| order is B, A
    for mode, first, second in ((0, (RED, aA), (GREEN, aB)), (1, (GREEN, aB), (RED, aA))):
        ref = O.render(scene, cam, O.Opts(filter_mode=0, order_mode=mode), with_alt=True)
        rgb, a = _composite(first, second)
        np.testing.assert_allclose(ref["rgba"][24, 32, :3], rgb, rtol=0, atol=1e-12)
        assert ref["rgba"][24, 32, 3] == pytest.approx(a, abs=1e-12)
        assert ref["n_dec"][24, 32] == 0
    # the two colours differ visibly, so a wrong key would fail above
    assert np.abs(_composite((RED, aA), (GREEN, aB))[0] - _composite((GREEN, aB), (RED, aA))[0]).max() > 0.01


def test_near_tied_keys_are_an_order_decision():
    """Two composited Gaussians whose keys |mu - o|^2 differ by less than float32 rounding
    of the key can be sorted either way by a renderer that rounds its key: the oracle
    flags the pixel and offers the swapped composite as the alternative.  Keys 3e-3 m
    apart across the ray (relative gap ~ 4e-7 in |mu - o|^2) are such a pair; 0.05 m apart
    (~ 1e-4) are not."""
    R = synth.look_at((0, 0, 0), (-0.6, 0.2, 1.0))
    o = np.array([1.25, -3.5, 2.0])
    for off, tied in ((3.2e-3, True), (0.05, False)):
        scene, cam, aA, aB, A, B, keys = _two_gaussian_frame(o, R, (0, 0, 5.0), (off, 0, 5.0), 0.4, 1.4)
        gap = (keys[1] - keys[0]) / keys[1]
        assert 0 < gap and ((gap < 1e-6) == tied)
        ref = O.render(scene, cam, O.Opts(filter_mode=0), with_alt=True)
        rgb, a = _composite((RED, aA), (GREEN, aB))
        np.testing.assert_allclose(ref["rgba"][24, 32, :3], rgb, rtol=0, atol=1e-12)
        assert ref["n_dec"][24, 32] == (1 if tied else 0)
        if tied:
            rgb2, a2 = _composite((GREEN, aB), (RED, aA))
            np.testing.assert_allclose(ref["alt"][24, 32, 0, :3], rgb2, rtol=0, atol=1e-12)
            assert ref["alt"][24, 32, 0, 3] == pytest.approx(a2, abs=1e-12)
            assert np.abs(rgb2 - rgb).max() > 0.1
