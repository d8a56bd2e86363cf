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
