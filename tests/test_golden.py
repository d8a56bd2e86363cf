"""Closed-form fixtures (tests/golden/closed_forms.json): each stored value is re-derived
from its formula here, and the oracle is checked against it."""
import json
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2609_13397_amd import synth

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


def _scene_one(mu, log_s):
    return {"n": 1, "color_mode": 0, "means": np.array(mu, np.float32).reshape(3, 1),
            "log_scales": np.full((3, 1), log_s, np.float32), "quats": np.array([[1.0], [0], [0], [0]], np.float32),
            "opacity_logits": np.array([6.0], np.float32), "color": np.ones((3, 1), np.float32),
            "rho2": np.zeros(1, np.float32)}


@pytest.mark.parametrize("case", GOLD["on_axis_isotropic"]["cases"])
def test_on_axis_isotropic(case):
    f, t, ls = case["f"], case["t"], case["log_s"]
    s = math.exp(ls)
    a = math.atan(1 / (2 * f))
    val = 1 / (1 + (t / s) ** 2 * math.sin(a) ** 2 / 3)
    assert val == pytest.approx(case["T_over_sigma"], rel=1e-5)
    cam = synth.camera(synth.PINHOLE, 65, 49, fx=f, fy=f, cx=32.5, cy=24.5, origin=(0, 0, -t))
    rays, _ = O.pixel_rays(cam)
    T = O.pair_batch(_scene_one((0, 0, 0), ls), 0, (0, 0, -t), rays[24, 32][None])[0, 0]
    sig = 1 / (1 + math.exp(-6.0))
    assert T / sig == pytest.approx(case["T_over_sigma"], rel=1e-5)


@pytest.mark.parametrize("case", GOLD["moment_matching"]["cases"])
def test_moment_matching_values(case):
    a = case["a"]
    assert (math.sqrt(2 * math.pi) * math.erf(a / math.sqrt(2)) / (2 * a)) ** 2 == pytest.approx(case["box"], abs=1e-6)
    assert 1 / (1 + a * a / 3) == pytest.approx(case["moment_matched"], abs=1e-6)


@pytest.mark.parametrize("case", GOLD["floor_on_axis"]["cases"])
def test_floor_on_axis(case):
    f, t = case["f"], case["t"]
    cam = synth.camera(synth.PINHOLE, 101, 101, fx=f, fy=f, cx=50.5, cy=50.5)
    r = O.bake_rho2(_scene_one((0, 0, t), -3.0), [cam])[0]
    assert r == pytest.approx(case["rho2"], rel=1e-6)
