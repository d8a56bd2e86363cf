"""Scratch guard bands on the GPU.  With a band of a fixed pattern after every scratch
buffer, the forward (whole tiles, split tiles, per-ray order, with training state),
the backward and the no-allocation forward leave every band intact, and their images
and gradients are bit for bit those of the same calls without bands.  A band
overwritten from the host (guard mode 2) is reported as CG_ERR_STATE."""
import sys

import pytest

from paper_2609_13397_amd import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _scene(n, seed):
    from paper_2609_13397_amd import render as R
    sc = synth.make_scene(n, seed=seed, layout="clusters", color="sh3", log_scale_mean=-3.5, log_scale_std=0.6)
    t = R.Scene.from_numpy(sc)
    t.rho2 = R.bake_rho2(t, synth.orbit_views(), 0.2)
    return t


def _calls(scene, small_scene):
    """Every scratch-using path once; returns the images and gradients."""
    import torch
    from paper_2609_13397_amd import render as R
    cams = [synth.scale_camera(c, 0.25) for c in synth.orbit_views(3)]
    crop = synth.with_crop(synth.scale_camera(synth.orbit_views(1)[0], 2.0), 1500, 700, 200, 136)
    outs = {}
    opts = R.RenderOpts(use_floor=True)
    outs["tiles"] = R.render_forward(scene, cams + [crop], opts)[0].clone()
    R.set_tile_split(4096, 64, 0)  # force the split tile render on these small views
    try:
        img, info, _ = R.render_forward(scene, cams[:2], opts)
        assert info["n_segments"] > 0
        outs["split"] = img.clone()
    finally:
        R.set_tile_split()
    outs["ray"] = R.render_forward(scene, cams[:1], R.RenderOpts(use_floor=True, order_mode=R.ORDER_RAY))[0].clone()
    img, _, st = R.render_forward(small_scene, cams[1:], opts, need_state=True)
    outs["train"] = img.clone()
    grads = R.render_backward(st, torch.linspace(-1, 1, img.numel(), device=img.device).view_as(img), small_scene)
    st.release()
    for k, v in grads.items():
        outs["grad_" + k] = v.clone()
    outs["noalloc"] = R.render_forward_noalloc(small_scene, cams[:2], opts)[0].clone()
    torch.cuda.synchronize()
    return outs


def test_guard_bands_stay_intact_and_change_nothing():
    import torch
    from paper_2609_13397_amd import render as R
    scene, small = _scene(200000, 81), _scene(20000, 82)
    _say("guards: reference calls without bands")
    ref = _calls(scene, small)
    before = R.guard_violations()
    R.set_scratch_guards(1)
    try:
        _say("guards: the same calls with bands")
        got = _calls(scene, small)
    finally:
        R.set_scratch_guards(0)
    assert R.guard_violations() == before
    for k in ref:
        assert torch.equal(ref[k], got[k]), k


def test_overwritten_band_is_reported():
    import torch
    from paper_2609_13397_amd import _lib
    from paper_2609_13397_amd import render as R
    small = _scene(5000, 83)
    cams = [synth.scale_camera(synth.orbit_views(1)[0], 0.125)]
    before = R.guard_violations()
    R.set_scratch_guards(2)
    try:
        _say("guards: a band overwritten from the host")
        with pytest.raises(_lib.CgError, match="guard"):
            R.render_forward(small, cams, R.RenderOpts())
    finally:
        R.set_scratch_guards(0)
    assert R.guard_violations() == before + 1
    img, _, _ = R.render_forward(small, cams, R.RenderOpts())  # and the next call is unaffected
    torch.cuda.synchronize()
    assert torch.isfinite(img).all()
