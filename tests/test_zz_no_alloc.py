"""cg_render_forward_noalloc, the forward entry point for callers that cannot allocate:
through the C ABI its images equal cg_render_forward's on the same inputs (same
kernels, so bit for bit), on consecutive calls whose second input is smaller (the
per-GPU scratch array keeps the first call's contents); a call that needs more than
the array holds is an argument error that leaves the next call unaffected."""
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


def _both(scene, cams, opts):
    import torch
    from paper_2609_13397_amd import render as R
    sc = R.Scene.from_numpy(scene)
    a, ia = R.render_forward_noalloc(sc, cams, opts)
    b, ib, _ = R.render_forward(sc, cams, opts)
    torch.cuda.synchronize()
    assert ia["n_pairs"] == ib["n_pairs"]
    return a, b


def test_noalloc_equals_forward_on_two_calls_second_smaller():
    import torch
    from paper_2609_13397_amd import render as R
    scene, cam = synth.tiny_config()
    ragged = synth.camera(synth.PINHOLE, 90, 60, fx=45.0, fy=45.0, cx=44.0, cy=31.0,
                          origin=(0.1, -0.1, -3.0), crop=(7, 11, 70, 37))
    _say("no-alloc forward: 256 Gaussians, two views")
    a, b = _both(scene, [cam, ragged], R.RenderOpts())
    assert torch.equal(a, b)
    views = R.split_views(a, [cam, ragged])
    for v, c in zip(views, [cam, ragged]):
        nfail, worst, det = compare_image(v.cpu().numpy().astype(np.float64),
                                          O.render(scene, c, O.Opts(), with_alt=True))
        _say(f"   parity fail={nfail} worst={worst:.3e}")
        assert nfail == 0, det
    # a smaller second call: fewer Gaussians, one smaller view, other options
    small = synth.subset_scene(scene, np.arange(0, 256, 2))
    crop = synth.with_crop(cam, 5, 3, 37, 29)
    _say("no-alloc forward: 128 Gaussians, one 37x29 crop, floor off, centre ray")
    a2, b2 = _both(small, [crop], R.RenderOpts(filter_mode=0, bg=(0.2, 0.1, 0.0)))
    assert torch.equal(a2, b2)
    nfail, worst, det = compare_image(a2.view(29, 37, 4).cpu().numpy().astype(np.float64),
                                      O.render(small, crop, O.Opts(filter_mode=0, bg=(0.2, 0.1, 0.0)),
                                               with_alt=True))
    assert nfail == 0, det


def test_noalloc_medium_scene_and_split_render():
    """20k SH Gaussians at 1/8 of the 1080p orbit view (the split tile render takes this
    launch: few tiles, long lists), then the 8-view orbit at 1/16."""
    import torch
    from paper_2609_13397_amd import render as R
    scene, cams = synth.pinhole_config(n=20_000)
    c8 = synth.scale_camera(cams[0], 1 / 8)
    _say("no-alloc forward: 20k Gaussians, 240x135, split tile render")
    R.set_tile_split(2048, 64, 0)  # split lists longer than 64 pairs per tile on average
    try:
        a, b = _both(scene, [c8], R.RenderOpts())
        _, info = R.render_forward_noalloc(R.Scene.from_numpy(scene), [c8], R.RenderOpts())
    finally:
        R.set_tile_split(0, 0, 0)
    assert info["n_segments"] > 0
    assert torch.equal(a, b)
    c16 = [synth.scale_camera(c, 1 / 16) for c in cams]
    _say("no-alloc forward: 20k Gaussians, 8 views 120x68")
    a, b = _both(scene, c16, R.RenderOpts())
    assert torch.equal(a, b)


def test_noalloc_rejects_calls_beyond_its_array():
    import torch
    from paper_2609_13397_amd import _lib
    from paper_2609_13397_amd import render as R
    big = synth.make_scene(400_000, seed=5, layout="clusters", color="rgb", log_scale_mean=-4.0)
    cam = synth.scale_camera(synth.orbit_views(1)[0], 1 / 8)
    _say("no-alloc forward beyond 64 MiB: 400k Gaussians")
    with pytest.raises(_lib.CgError) as ei:
        R.render_forward_noalloc(R.Scene.from_numpy(big), [cam], R.RenderOpts())
    torch.cuda.synchronize()
    assert ei.value.status == -1 and "fixed scratch region" in str(ei.value)
    scene, tcam = synth.tiny_config()
    a, b = _both(scene, [tcam], R.RenderOpts())
    assert torch.equal(a, b)
