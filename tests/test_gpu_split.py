"""GPU parity of the split tile render: launches with few tiles and long lists cut each
tile's depth-ordered list into segments rendered by separate workgroups, composited
from the transmittance product of the segments in front (Eq. 4 regrouped).  The image
must equal the one-workgroup-per-tile render up to the rounding order of those
products, and match the FP64 oracle like any forward image."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2609_13397_amd import synth
from parity import TOL_IMAGE, compare_image

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _render(scene, cams, opts, split):
    """split: (max_tiles, min_longest, seg_len) for cg_set_tile_split, or None for a
    render that never splits."""
    import torch
    from paper_2609_13397_amd import render as R
    assert torch.cuda.is_available(), "no GPU"
    if split is None:
        R.set_tile_split(1, 1 << 40, 0)  # no launch has fewer than 1 tile: never split
    else:
        R.set_tile_split(*split)
    try:
        sc = R.Scene.from_numpy(scene)
        rgba, info, _ = R.render_forward(sc, cams, opts)
        torch.cuda.synchronize()
    finally:
        R.set_tile_split(0, 0, 0)
    return [v.cpu().numpy().astype(np.float64) for v in R.split_views(rgba, cams)], info


U32 = 2.0 ** -24  # float32 unit roundoff


def _split_bounds(scene, cams, opts, longest):
    """Bounds on |split - unsplit| per pixel and channel, from the arithmetic.  Both renders
    evaluate the same pairs identically; the split one groups the transmittance product
    T_k = prod (1 - alpha_j) per segment and sums the colour per segment.  Each T_k is a
    product of at most L factors (L: the longest tile list), so its rounding differs by at
    most about 2 L u T_k between the two, and the colour sums by L u of their total, whose
    weights T_k alpha_k sum to at most 1: |dC| <= 3 L u cmax (first order, doubled here),
    cmax bounding every pair colour, the background and the alpha channel's 1.  Where the
    rounding moves Ttr (1 - alpha) across T_min, one render composites a pair that the
    other stops before; the transmittance there is below T_min / (1 - alpha_max), which
    bounds the rest of the pixel: |d| <= T_min / (1 - alpha_max) (cmax + |bg|) + the
    rounding bound.  Returns (rounding bound, termination bound)."""
    cmax = 1.0
    for c in cams:
        pre, _ = O.preprocess(scene, c["origin"], O.Opts(use_floor=int(opts.use_floor)))
        cmax = max(cmax, float(np.abs(pre[:, 4:7]).max()))
    bg = max(abs(b) for b in opts.bg)
    cmax = max(cmax, bg)
    b_round = 2 * 3 * longest * U32 * cmax
    b_flip = opts.T_min / (1.0 - opts.alpha_max) * (cmax + bg) + b_round
    return b_round, b_flip


def _check_split(ref, got, bounds, what):
    """Every pixel within the rounding bound, except pixels where the termination test
    fell differently, which stay within the termination bound and are rare."""
    b_round, b_flip = bounds
    n_px = sum(a.shape[0] * a.shape[1] for a in ref)
    over = sum(int((np.abs(a - b).max(axis=-1) > b_round).sum()) for a, b in zip(ref, got))
    worst = max(float(np.abs(a - b).max()) for a, b in zip(ref, got))
    _say(f"   {what}: max |split - unsplit| {worst:.3e} (rounding bound {b_round:.2e}, termination bound "
         f"{b_flip:.2e}); pixels beyond the rounding bound: {over} of {n_px}")
    assert worst <= b_flip
    assert over <= max(2, n_px // 1000)


def _small_wide_scene():
    scene = synth.make_scene(2000, seed=22, layout="clusters", color="sh3", log_scale_mean=-3.0, log_scale_std=0.6)
    scene["means"] *= 0.3
    kb, eq = synth.fisheye_cameras()
    cams = [synth.scale_camera(kb, 1 / 16), synth.scale_camera(eq, 1 / 16)]
    for c in cams:
        c["origin"] = (0.0, -1.0, 0.3)
    scene["rho2"] = O.bake_rho2(scene, [synth.scale_camera(c, 2.0) for c in cams]).astype(np.float32)
    return scene, cams


@pytest.mark.parametrize("seg_len", [64, 200, 1024])
def test_split_render_equals_unsplit_and_oracle(seg_len):
    from paper_2609_13397_amd import render as R
    scene, cams = _small_wide_scene()
    opts = R.RenderOpts(use_floor=True)
    _say(f"split render, segments of {seg_len} pairs")
    ref, info0 = _render(scene, cams, opts, None)
    got, info1 = _render(scene, cams, opts, (1 << 20, 1, seg_len))
    _say(f"   pairs {info1['n_pairs']} segments {info1['n_segments']} tiles {info1['n_tiles']}")
    assert info0["n_segments"] == 0
    assert info1["n_segments"] > info1["n_tiles"]  # some tile has more than one segment
    assert info1["n_pairs"] == info0["n_pairs"]
    _check_split(ref, got, _split_bounds(scene, cams, opts, info1["max_tile_pairs"]), f"seg_len {seg_len}")
    oopts = O.Opts(use_floor=1)
    for a, b, c in zip(ref, got, cams):
        refo = O.render(scene, c, oopts, mode="brute", with_alt=True)
        nfail, worst, det = compare_image(b, refo, TOL_IMAGE)
        _say(f"   oracle parity: fail={nfail} worst={worst:.3e} {det}")
        assert nfail == 0, (worst, det)


def test_split_render_options_and_batches():
    """Every filter mode, the additive composition, the ray-integral backbone and a
    multi-view batch take the split path and agree with the unsplit render."""
    from paper_2609_13397_amd import render as R
    scene, cams = _small_wide_scene()
    cams = cams + [synth.scale_camera(cams[0], 0.5)]
    for kw in (dict(filter_mode=0), dict(filter_mode=2, use_floor=True), dict(use_floor=True, composition=1),
               dict(use_floor=True, backbone=1), dict(bg=(0.2, 0.3, 0.4))):
        opts = R.RenderOpts(**kw)
        ref, _ = _render(scene, cams, opts, None)
        got, info = _render(scene, cams, opts, (1 << 20, 1, 128))
        assert info["n_segments"] > info["n_tiles"]
        _check_split(ref, got, _split_bounds(scene, cams, opts, info["max_tile_pairs"]),
                     f"{kw} ({info['n_segments']} segments)")


def test_small_view_of_large_scene_splits_by_default():
    """A 240x135 view of the 100k-Gaussian pinhole scene has few tiles and a few very
    long lists: the longest list exceeds the default thresholds, so the call takes the
    split path; its image matches the oracle."""
    from paper_2609_13397_amd import render as R
    scene, views = synth.pinhole_config()
    scene["rho2"] = O.bake_rho2(scene, views).astype(np.float32)
    cam = synth.scale_camera(views[2], 0.125)
    opts = R.RenderOpts(use_floor=True)
    _say("small view of the pinhole scene")
    got, info = _render(scene, [cam], opts, (0, 0, 0))
    _say(f"   pairs {info['n_pairs']} tiles {info['n_tiles']} segments {info['n_segments']}")
    assert info["max_tile_pairs"] > max(2048, info["n_pairs"] // 1024)
    assert info["n_segments"] > 0
    ref, _ = _render(scene, [cam], opts, None)
    _check_split(ref, got, _split_bounds(scene, [cam], opts, info["max_tile_pairs"]), "default thresholds")
    refo = O.render(scene, cam, O.Opts(use_floor=1), mode="culled", with_alt=True)
    nfail, worst, det = compare_image(got[0], refo, TOL_IMAGE)
    _say(f"   oracle parity: fail={nfail} worst={worst:.3e} {det}")
    assert nfail == 0, (worst, det)


def test_small_view_of_serving_scene_split_sampled_rows():
    """The 500k-Gaussian serving scene in a 256x128 equirect view (1/8 scale): about 1.7M
    pairs over 128 tiles, so the default thresholds split the lists into segments and
    pixels terminate across segment boundaries.  Sampled rows (crops of the same
    camera) match the oracle, with rho^2 baked by the oracle."""
    import torch
    from paper_2609_13397_amd import render as R
    scene = synth.make_scene(500_000, seed=51, layout="clusters", color="sh3", log_scale_mean=-4.0,
                             log_scale_std=0.7)
    scene["rho2"] = O.bake_rho2(scene, synth.orbit_views(), 0.2).astype(np.float32)
    cam = synth.scale_camera(synth.serving_base_cameras()[2], 0.125)
    opts = R.RenderOpts(use_floor=True)
    _say("serving scene, 1/8 equirect")
    got, info = _render(scene, [cam], opts, (0, 0, 0))
    _say(f"   pairs {info['n_pairs']} tiles {info['n_tiles']} segments {info['n_segments']}")
    assert info["n_segments"] > info["n_tiles"]
    w = cam["crop"][2]
    for row in (10, 64, 100):
        c = synth.with_crop(cam, 0, row, w, 1)
        ref = O.render(scene, c, O.Opts(use_floor=1), mode="culled", with_alt=True)
        nfail, worst, det = compare_image(got[0][row:row + 1], ref, TOL_IMAGE)
        _say(f"   row {row}: fail={nfail} worst={worst:.2e} amb={det['n_ambiguous']}")
        assert nfail == 0, det
    torch.cuda.synchronize()


def test_training_and_counting_calls_never_split():
    import torch
    from paper_2609_13397_amd import render as R
    scene, cams = _small_wide_scene()
    R.set_tile_split(1 << 20, 1, 64)
    try:
        sc = R.Scene.from_numpy(scene)
        _, info, fs = R.render_forward(sc, cams, R.RenderOpts(use_floor=True), need_state=True)
        assert info["n_segments"] == 0
        _, info, _ = R.render_forward(sc, cams, R.RenderOpts(use_floor=True, count_pairs=True))
        assert info["n_segments"] == 0
        torch.cuda.synchronize()
    finally:
        R.set_tile_split(0, 0, 0)
