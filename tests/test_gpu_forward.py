"""GPU parity of the forward path (through the C ABI) against the FP64 oracle.

Images must match within 2e-4 absolute per channel (the tolerance the method's
float32 arithmetic is held to); where the oracle reports a near-threshold decision
(alpha_min, T_min, t_near) the GPU may match the result with that decision flipped.
"""
import math
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2609_13397_amd import synth
from parity import TOL_IMAGE, compare_image

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    from paper_2609_13397_amd import render as R
    assert torch.cuda.is_available(), "no GPU"
    return torch, R


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _opts_pair(**kw):
    from paper_2609_13397_amd import render as R
    return R.RenderOpts(**kw), O.Opts(**kw)


def gpu_render(scene, cams, opts):
    torch, R = _gpu()
    sc = R.Scene.from_numpy(scene)
    rgba, info, _ = R.render_forward(sc, cams, opts)
    torch.cuda.synchronize()
    return [v.cpu().numpy().astype(np.float64) for v in R.split_views(rgba, cams)], info


def check_view(gpu_img, scene, cam, oopts, mode="brute", tol=TOL_IMAGE):
    ref = O.render(scene, cam, oopts, mode=mode, with_alt=True)
    nfail, worst, det = compare_image(gpu_img, ref, tol)
    _say(f"   parity: fail={nfail} worst={worst:.3e} {det}")
    assert nfail == 0, (worst, det)
    return ref


# --------------------------------------------------------------------------- cameras

@pytest.mark.parametrize("which", ["pinhole", "kb", "equirect"])
def test_camera_unproject_matches_oracle(which):
    torch, R = _gpu()
    k, _ = synth.draw_kb_coeffs(31, math.radians(95))
    cams = {
        "pinhole": synth.camera(synth.PINHOLE, 640, 480, fx=500.0, fy=510.0, cx=320.3, cy=241.7,
                                R_c2w=synth.look_at((0, 0, 0), (1, 2, 0.5))),
        "kb": synth.kb_camera(400, 400, 95.0, k, 200.0, synth.look_at((0, 0, 0), (1, -1, 0.2)), (0, 0, 0)),
        "equirect": synth.camera(synth.EQUIRECT, 512, 256, R_c2w=synth.look_at((0, 0, 0), (0.3, 1, 0))),
    }
    cam = cams[which]
    _say(f"unproject {which}")
    rng = np.random.default_rng(2)
    n = 20000
    px = rng.uniform(0, cam["full_w"], n).astype(np.float32)
    py = rng.uniform(0, cam["full_h"], n).astype(np.float32)
    xy = torch.from_numpy(np.stack([px, py])).cuda()
    dirs, valid = R.camera_unproject(cam, xy)
    dirs = dirs.cpu().numpy().T.astype(np.float64)
    valid = valid.cpu().numpy()
    dref, vref = O.unproject(cam, px.astype(np.float64), py.astype(np.float64))
    # validity decided in FP64 on both sides from the same float32 coordinates
    assert np.array_equal(valid, vref)
    err = np.max(np.abs(dirs[vref] - dref[vref]))
    _say(f"   max dir err {err:.3e}")
    assert err < 1e-6  # float32 rounding of a unit vector


def test_camera_unproject_equirect_known_pixels():
    """The GPU's equirect inverse at pixels whose directions are known without the
    formula (the optical axis at the centre, +x three quarters across, -x a quarter
    across, behind the camera at the left edge, 45 degrees up a quarter down)."""
    from test_oracle_pins import EQUIRECT_KNOWN
    torch, R = _gpu()
    Rw = synth.look_at((0, 0, 0), (0.3, 1, 0.2))
    cam = synth.camera(synth.EQUIRECT, 512, 256, R_c2w=Rw, origin=(1.0, -2.0, 0.5))
    R32 = np.array(cam["R_c2w"], np.float32).astype(np.float64)
    px = np.array([f[0] * 512 for f, _ in EQUIRECT_KNOWN], np.float32)
    py = np.array([f[1] * 256 for f, _ in EQUIRECT_KNOWN], np.float32)
    _say("unproject equirect known pixels")
    dirs, valid = R.camera_unproject(cam, torch.from_numpy(np.stack([px, py])).cuda())
    dirs = dirs.cpu().numpy().T.astype(np.float64)
    assert valid.cpu().numpy().all()
    expect = np.array([R32 @ np.array(dc) for _, dc in EQUIRECT_KNOWN])
    err = np.max(np.abs(dirs - expect))
    _say(f"   max dir err {err:.3e}")
    assert err < 1e-6


# --------------------------------------------------------------------------- floor bake

def test_bake_rho2_matches_oracle():
    torch, R = _gpu()
    scene = synth.make_scene(20000, seed=21, layout="clusters", color="sh3", log_scale_mean=-4.0, log_scale_std=0.7)
    cams = synth.orbit_views(8) + synth.fisheye_cameras()
    _say("bake rho2")
    sc = R.Scene.from_numpy(scene)
    r_gpu = R.bake_rho2(sc, cams).cpu().numpy().astype(np.float64)
    r_ref = O.bake_rho2(scene, cams)
    assert np.array_equal(r_gpu == 0, r_ref == 0)
    nz = r_ref > 0
    rel = np.abs(r_gpu[nz] - r_ref[nz]) / r_ref[nz]
    _say(f"   visible {nz.mean():.3f} max rel err {rel.max():.3e}")
    assert rel.max() < 1e-5


# --------------------------------------------------------------------------- forward parity

TINY_VARIANTS = [
    dict(filter_mode=1),
    dict(filter_mode=0),
    dict(filter_mode=2),
    dict(filter_mode=1, bg=(0.2, 0.4, 0.6)),
    dict(filter_mode=1, footprint_scale=3.0),
    dict(filter_mode=1, backbone=1),
    dict(filter_mode=0, backbone=1),
]


@pytest.mark.parametrize("kw", TINY_VARIANTS, ids=[str(v) for v in TINY_VARIANTS])
def test_tiny_forward_parity(kw):
    """256 Gaussians, 64x48 pinhole (config 1) plus a ragged 70x37 crop of a wider view."""
    scene, cam = synth.tiny_config()
    ragged = synth.camera(synth.PINHOLE, 90, 60, fx=45.0, fy=45.0, cx=44.0, cy=31.0,
                          origin=(0.1, -0.1, -3.0), crop=(7, 11, 70, 37))
    gopts, oopts = _opts_pair(**kw)
    _say(f"tiny forward {kw}")
    imgs, info = gpu_render(scene, [cam, ragged], gopts)
    _say(f"   pairs {info['n_pairs']}")
    for img, c in zip(imgs, [cam, ragged]):
        check_view(img, scene, c, oopts)


@pytest.mark.parametrize("composition,backbone", [(0, 0), (1, 0), (0, 1)])
def test_tiny_forward_floor_parity(composition, backbone):
    """Floor on, with rho^2 baked (by the oracle, Eq. 11) from the same camera at x2
    resolution, so the floor partly covers the render footprint."""
    scene, cam = synth.tiny_config()
    scene = dict(scene)
    scene["rho2"] = O.bake_rho2(scene, [synth.scale_camera(cam, 2.0)]).astype(np.float32)
    gopts, oopts = _opts_pair(use_floor=True, composition=composition, backbone=backbone)
    oopts.use_floor = 1
    _say(f"tiny floor composition={composition} backbone={backbone}")
    imgs, _ = gpu_render(scene, [cam], gopts)
    check_view(imgs[0], scene, cam, oopts)


@pytest.mark.parametrize("backbone", [0, 1])
def test_fisheye_and_equirect_small_parity(backbone):
    """Wide cameras with sheared peripheral footprints: a 190-degree KB fisheye and an
    equirectangular view, 2000 Gaussians around the camera, floor on."""
    scene = synth.make_scene(2000, seed=22, layout="clusters", color="sh3", log_scale_mean=-3.0, log_scale_std=0.6)
    scene["means"] *= 0.3
    kb, eq = synth.fisheye_cameras()
    kb = synth.scale_camera(kb, 1 / 16)
    eq = synth.scale_camera(eq, 1 / 16)
    cams = [kb, eq]
    for c in cams:
        c["origin"] = (0.0, -1.0, 0.3)
    scene["rho2"] = O.bake_rho2(scene, [synth.scale_camera(c, 2.0) for c in cams]).astype(np.float32)
    gopts, oopts = _opts_pair(use_floor=True, backbone=backbone)
    oopts.use_floor = 1
    _say(f"fisheye + equirect small, backbone {backbone}")
    imgs, info = gpu_render(scene, cams, gopts)
    _say(f"   pairs {info['n_pairs']}")
    for img, c in zip(imgs, cams):
        check_view(img, scene, c, oopts)


def test_more_than_65536_tiles_three_sort_passes():
    """Three 4096x2048 equirect views in one call: 98,304 tiles, so the tile ids need
    17 bits and the tile sort a third 8-bit pass, and the depth sort orders the items of
    three views together on the depth key alone.  Three rows of every view (near the
    top, the middle, the last) are checked against the oracle."""
    torch, R = _gpu()
    scene = synth.make_scene(2000, seed=23, layout="clusters", color="sh3", log_scale_mean=-3.0, log_scale_std=0.6)
    scene["means"] *= 0.3
    _, eq = synth.fisheye_cameras()
    eq = synth.scale_camera(eq, 2.0)
    cams = []
    for o in ((0.0, -1.0, 0.3), (0.8, 0.2, -0.2), (-0.5, 0.6, 0.1)):
        c = dict(eq)
        c["origin"] = o
        cams.append(c)
    w, h = cams[0]["crop"][2], cams[0]["crop"][3]
    assert (w, h) == (4096, 2048)
    _say("3 x equirect 4096x2048")
    rgba, info, _ = R.render_forward(R.Scene.from_numpy(scene), cams, R.RenderOpts())
    torch.cuda.synchronize()
    _say(f"   tiles {info['n_tiles']} sort bits {info['sort_bits']} pairs {info['n_pairs']}")
    assert info["n_tiles"] == 3 * (w // 16) * (h // 16)
    assert info["sort_bits"] == 17
    views = R.split_views(rgba, cams)
    for v, c in enumerate(cams):
        for row in (5, 1000, h - 1):
            img = views[v][row:row + 1].cpu().numpy().astype(np.float64)
            check_view(img, scene, synth.with_crop(c, 0, row, w, 1), O.Opts())


def _thin_scene(n, seed, log_s=(-1.0, -1.5, -6.0), spread=0.6):
    """Thin discs (aspect up to 150:1) in random orientations around the origin."""
    rng = np.random.default_rng(seed)
    return {
        "n": n, "color_mode": 0,
        "means": (rng.uniform(-1, 1, (3, n)) * spread).astype(np.float32),
        "log_scales": np.tile(np.array(log_s, np.float32)[:, None], (1, n)) + rng.normal(0, 0.2, (3, n)).astype(
            np.float32),
        "quats": rng.normal(0, 1, (4, n)).astype(np.float32),
        "opacity_logits": rng.normal(-1.0, 1.0, n).astype(np.float32),
        "color": rng.uniform(0, 1, (3, n)).astype(np.float32),
        "rho2": np.zeros(n, np.float32),
    }


@pytest.mark.parametrize("kw", [dict(), dict(use_floor=1), dict(filter_mode=2, use_floor=1), dict(backbone=1)],
                         ids=["aniso", "aniso_floor", "iso_floor", "ray_integral"])
def test_thin_gaussians_at_grazing_angles(kw):
    """Thin discs seen edge-on by a pinhole and a 190-degree fisheye: the whitened
    footprint reaches tr K ~ 1e4, where the 2x2 form of Eq. 9 cancels, and the render
    takes its cancellation-free form.  Whole images against the oracle at 2e-4."""
    torch, R = _gpu()
    scene = _thin_scene(300, seed=31)
    pin = synth.camera(synth.PINHOLE, 96, 72, fx=50.0, fy=50.0, cx=48.0, cy=36.0, origin=(0.2, -0.1, -3.0))
    kb = synth.kb_camera(112, 112, 95.0, (0.01, -0.004, 0.0, 0.0), 56.0, np.eye(3), (0.1, 0.0, -2.5))
    cams = [pin, kb]
    if kw.get("use_floor"):
        scene["rho2"] = O.bake_rho2(scene, [synth.scale_camera(c, 2.0) for c in cams]).astype(np.float32)
    gkw = {k: (bool(v) if k == "use_floor" else v) for k, v in kw.items()}
    _say(f"thin Gaussians {kw}")
    imgs, info = gpu_render(scene, cams, R.RenderOpts(**gkw))
    for img, c in zip(imgs, cams):
        check_view(img, scene, c, O.Opts(**kw))


def test_pair_total_beyond_32_bits_is_an_argument_error():
    """50,000 Gaussians of 1.6 m around three 4096x2048 equirect centres: every Gaussian
    reaches every one of the 98,304 tiles, about 4.9e9 (tile, Gaussian) pairs, more than
    32-bit pair indices hold.  The forward counts the pairs in 64 bits and returns
    CG_ERR_INVALID_ARG before anything is emitted; the next call renders normally."""
    torch, R = _gpu()
    from paper_2609_13397_amd import _lib
    n = 50_000
    scene = synth.make_scene(n, seed=29, layout="uniform", color="rgb", log_scale_mean=0.5, log_scale_std=0.01)
    scene["means"] *= 0.5
    scene["opacity_logits"][:] = 3.0
    _, eq = synth.fisheye_cameras()
    eq = synth.scale_camera(eq, 2.0)
    cams = []
    for o in ((0.0, 0.0, 0.0), (0.1, 0.0, 0.0), (0.0, 0.1, 0.0)):
        c = dict(eq)
        c["origin"] = o
        cams.append(c)
    _say("pair total beyond 32 bits: 50k Gaussians x 3 x equirect 4096x2048")
    with pytest.raises(_lib.CgError) as ei:
        R.render_forward(R.Scene.from_numpy(scene), cams, R.RenderOpts())
    torch.cuda.synchronize()
    _say(f"   {ei.value}")
    assert ei.value.status == -1 and "too many" in str(ei.value)  # CG_ERR_INVALID_ARG
    tiny, cam = synth.tiny_config()
    imgs, _ = gpu_render(tiny, [cam], R.RenderOpts())
    check_view(imgs[0], tiny, cam, O.Opts())


def test_empty_and_degenerate_inputs():
    torch, R = _gpu()
    _say("empty inputs")
    scene, cam = synth.tiny_config()
    empty = synth.subset_scene(scene, np.arange(0))
    imgs, info = gpu_render(empty, [cam], R.RenderOpts(bg=(0.1, 0.2, 0.3)))
    assert info["n_pairs"] == 0
    assert np.allclose(imgs[0][..., :3], [0.1, 0.2, 0.3]) and np.all(imgs[0][..., 3] == 0)
    # one Gaussian behind the camera: nothing is binned
    behind = synth.subset_scene(scene, np.arange(1))
    behind["means"] = np.array([[0.0], [0.0], [-5.0]], np.float32)
    imgs, info = gpu_render(behind, [cam], R.RenderOpts())
    assert info["n_pairs"] == 0 and np.all(imgs[0] == 0)
    # zero-sized crop next to a normal view
    c0 = synth.with_crop(cam, 0, 0, 0, 0)
    imgs, info = gpu_render(scene, [c0, cam], R.RenderOpts())
    assert imgs[0].shape == (0, 0, 4)
    check_view(imgs[1], scene, cam, O.Opts())
    # every view empty: a call without a single tile
    imgs, info = gpu_render(scene, [c0, c0], R.RenderOpts())
    assert all(im.shape == (0, 0, 4) for im in imgs) and info["n_pairs"] == 0


def test_large_gaussians_cover_many_tile_groups():
    """Gaussians close to the camera whose influence cones reach more than 16 of a
    view's 8x8-tile groups: the binning lists at most 16 group hits per Gaussian and
    tests every group of the view again for these, in the count and the emit pass.
    A 640x480 pinhole (20 tile groups), a 533x533 KB fisheye (25) and a 683x341
    equirect (18), floor off."""
    torch, R = _gpu()
    cam = synth.camera(synth.PINHOLE, 640, 480, fx=500.0, fy=500.0, cx=320.0, cy=240.0,
                       R_c2w=np.eye(3), origin=(0.0, 0.0, -3.0))
    scene = synth.make_scene(12, seed=71, layout="uniform", color="rgb", log_scale_mean=-1.2, log_scale_std=0.4)
    scene["means"][:, 0] = 0.0        # 3 m in front of the pinhole
    scene["log_scales"][:, 0] = 0.0   # 1 m: its cone covers the whole pinhole view
    scene["opacity_logits"][0] = -1.0
    _say("large Gaussians")
    # a Gaussian with more pairs than 16 groups of 64 tiles hold overlaps more than 16 groups
    _, info = gpu_render(synth.subset_scene(scene, np.arange(1)), [cam], R.RenderOpts())
    _say(f"   one large Gaussian: {info['n_pairs']} pairs")
    assert info["n_pairs"] > 16 * 64
    kb, eq = synth.fisheye_cameras()
    cams = [cam, synth.scale_camera(kb, 1 / 3), synth.scale_camera(eq, 1 / 3)]
    for c in cams[1:]:
        c["origin"] = (0.0, 0.0, -3.0)
    imgs, info = gpu_render(scene, cams, R.RenderOpts())
    _say(f"   pairs {info['n_pairs']}")
    for img, c in zip(imgs, cams):
        check_view(img, scene, c, O.Opts())


def test_multiview_batch_equals_single_views():
    """A batched call renders each view exactly as a call with that view alone."""
    torch, R = _gpu()
    scene, cam = synth.tiny_config()
    cams = [cam, synth.scale_camera(cam, 0.5), synth.scale_camera(cam, 2.0)]
    _say("multiview batch")
    batch, _ = gpu_render(scene, cams, R.RenderOpts())
    for img, c in zip(batch, cams):
        single, _ = gpu_render(scene, [c], R.RenderOpts())
        assert np.array_equal(img, single[0])


def test_determinism_and_permutation():
    torch, R = _gpu()
    scene, cam = synth.tiny_config()
    _say("determinism")
    a, _ = gpu_render(scene, [cam], R.RenderOpts())
    b, _ = gpu_render(scene, [cam], R.RenderOpts())
    assert np.array_equal(a[0], b[0])
    perm = np.random.default_rng(3).permutation(scene["n"])
    c, _ = gpu_render(synth.subset_scene(scene, perm), [cam], R.RenderOpts())
    assert np.array_equal(a[0], c[0])


def test_pinhole_config_eighth_resolution_parity():
    """Config 2 at 1/8 resolution (240x135): 100k clustered Gaussians with SH colour and
    rho^2 baked from the 8 full-resolution orbit views; two of the 8 views, floor on."""
    scene, views = synth.pinhole_config()
    _say("pinhole 1/8: baking rho2")
    torch, R = _gpu()
    sc = R.Scene.from_numpy(scene)
    rho2 = O.bake_rho2(scene, views)
    scene["rho2"] = rho2.astype(np.float32)
    cams = [synth.scale_camera(views[0], 0.125), synth.scale_camera(views[3], 0.125)]
    gopts, oopts = _opts_pair(use_floor=True)
    oopts.use_floor = 1
    imgs, info = gpu_render(scene, cams, gopts)
    _say(f"   pairs {info['n_pairs']}")
    for img, c in zip(imgs, cams):
        check_view(img, scene, c, oopts, mode="culled")


def test_contributing_pair_count_matches_oracle():
    """The counting render variant counts composited pairs exactly as the oracle does
    (pixels with a near-threshold decision may differ by their own pair counts)."""
    torch, R = _gpu()
    scene, cam = synth.tiny_config()
    _say("pair counts")
    sc = R.Scene.from_numpy(scene)
    rgba, info, _ = R.render_forward(sc, [cam], R.RenderOpts(count_pairs=True))
    plain, _, _ = R.render_forward(sc, [cam], R.RenderOpts())
    torch.cuda.synchronize()
    assert torch.equal(rgba, plain)  # the counting variant renders identically
    ref = O.render(scene, cam, O.Opts(), with_alt=True)
    amb = ref["n_dec"] > 0
    slack = int(ref["n_contrib"][amb].sum()) + int(amb.sum())
    _say(f"   gpu {info['n_contrib']} oracle {int(ref['n_contrib'].sum())} slack {slack}")
    assert abs(info["n_contrib"] - int(ref["n_contrib"].sum())) <= slack
    assert info["n_evaluated"] >= info["n_full"] >= info["n_contrib"] > 0


def _two_pinholes():
    cams = []
    for phi in (0.3, 2.2):
        o = (3.5 * math.cos(phi), 3.5 * math.sin(phi), 0.8)
        cams.append(synth.camera(synth.PINHOLE, 128, 96, fx=90.0, fy=90.0, cx=64.0, cy=48.0,
                                 R_c2w=synth.look_at(o, (0, 0, 0)), origin=o))
    return cams


def test_pair_buffers_sized_from_the_previous_call():
    """A forward call shaped like the thread's previous one (same Gaussian count, views,
    tiles and pixels) sizes its pair buffers from that call's pair count and queues the
    emit pass before reading its own count back; when its count exceeds that guess, the
    emit pass drops the pairs past it and the call emits again into buffers of the right
    size.  Images and pair counts do not depend on the path taken."""
    torch, R = _gpu()
    cams = _two_pinholes()
    opts = R.RenderOpts()
    small = synth.make_scene(512, seed=5, layout="uniform", color="rgb", log_scale_mean=-4.0, log_scale_std=0.3)
    big = dict(small)
    big["log_scales"] = small["log_scales"] + 2.0
    other = synth.subset_scene(small, np.arange(100))
    _say("pair buffers: big scene after a call of another shape (no guess)")
    gpu_render(other, cams, opts)
    ref_big, info_big = gpu_render(big, cams, opts)
    _say("small scene, guess from the big one (oversized)")
    img_small, info_small = gpu_render(small, cams, opts)
    assert info_small["n_pairs"] + info_small["n_pairs"] // 16 + 4096 < info_big["n_pairs"], (info_small, info_big)
    _say("big scene, guess from the small one (too small: emitted again)")
    img_big, info = gpu_render(big, cams, opts)
    assert info["n_pairs"] == info_big["n_pairs"]
    for a, b in zip(img_big, ref_big):
        assert np.array_equal(a, b)
    _say("small scene without a guess")
    gpu_render(other, cams, opts)
    ref_small, info = gpu_render(small, cams, opts)
    assert info["n_pairs"] == info_small["n_pairs"]
    for a, b in zip(img_small, ref_small):
        assert np.array_equal(a, b)
    for img, c in zip(ref_big, cams):
        check_view(img, big, c, O.Opts())


def test_many_items_take_the_general_scans():
    """Over 2048 x 2048 (view, Gaussian) items the counts scan in compositing order and
    the plain scans fall back from their two-launch form to the general one: 1.1M
    Gaussians in four small views (4.4M items) render bit for bit as each view does
    alone (1.1M items, the two-launch form)."""
    torch, R = _gpu()
    scene = synth.make_scene(1_100_000, seed=19, layout="clusters", color="rgb", log_scale_mean=-4.5,
                             log_scale_std=0.5)
    cams = []
    for phi in (0.0, 1.6, 3.1, 4.7):
        o = (12.0 * math.cos(phi), 12.0 * math.sin(phi), 1.0)
        cams.append(synth.camera(synth.PINHOLE, 160, 120, fx=120.0, fy=120.0, cx=80.0, cy=60.0,
                                 R_c2w=synth.look_at(o, (0, 0, 0)), origin=o))
    opts = R.RenderOpts()
    _say("4 views of 1.1M Gaussians in one call (4.4M items)")
    fused, info = gpu_render(scene, cams, opts)
    assert info["n_pairs"] > 0
    for v, c in enumerate(cams):
        alone, _ = gpu_render(scene, [c], opts)
        assert np.array_equal(alone[0], fused[v]), v
