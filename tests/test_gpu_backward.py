"""GPU parity of the backward pass (through the C ABI) against the FP64 oracle gradient.

The oracle gradient differentiates compositing exactly and each pair's response by
Richardson-extrapolated central differences of the FP64 closed form; it is itself
pinned to central differences of whole renders (tests/test_oracle_pins.py).  Here the
GPU's hand-written reverse mode must agree per parameter group within 1e-3 relative
(norm of the difference over the norm of the reference) and per element within
1e-3 * max(|ref|, 1e-2 * RMS of the group).  The upstream gradient is a seeded random
image, zeroed at pixels where the oracle saw a near-threshold decision (where the two
renderers may legitimately take different branches).
"""
import math
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2609_13397_amd import synth

pytestmark = pytest.mark.gpu

GROUPS = ("means", "log_scales", "quats", "opacity_logits", "color")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def grad_scene(n=512, seed=42, color="sh3"):
    scene = synth.make_scene(n, seed=seed, layout="uniform", color=color, log_scale_mean=-2.8, log_scale_std=0.4)
    return scene


def grad_cameras(scale=1.0):
    """Two orbit pinholes and two 190-degree fisheyes around the unit cube."""
    cams = []
    for phi in (0.3, 2.2):
        o = (3.5 * math.cos(phi), 3.5 * math.sin(phi), 0.8)
        cams.append(synth.camera(synth.PINHOLE, 128, 96, fx=90.0, fy=90.0, cx=64.0, cy=48.0,
                                 R_c2w=synth.look_at(o, (0, 0, 0)), origin=o))
    for o, tgt in (((0.0, -2.6, 0.2), (0, 0, 0)), ((2.4, 0.5, -0.6), (0, 0, 0))):
        cams.append(synth.kb_camera(112, 112, 95.0, (0.01, -0.004, 0.0, 0.0), 56.0, synth.look_at(o, tgt), o))
    if scale != 1.0:
        cams = [synth.scale_camera(c, scale) for c in cams]
    return cams


def run_gpu(scene, cams, opts, grads_img):
    import torch
    from paper_2609_13397_amd import render as R
    sc = R.Scene.from_numpy(scene)
    rgba, info, state = R.render_forward(sc, cams, opts, need_state=True)
    g = torch.from_numpy(np.concatenate([x.reshape(-1, 4) for x in grads_img]).astype(np.float32)).cuda()
    grads = R.render_backward(state, g, sc)
    torch.cuda.synchronize()
    mism = R.replay_mismatches(state)
    state.release()
    return {k: v.cpu().numpy().astype(np.float64) for k, v in grads.items()}, rgba, info, mism


def compare_grads(g, ref, tol=1e-3):
    worst = {}
    for k in GROUPS:
        a, b = g[k].ravel(), ref[k].ravel()
        nref = np.linalg.norm(b)
        rel = np.linalg.norm(a - b) / max(nref, 1e-30)
        rms = math.sqrt(np.mean(b * b)) if b.size else 0.0
        elem = np.abs(a - b) / np.maximum(np.abs(b), 1e-2 * rms + 1e-30)
        worst[k] = (rel, float(elem.max()), int((elem > tol).sum()))
    return worst


def upstream(cams, refs, seed=7):
    out = []
    for v, (c, ref) in enumerate(zip(cams, refs)):
        w, h = c["crop"][2], c["crop"][3]
        G = synth.seeded_image((h, w, 4), seed=seed + v)
        G[ref["n_dec"] > 0] = 0.0
        out.append(G)
    return out


@pytest.mark.parametrize("case", ["floor_marginal", "no_floor", "centre_ray", "isotropic_floor", "rgb_additive",
                                  "ray_integral_floor", "ragged_tiles"])
def test_backward_matches_oracle_gradient(case):
    from paper_2609_13397_amd import render as R
    color = "rgb" if case == "rgb_additive" else "sh3"
    scene = grad_scene(color=color)
    # ragged_tiles: 115x86 pinholes and 101x101 fisheyes, whose last tile row and
    # column hold pixels outside the image
    cams = grad_cameras(0.9 if case == "ragged_tiles" else 1.0)
    kw = {"floor_marginal": dict(use_floor=True),
          "no_floor": dict(),
          "centre_ray": dict(filter_mode=0, use_floor=True),
          "isotropic_floor": dict(filter_mode=2, use_floor=True),
          "rgb_additive": dict(use_floor=True, composition=1),
          "ray_integral_floor": dict(use_floor=True, backbone=1),
          "ragged_tiles": dict(use_floor=True)}[case]
    if kw.get("use_floor"):
        scene["rho2"] = O.bake_rho2(scene, [synth.scale_camera(c, 2.0) for c in cams]).astype(np.float32)
    oopts = O.Opts(**{k: (int(v) if isinstance(v, bool) else v) for k, v in kw.items()})
    gopts = R.RenderOpts(**kw)
    _say(f"backward {case}")
    refs = [O.render(scene, c, oopts, with_alt=True) for c in cams]
    G = upstream(cams, refs)
    ref = O.grad(scene, cams, G, oopts)
    g, rgba, info, mism = run_gpu(scene, cams, gopts, G)
    _say(f"   pairs {info['n_pairs']} replay mismatches {mism}")
    assert mism == 0
    worst = compare_grads(g, ref)
    for k, (rel, el, nbad) in worst.items():
        _say(f"   {k:15s} rel {rel:.2e} worst elem {el:.2e} bad {nbad}")
    for k, (rel, el, nbad) in worst.items():
        assert rel <= 1e-3, (k, rel)
        assert nbad == 0, (k, el, nbad)


def test_backward_with_cutoffs_matches_oracle_gradient():
    """Pairs clamped at alpha_max pass no gradient through T, and pixels stop before the
    pair that would take transmittance below T_min.  Ten SH Gaussians before a 96x72
    pinhole (several tiles and a ragged last tile row): Gaussian 0 near the camera is
    clamped at alpha_max = 0.95 on the central pixels, and the opaque Gaussian 1 behind
    it stops pixels at T_min = 3e-3.  The GPU gradient is held to the oracle's, whose
    cut-off branches are pinned to finite differences of whole renders.  Pixels where a
    pair's response lies within 1e-4 of alpha_max get no upstream gradient: there the
    FP32 and FP64 responses may fall on either side of the clamp."""
    from paper_2609_13397_amd import render as R
    sc = synth.make_scene(10, seed=23, layout="uniform", color="sh3", log_scale_mean=-2.0, log_scale_std=0.3)
    sc["means"] *= 0.6
    sc["means"][:, 0] = (0.02, -0.03, -1.8)
    sc["log_scales"][:, 0] = np.log([0.3, 0.25, 0.2])
    sc["opacity_logits"][0] = 9.0
    sc["means"][:, 1] = (0.1, 0.05, 0.9)
    sc["log_scales"][:, 1] = np.log([0.6, 0.5, 0.55])
    sc["opacity_logits"][1] = 6.0
    sc["rho2"] = np.full(10, 4e-4, np.float32)
    w, h = 96, 72
    cam = synth.camera(synth.PINHOLE, w, h, fx=80.0, fy=80.0, cx=w / 2, cy=h / 2, R_c2w=np.eye(3),
                       origin=(0.0, 0.0, -3.0))
    kw = dict(use_floor=True, alpha_max=0.95, T_min=3e-3)
    oopts = O.Opts(use_floor=1, alpha_max=0.95, T_min=3e-3)
    _say("backward with cut-offs")
    ref_img = O.render(sc, cam, oopts, with_alt=True)
    rays, _ = O.pixel_rays(cam)
    T = np.stack([O.pair_batch(sc, i, np.array(cam["origin"]), rays.reshape(-1, 9), oopts)[:, 0]
                  for i in range(sc["n"])])
    clamped = (T >= oopts.alpha_max).sum()
    stopped = int((ref_img["n_contrib"] < (T >= oopts.alpha_min).sum(0).reshape(h, w)).sum())
    _say(f"   clamped pairs {clamped} stopped pixels {stopped}")
    assert clamped >= 50 and stopped >= 20
    G = upstream([cam], [ref_img])
    near_clamp = (np.abs(T - oopts.alpha_max) < 1e-4).any(0).reshape(h, w)
    G[0][near_clamp] = 0.0
    ref = O.grad(sc, [cam], G, oopts)
    g, rgba, info, mism = run_gpu(sc, [cam], R.RenderOpts(**kw), G)
    _say(f"   pairs {info['n_pairs']} replay mismatches {mism} near-clamp pixels {int(near_clamp.sum())}")
    assert mism == 0
    worst = compare_grads(g, ref)
    for k, (rel, el, nbad) in worst.items():
        _say(f"   {k:15s} rel {rel:.2e} worst elem {el:.2e} bad {nbad}")
    for k, (rel, el, nbad) in worst.items():
        assert rel <= 1e-3, (k, rel)
        assert nbad == 0, (k, el, nbad)


def test_backward_deterministic_and_autograd():
    import torch
    from paper_2609_13397_amd import render as R
    scene = grad_scene()
    scene["rho2"] = O.bake_rho2(scene, grad_cameras(2.0)).astype(np.float32)
    cams = grad_cameras()
    opts = R.RenderOpts(use_floor=True)
    _say("backward determinism + autograd")
    G = [synth.seeded_image((c["crop"][3], c["crop"][2], 4), seed=11 + v) for v, c in enumerate(cams)]
    g1, _, _, _ = run_gpu(scene, cams, opts, G)
    g2, _, _, _ = run_gpu(scene, cams, opts, G)
    for k in GROUPS:
        assert np.array_equal(g1[k], g2[k]), k
    sc = R.Scene.from_numpy(scene)
    params = [getattr(sc, k).clone().requires_grad_(True) for k in GROUPS]
    rgba = R.ConeGaussRender.apply(*params, sc.rho2, cams, opts, sc.color_mode)
    Gt = torch.from_numpy(np.concatenate([x.reshape(-1, 4) for x in G])).cuda()
    (rgba * Gt).sum().backward()
    for k, p in zip(GROUPS, params):
        assert np.array_equal(p.grad.cpu().numpy().astype(np.float64), g1[k]), k


def test_backward_repeated_and_on_a_side_stream():
    """The backward returns without a host synchronisation, and its counters live in the
    forward state or its own scratch: two backward calls on one state, the second on
    another stream, give identical gradients and exact replays, and the state can be
    released after a backward on another stream."""
    import torch
    from paper_2609_13397_amd import render as R
    scene = grad_scene(seed=5)
    scene["rho2"] = O.bake_rho2(scene, grad_cameras(2.0)).astype(np.float32)
    cams = grad_cameras()
    opts = R.RenderOpts(use_floor=True)
    _say("backward twice on one state, the second on a side stream")
    sc = R.Scene.from_numpy(scene)
    _, _, state = R.render_forward(sc, cams, opts, need_state=True)
    G = torch.from_numpy(np.concatenate([synth.seeded_image((c["crop"][3], c["crop"][2], 4), seed=31 + v).reshape(-1, 4)
                                         for v, c in enumerate(cams)]).astype(np.float32)).cuda()
    g1 = R.render_backward(state, G, sc)
    m1 = R.replay_mismatches(state)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        g2 = R.render_backward(state, G, sc)
    state.release()  # waits for the side stream's backward before the blocks go back
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    assert m1 == 0
    for k in GROUPS:
        assert torch.equal(g1[k], g2[k]), k
    _, _, state = R.render_forward(sc, cams, opts, need_state=True)
    with torch.cuda.stream(side):
        side.wait_stream(torch.cuda.default_stream())
        R.render_backward(state, G, sc)
    assert R.replay_mismatches(state) == 0  # read after the side stream's backward
    state.release()
    torch.cuda.synchronize()


def test_backward_after_pair_buffers_guessed_too_small():
    """A training forward shaped like the previous one sizes its pair buffers from that
    call's pair count; one with far more pairs emits again into buffers of the right
    size.  Its gradients equal those of the same forward without a guess."""
    import torch
    from paper_2609_13397_amd import render as R
    cams = grad_cameras()[:2]
    opts = R.RenderOpts()
    small = synth.make_scene(512, seed=6, layout="uniform", color="rgb", log_scale_mean=-4.0, log_scale_std=0.3)
    big = dict(small)
    big["log_scales"] = small["log_scales"] + 2.0
    other = synth.subset_scene(small, np.arange(100))
    G = [synth.seeded_image((c["crop"][3], c["crop"][2], 4), seed=51 + v) for v, c in enumerate(cams)]
    _say("training forward + backward: big scene without a guess, then after the small one")
    run_gpu(other, cams, opts, G)
    g_ref, img_ref, info_ref, m_ref = run_gpu(big, cams, opts, G)
    _, _, info_small, _ = run_gpu(small, cams, opts, G)
    assert info_small["n_pairs"] + info_small["n_pairs"] // 16 + 4096 < info_ref["n_pairs"]
    g, img, info, m = run_gpu(big, cams, opts, G)
    assert m == 0 and m_ref == 0 and info["n_pairs"] == info_ref["n_pairs"]
    assert torch.equal(img, img_ref)
    for k in GROUPS:
        assert np.array_equal(g[k], g_ref[k]), k


def test_autograd_refuses_inputs_changed_in_place():
    """The backward reads the forward image and the parameters: changing either in
    place between the forward and the backward makes autograd raise instead of giving
    wrong gradients; an upstream gradient of the wrong shape or dtype is refused."""
    import torch
    from paper_2609_13397_amd import render as R
    scene, cam = synth.tiny_config()
    sc = R.Scene.from_numpy(scene)
    _say("autograd in-place checks")
    for which in ("image", "means"):
        params = [getattr(sc, k).clone().requires_grad_(True) for k in GROUPS]
        rgba = R.ConeGaussRender.apply(*params, sc.rho2, [cam], R.RenderOpts(), sc.color_mode)
        loss = rgba.sum()
        if which == "image":
            rgba.clamp_(0.0, 0.5)  # an in-place op on the saved output
        else:
            with torch.no_grad():
                params[0].add_(0.01)
        with pytest.raises(RuntimeError, match="inplace"):
            loss.backward()
    _, _, st = R.render_forward(sc, [cam], R.RenderOpts(), need_state=True)
    npx = cam["crop"][2] * cam["crop"][3]
    for bad in (torch.zeros((npx, 3), device="cuda"), torch.zeros((npx, 4), device="cuda", dtype=torch.float64),
                torch.zeros((npx, 4))):
        with pytest.raises(ValueError, match="grad_rgba"):
            R.render_backward(st, bad, sc)
    grads = R.render_backward(st, torch.zeros((npx, 4), device="cuda"), sc)
    torch.cuda.synchronize()
    st.release()
    assert all(float(v.abs().max()) == 0.0 for v in grads.values())


@pytest.mark.parametrize("kw", [dict(use_floor=True), dict(use_floor=True, count_pairs=True),
                                dict(filter_mode=2, use_floor=True), dict(filter_mode=0)],
                         ids=["floor", "floor_counting", "iso_floor", "centre"])
def test_training_forward_image_equals_inference(kw):
    """The training forward (state kept, per-wave replay mask recorded) renders the same
    image bit for bit as the inference forward, on ragged multi-view input (4 views
    whose sizes are not multiples of the 16-pixel tile)."""
    import torch
    from paper_2609_13397_amd import render as R
    scene = grad_scene(n=700, seed=7)
    scene["rho2"] = O.bake_rho2(scene, grad_cameras(2.0)).astype(np.float32)
    cams = [synth.with_crop(c, 3, 5, c["crop"][2] - 9, c["crop"][3] - 7) for c in grad_cameras()]
    sc = R.Scene.from_numpy(scene)
    opts = R.RenderOpts(**kw)
    a, ia, _ = R.render_forward(sc, cams, opts)
    a = a.clone()
    b, ib, st = R.render_forward(sc, cams, opts, need_state=True)
    torch.cuda.synchronize()
    st.release()
    _say(f"   pairs {ia['n_pairs']} / {ib['n_pairs']}")
    assert ia["n_pairs"] == ib["n_pairs"] and ia["n_pairs"] > 0
    assert torch.equal(a, b)


def test_backward_degenerate_inputs():
    """No pairs (one Gaussian behind the camera) gives zero gradients and an exact
    replay; an empty scene gives empty gradients; a zero-sized crop beside a normal
    view leaves that view's gradient unchanged."""
    from paper_2609_13397_amd import render as R
    scene, cam = synth.tiny_config()
    scene = dict(scene)
    w, h = cam["crop"][2], cam["crop"][3]
    G = [synth.seeded_image((h, w, 4), seed=3)]
    _say("backward with no pairs")
    behind = synth.subset_scene(scene, np.arange(1))
    behind["means"] = np.array([[0.0], [0.0], [-5.0]], np.float32)
    g, _, info, mism = run_gpu(behind, [cam], R.RenderOpts(), G)
    assert info["n_pairs"] == 0 and mism == 0
    for k in GROUPS:
        assert g[k].size > 0 and np.all(g[k] == 0.0), k
    _say("backward of an empty scene")
    g, _, info, mism = run_gpu(synth.subset_scene(scene, np.arange(0)), [cam], R.RenderOpts(), G)
    assert info["n_pairs"] == 0
    for k in GROUPS:
        assert g[k].size == 0, k
    _say("backward with a zero-sized crop beside a normal view")
    g1, _, _, m1 = run_gpu(scene, [cam], R.RenderOpts(), G)
    g2, _, _, m2 = run_gpu(scene, [synth.with_crop(cam, 0, 0, 0, 0), cam], R.RenderOpts(),
                           [np.zeros((0, 0, 4), np.float32)] + G)
    assert m1 == 0 and m2 == 0
    for k in GROUPS:
        np.testing.assert_allclose(g2[k], g1[k], rtol=1e-6, atol=1e-9, err_msg=k)
    _say("backward of a call whose views are all empty")
    c0 = synth.with_crop(cam, 0, 0, 0, 0)
    g, _, info, mism = run_gpu(scene, [c0, c0], R.RenderOpts(), [np.zeros((0, 0, 4), np.float32)] * 2)
    assert info["n_pairs"] == 0 and mism == 0
    for k in GROUPS:
        assert g[k].size > 0 and np.all(g[k] == 0.0), k
