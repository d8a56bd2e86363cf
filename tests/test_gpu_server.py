"""The render server on the GPU: every request's image is the same whether it is
rendered alone or fused with others in a continuous batch (bit for bit: a fused call
renders each view exactly as a call with that view alone), and a small HBM budget
only delays requests."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2609_13397_amd import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _setup(n_scenes=2, sizes=(20000, 40000)):
    import torch
    from paper_2609_13397_amd import render as R
    scenes = []
    for k in range(n_scenes):
        sc = synth.make_scene(sizes[k], seed=60 + k, layout="clusters", color="sh3", log_scale_mean=-3.5,
                              log_scale_std=0.6)
        t = R.Scene.from_numpy(sc)
        t.rho2 = R.bake_rho2(t, synth.orbit_views(), 0.2)
        scenes.append(t)
    torch.cuda.synchronize()
    return scenes


def _serve(scenes, reqs, **cfg):
    import torch
    from paper_2609_13397_amd import render as R
    from paper_2609_13397_amd import serving
    srv = serving.RenderServer(serving.default_config(**cfg))
    opts = R.RenderOpts(use_floor=True).to_c()
    sids = [srv.add_scene(s.to_c(), opts, keep=s) for s in scenes]
    outs = [torch.full((r.pixels, 4), -1.0, device="cuda") for r in reqs]
    res = serving.replay(srv, sids, reqs, [o.data_ptr() for o in outs], R.camera_struct, burst=True)
    stats = srv.stats()
    srv.close()
    torch.cuda.synchronize()
    return outs, res, stats


def test_served_equals_alone():
    import torch
    from paper_2609_13397_amd import render as R
    scenes = _setup()
    reqs = synth.serving_trace(48, qps=1000.0, seed=71, n_scenes=2, scales=(0.125, 0.25, 0.5))
    _say("server: batched, 3 workers")
    outs, res, stats = _serve(scenes, reqs, n_workers=3, max_batch_views=8)
    _say(f"   {res.summary()} stats {stats}")
    assert (res.statuses == 0).all()
    assert stats["max_batch_views"] > 1  # requests were actually fused
    for r, out in zip(reqs, outs):
        alone, _, _ = R.render_forward(scenes[r.scene], [r.camera], R.RenderOpts(use_floor=True))
        assert torch.equal(out, alone), r.rid


def test_served_equals_alone_all_scales_and_split_views():
    """Requests at every serving scale, 1/8 to x8 (the x2..x8 ones crops of the base size
    of a larger virtual image), over a 20k and a 500k scene: small views of the 500k scene
    take the split tile render (decided per view, from the view's own lists), fused or
    alone.  Every served image equals the request rendered alone, bit for bit."""
    import torch
    from paper_2609_13397_amd import render as R
    scenes = _setup(2, (20000, 500000))
    reqs = synth.serving_trace(40, qps=1000.0, seed=74, n_scenes=2)
    _say("server: all scales, 3 workers")
    outs, res, stats = _serve(scenes, reqs, n_workers=3, max_batch_views=8)
    _say(f"   {res.summary()} stats {stats}")
    assert (res.statuses == 0).all()
    assert stats["max_batch_views"] > 1
    n_split = 0
    for r, out in zip(reqs, outs):
        alone, info, _ = R.render_forward(scenes[r.scene], [r.camera], R.RenderOpts(use_floor=True))
        n_split += info["n_segments"] > 0
        assert torch.equal(out, alone), (r.rid, r.camera["full_w"], r.camera["crop"], info["n_segments"])
    zoomed = sum(r.camera["full_w"] > 2048 for r in reqs)
    _say(f"   requests rendered alone with the split tile render: {n_split}; zoomed crops: {zoomed}")
    assert n_split > 0 and zoomed > 0


def test_served_matches_oracle_sample():
    """One served view checked against the FP64 oracle (a small scene so the oracle is
    quick), to tie the serving path to the same parity bar as the renderer."""
    import torch
    from paper_2609_13397_amd import render as R
    from parity import compare_image
    sc_np = synth.make_scene(3000, seed=73, layout="clusters", color="sh3", log_scale_mean=-3.0, log_scale_std=0.5)
    cam = synth.scale_camera(synth.orbit_views(1)[0], 0.0625)
    sc_np["rho2"] = O.bake_rho2(sc_np, [synth.scale_camera(cam, 2.0)]).astype(np.float32)
    scene = R.Scene.from_numpy(sc_np)
    reqs = [synth.Request(0, 0.0, 0, cam), synth.Request(1, 0.0, 0, synth.scale_camera(cam, 0.5))]
    outs, res, _ = _serve([scene], reqs, n_workers=2, max_batch_views=4)
    img = outs[0].view(cam["crop"][3], cam["crop"][2], 4).cpu().numpy().astype(np.float64)
    ref = O.render(sc_np, cam, O.Opts(use_floor=1), with_alt=True)
    nfail, worst, det = compare_image(img, ref)
    _say(f"   served vs oracle: fail={nfail} worst={worst:.2e}")
    assert nfail == 0


def test_tiny_budget_delays_but_completes():
    scenes = _setup(1, (200000,))
    reqs = synth.serving_trace(12, qps=1000.0, seed=72, n_scenes=1, scales=(0.25, 0.5))
    budget = 256 << 20
    _say("server: 256 MiB budget")
    outs, res, stats = _serve(scenes, reqs, n_workers=4, max_batch_views=4, hbm_budget_bytes=budget)
    _say(f"   {res.summary()} stats {stats}")
    assert (res.statuses == 0).all()
    # a 200k-Gaussian view needs ~35 MiB of per-Gaussian scratch: several fit, not all twelve
    assert stats["peak_reserved_bytes"] <= budget
