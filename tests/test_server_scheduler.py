"""Scheduler logic of the render server, on the CPU: the server's stand-in executor
(a timed sleep) replaces rendering, so admission, batching, ordering, back-pressure
and cancellation are tested without a GPU."""
import os

import numpy as np
import pytest

from paper_2609_13397_amd import _lib, synth

pytestmark = pytest.mark.skipif(not os.path.exists(_lib.LIB_PATH), reason="library not built")


def _fake_scene(n=1000):
    """A host-side stand-in scene: the fake executor never dereferences the pointers."""
    buf = np.zeros(64 * n, np.float32)
    g = _lib.CgGaussians()
    g.n = n
    g.color_mode = 0
    for k in ("means", "log_scales", "quats", "opacity_logits", "color"):
        setattr(g, k, buf.ctypes.data)
    g.rho2 = None
    o = _lib.CgOpts()
    _lib.lib().cg_default_opts(_lib.byref(o))
    return g, o, buf


def _server(**kw):
    from paper_2609_13397_amd import serving
    base = dict(fake_executor=1, fake_ns_per_call=2e5, fake_ns_per_pixel=2.0)
    base.update(kw)
    cfg = serving.default_config(**base)
    return serving.RenderServer(cfg)


def _cam(w=64, h=48):
    from paper_2609_13397_amd.render import camera_struct
    return camera_struct(synth.camera(synth.PINHOLE, w, h, fx=50.0, fy=50.0, cx=w / 2, cy=h / 2))


def _collect(s, n):
    out = []
    while len(out) < n:
        out.extend(s.poll(64, 200))
    return out


def test_fifo_single_worker_per_view():
    s = _server(n_workers=1, max_batch_views=1)
    g, o, keep = _fake_scene()
    sid = s.add_scene(g, o, keep)
    ids = [s.submit(sid, _cam(), 1) for _ in range(12)]
    done = _collect(s, 12)
    assert [c.request_id for c in done] == ids
    assert all(c.batch_views == 1 and c.status == 0 for c in done)
    assert all(c.t_submit <= c.t_admit <= c.t_start <= c.t_done for c in done)
    st = s.stats()
    assert st["batches"] == 12 and st["max_batch_views"] == 1
    s.close()


def test_requests_queued_behind_a_running_call_are_fused():
    s = _server(n_workers=1, max_batch_views=4)
    g, o, keep = _fake_scene()
    sid = s.add_scene(g, o, keep)
    for _ in range(9):
        s.submit(sid, _cam(), 1)
    done = _collect(s, 9)
    views = sorted(c.batch_views for c in done)
    # the first call starts alone; the rest arrive while it runs and are fused 4 at a time
    assert max(views) == 4
    assert s.stats()["batches"] < 9
    s.close()


def test_batches_never_mix_scenes_and_respect_pixel_cap():
    s = _server(n_workers=1, max_batch_views=8, max_batch_pixels=64 * 48 * 3)
    g, o, keep = _fake_scene()
    a = s.add_scene(g, o, keep)
    b = s.add_scene(g, o, keep)
    rid_scene = {}
    for k in range(16):
        sc = a if k % 2 == 0 else b
        rid_scene[s.submit(sc, _cam(), 1)] = sc
    done = _collect(s, 16)
    by_start = {}
    for c in done:
        by_start.setdefault(c.t_start, []).append(c)
    for group in by_start.values():
        assert len({c.scene for c in group}) == 1
        assert len(group) <= 3
        assert all(rid_scene[c.request_id] == c.scene for c in group)
    s.close()


def test_hbm_budget_back_pressure():
    """With a budget that fits about two requests, admitted scratch never exceeds it and
    requests wait in the queue instead of failing."""
    g, o, keep = _fake_scene(n=100000)
    one = 100000 * 192 + (1 << 20)  # the per-Gaussian part of a request's estimate
    s = _server(n_workers=4, max_batch_views=1, hbm_budget_bytes=int(2.5 * one) + (1 << 21))
    sid = s.add_scene(g, o, keep)
    for _ in range(20):
        s.submit(sid, _cam(), 1)
    done = _collect(s, 20)
    st = s.stats()
    assert all(c.status == 0 for c in done)
    assert st["peak_reserved_bytes"] <= s.config.hbm_budget_bytes
    # at most two calls overlap in time
    ev = sorted([(c.t_start, 1) for c in done] + [(c.t_done, -1) for c in done])
    run = peak = 0
    for _, d in ev:
        run += d
        peak = max(peak, run)
    assert peak <= 2
    s.close()


def test_oversized_request_still_runs_alone():
    g, o, keep = _fake_scene(n=100000)
    s = _server(n_workers=2, max_batch_views=4, hbm_budget_bytes=1 << 20)
    sid = s.add_scene(g, o, keep)
    for _ in range(3):
        s.submit(sid, _cam(), 1)
    done = _collect(s, 3)
    assert all(c.status == 0 and c.batch_views == 1 for c in done)
    s.close()


def test_cancel_queued_request_and_invalid_submit():
    s = _server(n_workers=1, max_batch_views=1, fake_ns_per_call=5e6)
    g, o, keep = _fake_scene()
    sid = s.add_scene(g, o, keep)
    ids = [s.submit(sid, _cam(), 1) for _ in range(4)]
    assert s.cancel(ids[-1])
    assert not s.cancel(123456)
    done = _collect(s, 4)
    st = {c.request_id: c.status for c in done}
    assert st[ids[-1]] == -5 and all(st[i] == 0 for i in ids[:-1])
    bad = _cam()
    bad.model = 9
    with pytest.raises(_lib.CgError):
        s.submit(sid, bad, 1)
    with pytest.raises(_lib.CgError):
        s.submit(7, _cam(), 1)
    s.drain()
    s.close()


def test_request_timeout_completes_unrendered():
    """A request still queued past request_timeout_ms completes with CG_ERR_TIMEOUT and
    is never handed to the executor; the one admitted at once completes normally."""
    s = _server(n_workers=1, max_batch_views=1, fake_ns_per_call=80e6, fake_ns_per_pixel=0.0,
                request_timeout_ms=20.0)
    g, o, keep = _fake_scene()
    sid = s.add_scene(g, o, keep)
    ids = [s.submit(sid, _cam(), 1) for _ in range(4)]
    s.drain()
    done = {c.request_id: c for c in _collect(s, 4)}
    assert done[ids[0]].status == 0
    for rid in ids[1:]:
        c = done[rid]
        assert c.status == -6, c.status  # CG_ERR_TIMEOUT
        assert c.t_done - c.t_submit >= 0.020
        assert c.batch_views == 0 and c.t_start == 0.0  # never started
    st = s.stats()
    assert st["timed_out"] == 3 and st["batches"] == 1 and st["completed"] == 4
    s.close()


def test_request_timeout_generous_limit_changes_nothing():
    s = _server(n_workers=2, max_batch_views=4, request_timeout_ms=10000.0)
    g, o, keep = _fake_scene()
    sid = s.add_scene(g, o, keep)
    ids = [s.submit(sid, _cam(), 1) for _ in range(16)]
    done = _collect(s, 16)
    assert sorted(c.request_id for c in done) == sorted(ids)
    assert all(c.status == 0 for c in done)
    assert s.stats()["timed_out"] == 0
    s.close()


def test_negative_timeout_is_an_argument_error():
    from paper_2609_13397_amd import serving
    with pytest.raises(_lib.CgError, match="request_timeout_ms"):
        serving.RenderServer(serving.default_config(fake_executor=1, request_timeout_ms=-1.0))
