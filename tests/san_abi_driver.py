"""Exercises the host code of the C ABI in a process that loads a build of the library
whose host code is instrumented (ASan + UBSan): argument checking of every entry
point (no GPU is needed: each call returns an error before any device work, or a
HIP error where there is no device), the debugging and profiling switches, and the
render server's scheduler under its CPU stand-in executor, with submissions from
several threads, cancellation, time limits and shutdown with requests queued.
Started by test_sanitizers.py.  argv[1]: path of the instrumented library."""
import ctypes as C
import math
import os
import sys
import threading

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

from paper_2609_13397_amd import _lib, serving, synth  # noqa: E402
from paper_2609_13397_amd.render import camera_struct  # noqa: E402

L = C.CDLL(sys.argv[1])
for name, (res, args) in {**_lib.SIGNATURES, **serving.SERVER_SIGNATURES}.items():
    f = getattr(L, name)
    f.restype = res
    f.argtypes = args
_lib._LIB = L  # the serving wrapper calls through the instrumented build
serving._L = lambda: L


def expect_error(status, what):
    assert status != 0, f"{what}: accepted"
    msg = L.cg_last_error()
    assert msg, f"{what}: no message"
    return msg.decode()


def host_scene(n=64, color_mode=0):
    buf = np.zeros(64 * max(n, 1), np.float32)
    g = _lib.CgGaussians()
    g.n = n
    g.color_mode = color_mode
    for k in ("means", "log_scales", "quats", "opacity_logits", "color"):
        setattr(g, k, buf.ctypes.data)
    g.rho2 = None
    return g, buf


def main():
    assert L.cg_version() >= 1
    o = _lib.CgOpts()
    L.cg_default_opts(_lib.byref(o))
    L.cg_default_opts(None)
    g, keep = host_scene()
    cam = camera_struct(synth.camera(synth.PINHOLE, 32, 24, fx=30.0, fy=30.0, cx=16.0, cy=12.0))
    out = np.zeros(32 * 24 * 4, np.float32)
    st = _lib.CgStats()
    fwd = L.cg_render_forward
    bp = _lib.byref
    ptr = C.c_void_p(out.ctypes.data)

    def forward(g_=None, cam_=None, n=1, o_=None, out_=ptr):
        return fwd(bp(g_ or g), bp(cam_ or cam), n, bp(o_ or o), None, out_, None, bp(st), None)

    expect_error(fwd(None, None, 1, None, None, None, None, None, None), "null scene")
    for n in (0, -1, 4097):
        expect_error(forward(n=n), f"n_views {n}")
    bad_cams = []
    for field, value in (("model", 7), ("crop_w", -1), ("crop_x0", 30), ("full_w", 0), ("fx", float("nan")),
                         ("fy", 0.0), ("theta_max", -1.0)):
        c = camera_struct(synth.camera(synth.PINHOLE, 32, 24, fx=30.0, fy=30.0, cx=16.0, cy=12.0))
        setattr(c, field, value)
        bad_cams.append((field, c))
    fc = camera_struct(synth.kb_camera(32, 32, 100.0, (0.0, 0.0, 0.0, 0.0), 12.0, np.eye(3), (0.0, 0.0, 0.0)))
    fc.theta_max = 4.0
    bad_cams.append(("theta_max", fc))
    for field, c in bad_cams:
        expect_error(forward(cam_=c), f"camera {field}")
    for field, value in (("filter_mode", 5), ("composition", 3), ("order_mode", 9), ("backbone", 4),
                         ("alpha_min", -0.5), ("alpha_max", 1.5), ("T_min", float("nan")), ("t_near", -1.0),
                         ("footprint_scale", 0.0)):
        ob = _lib.CgOpts()
        L.cg_default_opts(bp(ob))
        setattr(ob, field, value)
        expect_error(forward(o_=ob), f"option {field}")
    for field, value in (("n", -1), ("color_mode", 9), ("means", None)):
        gb, kb = host_scene()
        setattr(gb, field, value)
        expect_error(forward(g_=gb), f"scene {field}")
    expect_error(forward(out_=None), "null output")
    # every check passed: the call reaches the device (none here) and reports it
    forward()
    expect_error(L.cg_render_forward_noalloc(None, None, 1, None, None, None, None), "noalloc null")
    expect_error(L.cg_render_backward(None, None, None, None, None, None, None, None), "backward null state")
    L.cg_fwd_state_release(None)
    assert L.cg_bwd_replay_mismatches(None) < 0
    xy = np.zeros(8, np.float32)
    expect_error(L.cg_camera_unproject(None, 4, None, None, None, None), "unproject null")
    expect_error(L.cg_camera_unproject(bp(cam), -1, C.c_void_p(xy.ctypes.data), None, None, None), "unproject n")
    expect_error(L.cg_bake_rho2(None, None, 1, 0.2, None, None), "bake null")
    expect_error(L.cg_bake_rho2(bp(g), bp(cam), 0, 0.2, None, None), "bake n_views")
    # profiling and debugging switches
    n_st = L.cg_profile_num_stages()
    names = [L.cg_profile_stage_name(i) for i in range(-2, n_st + 2)]
    assert all(nm for nm in names[2:2 + n_st]) and not names[0] and not names[-1]
    L.cg_profile_enable(0)
    L.cg_profile_enable_stages(0)
    assert L.cg_profile_collect() == 0
    ms = np.zeros(n_st, np.float64)
    cnt = np.zeros(n_st, np.int64)
    L.cg_profile_read(C.c_void_p(ms.ctypes.data), C.c_void_p(cnt.ctypes.data))
    for args in ((1, 1, 1), (0, 0, 0), (-5, -5, -5)):
        L.cg_set_tile_split(*args)
    for mode in (1, 2, 99, 0):
        L.cg_debug_set_scratch_guards(mode)
    assert L.cg_debug_guard_violations() == 0
    server_checks()
    print("host ABI ran clean", flush=True)


def server_checks():
    bad = serving.default_config(fake_executor=1)
    for field, value in (("n_workers", 0), ("max_batch_views", 0), ("max_batch_pixels", 0),
                         ("hbm_budget_bytes", 0), ("request_timeout_ms", -1.0)):
        cfg = serving.default_config(fake_executor=1)
        setattr(cfg, field, value)
        h = C.c_void_p()
        expect_error(L.cg_server_create(_lib.byref(cfg), C.byref(h)), f"server {field}")
    g, keep = host_scene(256)
    o = _lib.CgOpts()
    L.cg_default_opts(_lib.byref(o))
    cam = camera_struct(synth.camera(synth.PINHOLE, 64, 48, fx=50.0, fy=50.0, cx=32.0, cy=24.0))
    for timeout in (0.0, 2.0):
        srv = serving.RenderServer(serving.default_config(fake_executor=1, n_workers=3, max_batch_views=4,
                                                          fake_ns_per_call=2e5, fake_ns_per_pixel=1.0,
                                                          hbm_budget_bytes=1 << 20, request_timeout_ms=timeout))
        sid = srv.add_scene(g, o, keep)
        with_crop = camera_struct(synth.with_crop(synth.camera(synth.PINHOLE, 64, 48, fx=50.0, fy=50.0, cx=32.0,
                                                               cy=24.0), 8, 8, 16, 16))
        ids = []
        lock = threading.Lock()

        def submitter(k):
            for i in range(40):
                rid = srv.submit(sid, cam if (i + k) % 3 else with_crop, 1)
                with lock:
                    ids.append(rid)

        threads = [threading.Thread(target=submitter, args=(k,)) for k in range(3)]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        cancelled = sum(srv.cancel(rid) for rid in ids[::7])
        assert not srv.cancel(-12345)
        h = C.c_int64()
        expect_error(L.cg_server_submit(srv.h, 99, _lib.byref(cam), C.c_void_p(1), C.byref(h)), "unknown scene")
        bad_cam = camera_struct(synth.camera(synth.PINHOLE, 64, 48, fx=50.0, fy=50.0, cx=32.0, cy=24.0))
        bad_cam.crop_w = 1000
        expect_error(L.cg_server_submit(srv.h, sid, _lib.byref(bad_cam), C.c_void_p(1), C.byref(h)), "bad camera")
        srv.drain()
        got = []
        while True:
            batch = srv.poll(16, 0)
            if not batch:
                break
            got.extend(batch)
        assert sorted(c.request_id for c in got) == sorted(ids), (len(got), len(ids), cancelled)
        stats = srv.stats()
        assert stats["completed"] + cancelled == len(ids)  # cancelled requests are not counted as completed
        assert math.isfinite(L.cg_server_now())
        # shut down with requests still queued
        for _ in range(30):
            srv.submit(sid, cam, 1)
        srv.close()


if __name__ == "__main__":
    main()
