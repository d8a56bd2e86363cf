"""Python side of the render server: ctypes binding of the cg_server_* calls and a
Poisson load generator that reports latency percentiles and throughput.

The scheduling itself (admission, batching, worker streams) is the C++ server; this
module only marshals arguments and replays request traces against it.
"""
from __future__ import annotations

import ctypes as C
import time
from dataclasses import dataclass
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import _lib


class CgServerConfig(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_size_t), ("max_batch_views", C.c_int32), ("n_workers", C.c_int32),
                ("max_batch_pixels", C.c_int64), ("fake_executor", C.c_int32), ("device", C.c_int32),
                ("fake_ns_per_pixel", C.c_double), ("fake_ns_per_call", C.c_double),
                ("request_timeout_ms", C.c_double), ("max_batch_pairs", C.c_double)]


class CgServerCompletion(C.Structure):
    _fields_ = [("request_id", C.c_int64), ("status", C.c_int32), ("scene", C.c_int32), ("batch_views", C.c_int32),
                ("reserved", C.c_int32), ("t_submit", C.c_double), ("t_admit", C.c_double),
                ("t_start", C.c_double), ("t_done", C.c_double), ("n_pairs", C.c_int64)]


class CgServerStats(C.Structure):
    _fields_ = [("queued", C.c_int64), ("in_flight", C.c_int64), ("completed", C.c_int64), ("batches", C.c_int64),
                ("views", C.c_int64), ("max_batch_views", C.c_int64), ("reserved_bytes", C.c_int64),
                ("peak_reserved_bytes", C.c_int64), ("timed_out", C.c_int64)]


SERVER_SIGNATURES = {
    "cg_server_default_config": (None, [C.c_void_p]),
    "cg_server_create": (C.c_int, [C.c_void_p, C.c_void_p]),
    "cg_server_add_scene": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "cg_server_submit": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "cg_server_cancel": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p]),
    "cg_server_poll": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_int32]),
    "cg_server_drain": (C.c_int, [C.c_void_p]),
    "cg_server_get_stats": (C.c_int, [C.c_void_p, C.c_void_p]),
    "cg_server_destroy": (None, [C.c_void_p]),
    "cg_server_now": (C.c_double, []),
}


def _L():
    L = _lib.lib()
    if not getattr(L, "_server_sigs", False):
        for name, (res, args) in SERVER_SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        L._server_sigs = True
    return L


def default_config(**kw) -> CgServerConfig:
    c = CgServerConfig()
    _L().cg_server_default_config(_lib.byref(c))
    for k, v in kw.items():
        setattr(c, k, v)
    return c


class RenderServer:
    """A cg_server.  Scenes and output buffers must stay alive while in use."""

    def __init__(self, config: Optional[CgServerConfig] = None, **kw):
        self.config = config or default_config(**kw)
        h = C.c_void_p()
        _lib.check(_L().cg_server_create(_lib.byref(self.config), C.byref(h)))
        self.h = h
        self._keep = []

    def add_scene(self, g: _lib.CgGaussians, opts: _lib.CgOpts, keep=None) -> int:
        sid = C.c_int32()
        _lib.check(_L().cg_server_add_scene(self.h, _lib.byref(g), _lib.byref(opts), C.byref(sid)))
        self._keep.append((g, opts, keep))
        return sid.value

    def submit(self, scene: int, cam: _lib.CgCamera, out_ptr: int) -> int:
        rid = C.c_int64()
        _lib.check(_L().cg_server_submit(self.h, scene, _lib.byref(cam), C.c_void_p(out_ptr), C.byref(rid)))
        return rid.value

    def cancel(self, rid: int) -> bool:
        c = C.c_int32()
        _lib.check(_L().cg_server_cancel(self.h, rid, C.byref(c)))
        return bool(c.value)

    def poll(self, capacity: int = 256, wait_ms: int = 0) -> List[CgServerCompletion]:
        arr = (CgServerCompletion * capacity)()
        n = C.c_int32()
        _lib.check(_L().cg_server_poll(self.h, C.cast(arr, C.c_void_p), capacity, C.byref(n), wait_ms))
        return [arr[i] for i in range(n.value)]

    def drain(self):
        _lib.check(_L().cg_server_drain(self.h))

    def stats(self) -> Dict[str, int]:
        s = CgServerStats()
        _lib.check(_L().cg_server_get_stats(self.h, _lib.byref(s)))
        return {f: getattr(s, f) for f, _ in CgServerStats._fields_}

    def close(self):
        if self.h:
            _L().cg_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def now() -> float:
    return _L().cg_server_now()


@dataclass
class TraceResult:
    latencies_ms: np.ndarray
    pixels: int
    wall_s: float
    batch_views: np.ndarray
    statuses: np.ndarray

    def summary(self) -> dict:
        lat = self.latencies_ms
        # render calls by the number of views they fused (a call of k views completes k
        # requests, each reporting k)
        calls = {int(k): int(round((self.batch_views == k).sum() / k)) for k in np.unique(self.batch_views) if k > 0}
        return {"requests": int(lat.size), "p50_ms": float(np.percentile(lat, 50)),
                "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean()),
                "mpix_per_s": self.pixels / self.wall_s / 1e6, "wall_s": self.wall_s,
                "mean_batch_views": float(self.batch_views.mean()),
                "calls_by_views": calls,
                "failed": int((self.statuses != 0).sum())}


def replay(server: RenderServer, scene_ids: Sequence[int], requests, out_ptrs: Sequence[int],
           camera_struct, time_scale: float = 1.0, burst: bool = False) -> TraceResult:
    """Submits `requests` (synth.Request) at their arrival times (or all at once with
    burst=True), waits for all completions, and returns latencies (completion minus
    submission, server clock) and throughput (pixels over first submission to last
    completion)."""
    structs = [camera_struct(r.camera) for r in requests]
    t0 = time.perf_counter()
    done = []
    for r, cs, ptr in zip(requests, structs, out_ptrs):
        if not burst:
            wait = r.arrival_s * time_scale - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
        server.submit(scene_ids[r.scene], cs, ptr)
        done.extend(server.poll(256, 0))
    while len(done) < len(requests):
        done.extend(server.poll(256, 100))
    lat = np.array([(c.t_done - c.t_submit) * 1e3 for c in done])
    first = min(c.t_submit for c in done)
    last = max(c.t_done for c in done)
    px = sum(r.pixels for r in requests)
    return TraceResult(lat, px, last - first, np.array([c.batch_views for c in done]),
                       np.array([c.status for c in done]))
