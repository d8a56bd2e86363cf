"""Benchmark of the ConeGaussian hot path on one MI355X.

A step is one batched forward render (cg_render_forward) of the 1M-Gaussian fisheye
workload: 1M clustered Gaussians with degree-3 SH colour and the Eq. 11 floor baked
from 8 pinhole orbit views, rendered into a 190-degree Kannala-Brandt fisheye
(1600x1600) and an equirectangular view (2048x1024) -- 4.66 Mpixel per step, floor
and anisotropic footprint filter on, marginal composition.  Inputs are resident in
HBM before the timed region.

Prints one JSON line: throughput (Mpix/s), the roofline of the dominant kernel (the
tile render, ALU-bound: algorithmic flops = contributing pairs x flops per pair,
divided by the kernel's average duration from HIP events on its stream), and the FP64
CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic work per contributing (pixel, Gaussian) pair: flops of the closed form
# (FMA = 2), floor on / off, plus transcendentals, frozen before tuning; the backward
# is three times the forward per pair.
FLOPS_PER_PAIR = {True: 225, False: 156}
TRANSC_PER_PAIR = {True: 8, False: 4}
BWD_FLOPS_FACTOR = 3
PEAK_FP32_VECTOR_TFLOPS = 157.3   # MI355X published FP32 vector peak
PEAK_HBM_GBS = 8000.0
# Algorithmic HBM bytes, frozen before tuning: the render reads per pair a 4-byte
# Gaussian id and an 80-byte record and writes per pixel 24 bytes (RGBA and state);
# per Gaussian and view the preprocess reads 240 bytes of raw parameters (SH) and
# writes 100 bytes of record, key and cone; the sort moves 64 bytes per Gaussian and
# view plus 24 per pair; the backward writes and reads an 80-byte partial gradient per
# pair and writes 236 bytes of gradient per Gaussian.
BYTES_PER_PAIR = 84
BYTES_PER_PIXEL = 24
BYTES_RAW_PER_GAUSSIAN = 240
BYTES_RECORD_PER_ITEM = 100
BYTES_SORT_PER_ITEM, BYTES_SORT_PER_PAIR = 64, 24
BYTES_BWD_PARTIAL_PER_PAIR = 160
BYTES_BWD_GRAD_PER_GAUSSIAN = 236
# this design's render actually reads a 128-byte record per pair and a 64-byte ray
# record per pixel (reported beside the frozen figure)
DESIGN_BYTES_PER_PAIR = 132
DESIGN_BYTES_PER_PIXEL = 80


def frame_roofline_ms(n_gauss, n_views, pairs, pixels, contrib, floor=True, backward=False):
    """Time the whole step would take at the roofline: the tile render (and backward
    render) at the FP32 vector peak on their algorithmic flops, plus every algorithmic
    HBM byte of the step at 8 TB/s (stages bound by memory)."""
    flops = contrib * FLOPS_PER_PAIR[floor] * (1 + (BWD_FLOPS_FACTOR if backward else 0))
    items = n_gauss * n_views
    byts = (n_gauss * BYTES_RAW_PER_GAUSSIAN + items * BYTES_RECORD_PER_ITEM + items * BYTES_SORT_PER_ITEM +
            pairs * (BYTES_SORT_PER_PAIR + BYTES_PER_PAIR) + pixels * BYTES_PER_PIXEL)
    if backward:
        byts += pairs * BYTES_BWD_PARTIAL_PER_PAIR + n_gauss * BYTES_BWD_GRAD_PER_GAUSSIAN
    return (flops / (PEAK_FP32_VECTOR_TFLOPS * 1e12) + byts / (PEAK_HBM_GBS * 1e9)) * 1e3, flops, byts

# sources whose change invalidates the measured HBM traffic of the render kernel (the
# kernel itself, the pair arithmetic and culling it inlines, and the records it reads)
RENDER_SOURCES = ["paper_2609_13397_amd/csrc/render_fwd.hip", "paper_2609_13397_amd/csrc/pair_math.hpp",
                  "paper_2609_13397_amd/csrc/record_bounds.hpp", "paper_2609_13397_amd/csrc/camera_dev.hpp",
                  "paper_2609_13397_amd/csrc/cg_common.hpp", "paper_2609_13397_amd/csrc/preprocess.hip",
                  "paper_2609_13397_amd/csrc/pixel_buf.hpp", "paper_2609_13397_amd/csrc/wave_ops.hpp",
                  "paper_2609_13397_amd/csrc/camera.hip"]
# the anisotropic, marginal-floor, max-response, inference variant the bench times
TRAFFIC_KERNEL = "cg::k_render<1, true, false, false, false>"


def render_source_hash() -> str:
    h = hashlib.sha256()
    for p in RENDER_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic():
    """HBM traffic of the render kernel from rocprofv3 counters (profiles/), if taken
    on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "render_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("render_source_hash") != render_source_hash():
        return None
    return t


def build_workload(torch, R, synth, device):
    scene_np, cams = synth.fisheye_config()
    scene = R.Scene.from_numpy(scene_np, device=device)
    scene.rho2 = R.bake_rho2(scene, synth.orbit_views(), t_near=0.2)
    torch.cuda.synchronize()
    return scene_np, scene, cams


def order_ray_bench(torch, R, scene, cams, out_key, steps, warmup):
    """Per-ray compositing order (order_mode RAY) on the forward workload: throughput,
    pending-buffer overflows, and how far its image is from the key-order image."""
    opts = R.RenderOpts(filter_mode=R.FILTER_ANISOTROPIC, use_floor=True, order_mode=R.ORDER_RAY)
    npx = out_key.shape[0]
    out = torch.empty_like(out_key)
    _, info, _ = R.render_forward(scene, cams, opts, out=out)
    for _ in range(warmup):
        R.render_forward(scene, cams, opts, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        R.render_forward(scene, cams, opts, out=out)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    diff = (out.double() - out_key.double()).abs().amax(dim=1)
    return {"value": npx * steps / dt / 1e6, "unit": "Mpix/s", "ms_per_step": dt / steps * 1e3, "steps": steps,
            "n_order_overflow": int(info["n_order_overflow"]),
            "overflow_per_pixel": info["n_order_overflow"] / npx,
            "diff_vs_key_order": {"max": float(diff.max()), "rmse": float(diff.pow(2).mean().sqrt()),
                                  "frac_pixels_above_2e-4": float((diff > 2e-4).double().mean())}}


def train_step_bench(torch, R, synth, device, steps, warmup):
    """fwd + L1 + bwd on the training-step workload: 1M Gaussians, 2 orbit pinholes + 2
    centre fisheyes at 1280x720, L1 loss against the render of a perturbed copy of the
    scene (seeded), gradients for means / log-scales / rotations / opacity / SH."""
    scene_np, target_np, cams = synth.training_config()
    scene = R.Scene.from_numpy(scene_np, device=device)
    scene.rho2 = R.bake_rho2(scene, synth.orbit_views(), t_near=0.2)
    target = R.Scene.from_numpy(target_np, device=device)
    target.rho2 = scene.rho2
    opts = R.RenderOpts(filter_mode=R.FILTER_ANISOTROPIC, use_floor=True)
    with torch.no_grad():
        tgt, _, _ = R.render_forward(target, cams, opts)
        tgt = tgt.clone()
    params = [getattr(scene, k).clone().requires_grad_(True) for k in R.PARAM_NAMES]
    npx = sum(R.view_pixels(cams))

    def step():
        # gradients reset as an optimizer's zero_grad(set_to_none=True) does, so autograd
        # stores the library's gradient tensors instead of adding them into old ones
        for p in params:
            p.grad = None
        rgba = R.ConeGaussRender.apply(*params, scene.rho2, cams, opts, scene.color_mode)
        loss = (rgba - tgt).abs().mean()
        loss.backward()
        return loss

    # contributing pairs of the training forward (counting variant, outside the timed region)
    copts = R.RenderOpts(filter_mode=R.FILTER_ANISOTROPIC, use_floor=True, count_pairs=True)
    _, info, _ = R.render_forward(scene, cams, copts)
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    # timed region: HIP events bracket the backward render kernel only, for its roofline
    bprof = R.Profiler(stages=["bwd_render"])
    with bprof:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    bwd = bprof.read()["bwd_render"]
    # per-stage breakdown from a separate pass
    prof = R.Profiler()
    with prof:
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
    stages = prof.read()
    bwd_ms = bwd["ms"] / max(bwd["launches"], 1)
    bflops = info["n_contrib"] * FLOPS_PER_PAIR[True] * BWD_FLOPS_FACTOR
    achieved = bflops / (bwd_ms * 1e-3) / 1e12
    ms_per_step = dt / steps * 1e3
    frame_ms, _, frame_bytes = frame_roofline_ms(scene.n, len(cams), info["n_pairs"], npx, info["n_contrib"],
                                                 backward=True)
    return {"value": npx * steps / dt / 1e6, "unit": "Mpix/s", "ms_per_step": ms_per_step, "steps": steps,
            "workload": "train_1M: 1M Gaussians, 2 pinhole + 2 KB fisheye 1280x720, L1 vs seeded target",
            "pixels_per_step": npx, "pairs": info["n_pairs"],
            "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                         "frac": achieved / PEAK_FP32_VECTOR_TFLOPS, "kernel": "k_render_bwd (backward tile render)",
                         "kernel_ms": bwd_ms, "units_per_launch": info["n_contrib"], "unit_name": "contributing pair",
                         "flops_per_unit": FLOPS_PER_PAIR[True] * BWD_FLOPS_FACTOR},
            "frame_roofline": {"ms": frame_ms, "frac": frame_ms / ms_per_step, "algorithmic_bytes": frame_bytes},
            "stages_ms_per_step": {k: v["ms"] / steps for k, v in stages.items() if v["launches"]}}


def valu_ceiling(torch, R, device, blocks=256 * 8, iters=20000):
    """The FP32 FMA rate the chip sustains without packed instructions, from the
    library's calibration kernel (8 independent FMA chains per thread, 8 waves per
    SIMD): wave instructions per SIMD per clock and TFLOP/s, from HIP events."""
    from paper_2609_13397_amd import _lib
    L = _lib.lib()
    out = torch.zeros(1, dtype=torch.float32, device=device)
    stream = torch.cuda.current_stream(device).cuda_stream
    import ctypes as C
    _lib.check(L.cg_profile_valu_probe(blocks, iters, C.c_void_p(out.data_ptr()), C.c_void_p(stream)))
    prof = R.Profiler(stages=["valu_probe"])
    with prof:
        for _ in range(3):
            _lib.check(L.cg_profile_valu_probe(blocks, iters, C.c_void_p(out.data_ptr()), C.c_void_p(stream)))
        torch.cuda.synchronize()
    p = prof.read()["valu_probe"]
    ms = p["ms"] / max(p["launches"], 1)
    waves = blocks * 4
    insts = waves * iters * 8
    return {"kernel": "k_valu_probe (8 independent v_fma_f32 chains per thread, 8 waves per SIMD)",
            "ms": ms, "fma_wave_inst": insts,
            "inst_per_simd_per_clk": insts / (ms * 1e-3 * CLOCK_GHZ * 1e9 * N_SIMD),
            "tflops": insts * 64 * 2 / (ms * 1e-3) / 1e12}


def config2_bench(torch, R, synth, device, steps, warmup):
    """Pinhole workload at four resolutions: 100k clustered Gaussians with SH colour, the
    8 orbit views at 1920x1080, 1/2, 1/4 and 1/8 (calibration scaled with resolution),
    each resolution one batched call of its 8 views; rho^2 baked from the full-resolution
    views.  Per resolution: Mpix/s, the tile render's roofline fraction, and the
    frame-level roofline fraction."""
    scene_np, full = synth.pinhole_config()
    scene = R.Scene.from_numpy(scene_np, device=device)
    scene.rho2 = R.bake_rho2(scene, full, t_near=0.2)
    opts = R.RenderOpts(filter_mode=R.FILTER_ANISOTROPIC, use_floor=True)
    copts = R.RenderOpts(filter_mode=R.FILTER_ANISOTROPIC, use_floor=True, count_pairs=True)
    res = {"workload": "100k Gaussians, 8 orbit pinhole views, one batched call per resolution",
           "gaussians": scene.n, "resolutions": {}}
    for name, s in (("1", 1.0), ("1/2", 0.5), ("1/4", 0.25), ("1/8", 0.125)):
        cams = full if s == 1.0 else [synth.scale_camera(c, s) for c in full]
        npx = sum(R.view_pixels(cams))
        out = torch.empty((npx, 4), dtype=torch.float32, device=device)
        _, info, _ = R.render_forward(scene, cams, copts, out=out)
        for _ in range(warmup):
            R.render_forward(scene, cams, opts, out=out)
        prof = R.Profiler(stages=["render"])
        with prof:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                R.render_forward(scene, cams, opts, out=out)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
        rk = prof.read()["render"]
        render_ms = rk["ms"] / max(rk["launches"], 1)
        ms = dt / steps * 1e3
        frame_ms, _, _ = frame_roofline_ms(scene.n, len(cams), info["n_pairs"], npx, info["n_contrib"])
        achieved = info["n_contrib"] * FLOPS_PER_PAIR[True] / (render_ms * 1e-3) / 1e12
        res["resolutions"][name] = {
            "view": f"{cams[0]['crop'][2]}x{cams[0]['crop'][3]}", "value": npx * steps / dt / 1e6, "unit": "Mpix/s",
            "ms_per_step": ms, "pixels_per_step": npx, "pairs": info["n_pairs"], "contrib": info["n_contrib"],
            "render_ms": render_ms, "render_frac": achieved / PEAK_FP32_VECTOR_TFLOPS,
            "frame_frac": frame_ms / ms}
        print(f"bench: config 2 at {name}: {ms:.3f} ms/step, {npx * steps / dt / 1e6:.1f} Mpix/s",
              file=sys.stderr, flush=True)
    return res


def serving_bench(torch, R, synth, device, n_requests=200, levels=(0.25, 0.5, 0.75, 0.9)):
    """Three device-resident scenes (500k, 1.5M, 3M Gaussians); Poisson view requests
    with camera model uniform over {pinhole, KB fisheye, equirect} and scale uniform over
    1/8 .. x8 (x2..x8 as crops of the base size).  The per-view-launch baseline (one
    worker, one view per call) is driven by a burst to find its saturation rate; both
    it and the continuous-batching server (3 workers, up to 8 fused views) are then
    replayed at 25/50/75/90 % of that rate: p50/p99 latency (completion minus
    submission) and Mpix/s."""
    from paper_2609_13397_amd import serving

    scenes = []
    for n, seed in ((500_000, 51), (1_500_000, 52), (3_000_000, 53)):
        sc = R.Scene.from_numpy(synth.make_scene(n, seed=seed, layout="clusters", color="sh3",
                                                 log_scale_mean=-4.0, log_scale_std=0.7), device=device)
        sc.rho2 = R.bake_rho2(sc, synth.orbit_views(), 0.2)
        scenes.append(sc)
    torch.cuda.synchronize()
    trace = synth.serving_trace(n_requests, qps=1.0, seed=54)
    total_px = sum(r.pixels for r in trace)
    buf = torch.empty((total_px, 4), dtype=torch.float32, device=device)
    ptrs, off = [], 0
    for r in trace:
        ptrs.append(buf.data_ptr() + off * 16)
        off += r.pixels
    opts = R.RenderOpts(use_floor=True).to_c()

    def make(batched):
        cfg = serving.default_config(n_workers=3, max_batch_views=8) if batched else \
            serving.default_config(n_workers=1, max_batch_views=1)
        srv = serving.RenderServer(cfg)
        sids = [srv.add_scene(sc.to_c(), opts, keep=sc) for sc in scenes]
        return srv, sids

    # warm the caching pools of both configurations
    for batched in (False, True):
        srv, sids = make(batched)
        serving.replay(srv, sids, trace[:20], ptrs[:20], R.camera_struct, burst=True)
        srv.close()
    srv, sids = make(False)
    sat = serving.replay(srv, sids, trace, ptrs, R.camera_struct, burst=True)
    srv.close()
    sat_rps = len(trace) / sat.wall_s
    out = {"requests_per_level": n_requests, "baseline_saturation_rps": sat_rps,
           "baseline_saturation_mpix_per_s": sat.summary()["mpix_per_s"], "levels": []}
    for lv in levels:
        qps = lv * sat_rps
        row = {"load": lv, "qps": qps}
        for name, batched in (("per_view_launch", False), ("batched", True)):
            srv, sids = make(batched)
            res = serving.replay(srv, sids, trace, ptrs, R.camera_struct, time_scale=1.0 / qps)
            srv.close()
            row[name] = res.summary()
        out["levels"].append(row)
        print(f"bench: serving load {lv:.2f} qps {qps:.1f}: baseline p50 {row['per_view_launch']['p50_ms']:.2f} "
              f"p99 {row['per_view_launch']['p99_ms']:.2f} | batched p50 {row['batched']['p50_ms']:.2f} "
              f"p99 {row['batched']['p99_ms']:.2f} ms", file=sys.stderr, flush=True)
    # saturation of the batched server (burst)
    srv, sids = make(True)
    bsat = serving.replay(srv, sids, trace, ptrs, R.camera_struct, burst=True)
    srv.close()
    out["batched_saturation_rps"] = len(trace) / bsat.wall_s
    out["batched_saturation_mpix_per_s"] = bsat.summary()["mpix_per_s"]
    # a small view of the largest scene, whole forward call: the split tile render
    # against one workgroup per tile (cg_set_tile_split forcing the latter)
    small_cam = synth.scale_camera(synth.serving_base_cameras()[2], 0.125)
    ropts = R.RenderOpts(use_floor=True)
    small = {"workload": "3M-Gaussian serving scene, equirect 256x128 (1/8 scale)"}
    for name, thresholds in (("split", (0, 0, 0)), ("one_workgroup_per_tile", (1, 1 << 40, 0))):
        R.set_tile_split(*thresholds)
        try:
            for _ in range(2):
                R.render_forward(scenes[2], [small_cam], ropts)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(5):
                _, sinfo, _ = R.render_forward(scenes[2], [small_cam], ropts)
            torch.cuda.synchronize()
            small[name + "_ms"] = (time.perf_counter() - t0) / 5 * 1e3
            small[name + "_segments"] = sinfo["n_segments"]
        finally:
            R.set_tile_split(0, 0, 0)
    small["pairs"] = sinfo["n_pairs"]
    print(f"bench: small view of the 3M scene: split {small['split_ms']:.2f} ms, one workgroup per tile "
          f"{small['one_workgroup_per_tile_ms']:.2f} ms", file=sys.stderr, flush=True)
    out["small_view"] = small
    return out


def cpu_baseline(scene_np, bake_cams, cams, opts_kw, rows=16):
    """The FP64 oracle (culled mode) on a band of `rows` rows through the middle of each
    view, all host threads.  rho^2 is baked by the oracle (Eq. 11) from `bake_cams`, the
    views the GPU bake uses, before the timed region."""
    import numpy as np

    from oracle import oracle as O
    from paper_2609_13397_amd import synth

    sc = dict(scene_np)
    sc["rho2"] = O.bake_rho2(sc, bake_cams, 0.2).astype(np.float32)
    opts = O.Opts(**opts_kw)
    threads = os.cpu_count() or 1
    px = 0
    t0 = time.perf_counter()
    for c in cams:
        w, h = c["crop"][2], c["crop"][3]
        band = synth.with_crop(c, 0, h // 2 - rows // 2, w, rows)
        O.render(sc, band, opts, mode="culled", n_threads=threads)
        px += w * rows
    dt = time.perf_counter() - t0
    return {"value": px / dt / 1e6, "unit": "Mpix/s", "cores": threads, "kind": "oracle",
            "sample": f"{rows} middle rows of each view ({px} px), culled FP64 oracle incl. its per-call set-up",
            "seconds": dt}


def _counter_rows(path: str, counter: str):
    import csv
    with open(path) as f:
        return [r for r in csv.DictReader(f) if r["Counter_Name"] == counter]


def summarize_traffic(fetch_csv: str, write_csv: str, commands) -> dict:
    """profiles/render_traffic.json from two rocprofv3 --pmc runs (FETCH_SIZE, then
    WRITE_SIZE, both with --copy-calibration): per-dispatch KiB of the render kernel,
    each scaled by what the counter reads for the 256 MiB calibration copies."""
    fetch = _counter_rows(fetch_csv, "FETCH_SIZE")
    write = _counter_rows(write_csv, "WRITE_SIZE")

    def pick(rows, name):
        return [float(r["Counter_Value"]) for r in rows if name in r["Kernel_Name"]]

    def copies(rows):
        vals = sorted(((float(r["Counter_Value"]), r) for r in rows if "copyBuffer" in r["Kernel_Name"]),
                      key=lambda x: -x[0])
        return [v for v, _ in vals[:3]]

    copy_kib = 256 * 1024
    fc, wc = copies(fetch), copies(write)
    ff = copy_kib / (sum(fc) / len(fc))
    wf = copy_kib / (sum(wc) / len(wc))
    fr, wr = pick(fetch, TRAFFIC_KERNEL), pick(write, TRAFFIC_KERNEL)
    if not fr or not wr:
        raise SystemExit(f"no {TRAFFIC_KERNEL} dispatches in the counter files")
    per_launch = (sum(fr) / len(fr) * ff + sum(wr) / len(wr) * wf) * 1024
    out = {"render_source_hash": render_source_hash(), "kernel": TRAFFIC_KERNEL, "workload": "fisheye_1M",
           "fetch_kib_per_dispatch": fr, "write_kib_per_dispatch": wr,
           "copy_calibration": {"bytes_kib": copy_kib, "fetch_kib": sum(fc) / len(fc), "write_kib": sum(wc) / len(wc),
                                "fetch_factor": ff, "write_factor": wf},
           "bytes_per_launch": per_launch, "commands": list(commands)}
    with open(os.path.join(ROOT, "profiles", "render_traffic.json"), "w") as f:
        json.dump(out, f, indent=1)
    return out


def summarize_kernel_traffic(fetch_csv: str, write_csv: str, trace_csv: str, out_md: str, kernels, commands,
                             title: str, notes: str = "") -> None:
    """HBM bytes per dispatch of the given kernels from two rocprofv3 --pmc runs
    (FETCH_SIZE, then WRITE_SIZE, both with --copy-calibration), each scaled by what the
    counter reads for the 256 MiB calibration copies, over the average duration of the
    same kernel in a --kernel-trace run of the same command."""
    import csv
    fetch = _counter_rows(fetch_csv, "FETCH_SIZE")
    write = _counter_rows(write_csv, "WRITE_SIZE")

    def calib(rows):
        vals = sorted((float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]), reverse=True)[:3]
        return 256 * 1024 / (sum(vals) / len(vals))

    ff, wf = calib(fetch), calib(write)
    with open(trace_csv) as f:
        trace = list(csv.DictReader(f))
    lines = [f"# {title}", "", "Commands (run from the repository root on the GPU box):", "", "```", *commands, "```", "",
             f"Bytes = counter KiB x 1024 x calibration factor (FETCH_SIZE {ff:.4f}, WRITE_SIZE {wf:.4f}: 256 MiB "
             "device copies read as that much); ms = average duration of the kernel in the kernel trace; "
             "share = (fetch + write) / ms against MI355X's 8 TB/s.", ""]
    if notes:
        lines += [notes, ""]
    lines += ["| kernel | dispatches | fetch (MB) | write (MB) | avg ms | TB/s | share of 8 TB/s |",
              "|---|---:|---:|---:|---:|---:|---:|"]
    for k in kernels:
        fr = [float(r["Counter_Value"]) for r in fetch if k in r["Kernel_Name"]]
        wr = [float(r["Counter_Value"]) for r in write if k in r["Kernel_Name"]]
        ns = [int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in trace if k in r["Kernel_Name"]]
        if not fr or not wr or not ns:
            continue
        fb = sum(fr) / len(fr) * 1024 * ff
        wb = sum(wr) / len(wr) * 1024 * wf
        ms = sum(ns) / len(ns) / 1e6
        tbs = (fb + wb) / (ms * 1e-3) / 1e12
        lines.append(f"| `{k}` | {len(fr)} | {fb / 1e6:.1f} | {wb / 1e6:.1f} | {ms:.3f} | {tbs:.2f} | {tbs / 8.0:.1%} |")
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")


# Two rocprofv3 --pmc passes (at most 8 SQ counters each):
SQ_COUNTERS = ["SQ_INSTS_VALU", "SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_VALU2", "SQ_THREAD_CYCLES_VALU",
               "SQ_INSTS_VALU_TRANS_F32", "SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES", "SQ_WAVES"]
SQ_COUNTERS_2 = ["SQ_INSTS_LDS", "SQ_LDS_BANK_CONFLICT", "SQ_LDS_IDX_ACTIVE", "SQ_INSTS_SALU", "SQ_WAIT_INST_ANY",
                 "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR", "SQ_INST_LEVEL_LDS"]
N_SIMD = 256 * 4          # MI355X: 256 CUs x 4 SIMDs
CLOCK_GHZ = 2.4


def summarize_valu(sq_csv: str, trace_csv: str, out_md: str, commands, kernels, sq2_csv: str = None) -> None:
    """VALU and LDS utilisation of the given kernels from rocprofv3 --pmc runs of
    SQ_COUNTERS (and SQ_COUNTERS_2) and a --kernel-trace run of the same command
    (per-dispatch durations, kernel_trace.csv), grouped by kernel and grid size (one
    row per workload).  SQ_ACTIVE_INST_VALU counts quad-cycles in which a wave works on
    a VALU instruction, summed over the SIMDs: VALU busy = 4 x that / (SIMDs x cycles).
    SQ_ACTIVE_INST_VALU2 counts the quad-cycles in which two VALU instructions issue
    (gfx950 issues up to two per SIMD and cycle).  A kernel whose VALU is busy most of
    its cycles is issue-bound; one that is not is latency-bound."""
    import csv

    def load(path, names):
        with open(path) as f:
            rows = list(csv.DictReader(f))
        groups = {}
        for k in kernels:
            for r in rows:
                if k in r["Kernel_Name"] and r["Counter_Name"] in names:
                    groups.setdefault((k, int(r["Grid_Size"])), {}).setdefault(r["Counter_Name"], []).append(
                        float(r["Counter_Value"]))
        return groups

    g1 = load(sq_csv, SQ_COUNTERS)
    g2 = load(sq2_csv, SQ_COUNTERS_2) if sq2_csv else {}
    with open(trace_csv) as f:
        trace = list(csv.DictReader(f))
    lines = ["# VALU and LDS utilisation: " + ", ".join(kernels), "",
             "Commands (run from the repository root on the GPU box):", "", "```", *commands, "```", "",
             f"Per kernel and grid size (4657152 threads: fisheye_1M; 3686400: train_1M), averaged over its "
             f"dispatches; cycles = average duration in the kernel trace x {CLOCK_GHZ} GHz.", "",
             "* VALU inst rate = SQ_INSTS_VALU / (cycles x 1024 SIMDs): wave instructions per SIMD per clock.",
             "* VALU busy = 4 x SQ_ACTIVE_INST_VALU / (cycles x 1024 SIMDs): share of SIMD cycles with a VALU "
             "instruction in flight (SQ_ACTIVE_INST_VALU is in quad-cycles, summed over SIMDs).",
             "* dual issue = SQ_ACTIVE_INST_VALU2 / SQ_ACTIVE_INST_VALU: share of VALU quad-cycles in which two "
             "VALU instructions issue.",
             "* lane utilisation = SQ_THREAD_CYCLES_VALU / (64 x SQ_ACTIVE_INST_VALU) (the profiler's "
             "VALUUtilization).",
             "* trans = SQ_INSTS_VALU_TRANS_F32 / SQ_INSTS_VALU.",
             "* LDS bank conflict = SQ_LDS_BANK_CONFLICT / SQ_LDS_IDX_ACTIVE (stall cycles per active LDS cycle).",
             "",
             "| kernel | grid | dispatches | avg ms | waves | VALU inst | inst/SIMD/clk | VALU busy | dual issue | "
             "lane util | trans | LDS inst | LDS bank conflict |",
             "|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for (k, grid) in sorted(g1, key=lambda x: (kernels.index(x[0]), -x[1])):
        per = g1[(k, grid)]
        avg = {c: sum(v) / len(v) for c, v in per.items()}
        avg2 = {c: sum(v) / len(v) for c, v in g2.get((k, grid), {}).items()}
        ns = [int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in trace
              if k in r["Kernel_Name"] and int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"]) == grid]
        if not ns:
            raise SystemExit(f"no {k} with grid {grid} in {trace_csv}")
        t = sum(ns) / len(ns) * 1e-9
        cyc = t * CLOCK_GHZ * 1e9
        issue = avg["SQ_INSTS_VALU"] / (cyc * N_SIMD)
        busy = 4.0 * avg["SQ_ACTIVE_INST_VALU"] / (cyc * N_SIMD)
        dual = avg["SQ_ACTIVE_INST_VALU2"] / max(avg["SQ_ACTIVE_INST_VALU"], 1.0)
        lane = avg["SQ_THREAD_CYCLES_VALU"] / (64.0 * max(avg["SQ_ACTIVE_INST_VALU"], 1.0))
        trans = avg["SQ_INSTS_VALU_TRANS_F32"] / max(avg["SQ_INSTS_VALU"], 1.0)
        lds = avg2.get("SQ_INSTS_LDS")
        conf = (avg2["SQ_LDS_BANK_CONFLICT"] / max(avg2["SQ_LDS_IDX_ACTIVE"], 1.0)) if "SQ_LDS_BANK_CONFLICT" in avg2 \
            else None
        lines.append(f"| `{k}` | {grid} | {len(per['SQ_INSTS_VALU'])} | {t * 1e3:.3f} | {avg['SQ_WAVES']:.0f} | "
                     f"{avg['SQ_INSTS_VALU']:.3e} | {issue:.3f} | {busy:.2f} | {dual:.2f} | {lane:.2f} | {trans:.3f} | "
                     + (f"{lds:.3e}" if lds is not None else "-") + " | "
                     + (f"{conf:.3f}" if conf is not None else "-") + " |")
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")


def summarize_trace(stats_csv: str, out_md: str, title: str, commands, notes: str = ""):
    """Markdown table of a rocprofv3 --kernel-trace --stats kernel_stats.csv."""
    import csv
    with open(stats_csv) as f:
        rows = list(csv.DictReader(f))
    lines = [f"# {title}", "", "Command (run from the repository root on the GPU box):", "", "```", *commands, "```", ""]
    if notes:
        lines += [notes, ""]
    lines += ["| kernel | calls | avg (us) | total (ms) | % |", "|---|---:|---:|---:|---:|"]
    for r in rows[:20]:
        name = r["Name"].replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "")
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['Percentage']):.1f} |")
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=240)
    ap.add_argument("--no-train", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-order", action="store_true", help="skip the per-ray compositing order leg")
    ap.add_argument("--no-config2", action="store_true", help="skip the pinhole workload at four resolutions")
    ap.add_argument("--serving-requests", type=int, default=2000)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (reference for HBM byte counters)")
    # offline summaries of rocprofv3 output into profiles/ (no GPU needed)
    ap.add_argument("--summarize-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"))
    ap.add_argument("--summarize-trace", nargs=2, metavar=("KERNEL_STATS_CSV", "OUT_MD"))
    ap.add_argument("--summarize-valu", nargs=3, metavar=("SQ_COUNTER_CSV", "KERNEL_TRACE_CSV", "OUT_MD"))
    ap.add_argument("--summarize-kernel-traffic", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "KERNEL_TRACE_CSV", "OUT_MD"))
    ap.add_argument("--sq2", default=None, help="second SQ counter CSV (SQ_COUNTERS_2) for --summarize-valu")
    ap.add_argument("--kernel", action="append", default=[], help="kernel name (substring) for --summarize-valu")
    ap.add_argument("--title", default="")
    ap.add_argument("--notes", default="")
    ap.add_argument("--command", action="append", default=[], help="profiling command recorded in the summary")
    args = ap.parse_args()
    if args.summarize_traffic:
        t = summarize_traffic(*args.summarize_traffic, args.command)
        print(json.dumps({k: t[k] for k in ("kernel", "bytes_per_launch", "copy_calibration")}))
        return
    if args.summarize_trace:
        summarize_trace(*args.summarize_trace, args.title, args.command, args.notes)
        return
    if args.summarize_kernel_traffic:
        summarize_kernel_traffic(*args.summarize_kernel_traffic, args.kernel, args.command, args.title, args.notes)
        return
    if args.summarize_valu:
        summarize_valu(*args.summarize_valu, args.command, args.kernel, sq2_csv=args.sq2)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the path is not "
              "built for more than one GPU.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2609_13397_amd import render as R
    from paper_2609_13397_amd import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    device = torch.device("cuda:0")
    if args.copy_calibration:
        src = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device=device).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print("bench: copy calibration done (3 x 256 MiB device copies)", file=sys.stderr, flush=True)
    print("bench: building workload", file=sys.stderr, flush=True)
    scene_np, scene, cams = build_workload(torch, R, synth, device)
    use_floor = True
    opts = R.RenderOpts(filter_mode=R.FILTER_ANISOTROPIC, use_floor=use_floor)
    npx = sum(R.view_pixels(cams))
    out = torch.empty((npx, 4), dtype=torch.float32, device=device)

    # pair counts (counting variant of the render kernel, outside the timed region)
    copts = R.RenderOpts(filter_mode=R.FILTER_ANISOTROPIC, use_floor=use_floor, count_pairs=True)
    _, info, _ = R.render_forward(scene, cams, copts, out=out)
    torch.cuda.synchronize()
    print(f"bench: pairs={info['n_pairs']} evaluated={info['n_evaluated']} full={info['n_full']} "
          f"contrib={info['n_contrib']}", file=sys.stderr, flush=True)

    for _ in range(args.warmup):
        R.render_forward(scene, cams, opts, out=out)
    torch.cuda.synchronize()
    # timed region: HIP events bracket the render kernel only (each bracket costs an
    # event record on the stream); the per-stage breakdown comes from a separate pass
    prof = R.Profiler(stages=["render"])
    with prof:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            R.render_forward(scene, cams, opts, out=out)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    stages = prof.read()
    stage_prof = R.Profiler()
    stage_steps = min(args.steps, 5)
    with stage_prof:
        for _ in range(stage_steps):
            R.render_forward(scene, cams, opts, out=out)
        torch.cuda.synchronize()
    stage_ms = {k: v["ms"] / stage_steps for k, v in stage_prof.read().items() if v["launches"]}
    ms_per_step = dt / args.steps * 1e3
    value = npx * args.steps / dt / 1e6
    print(f"bench: {ms_per_step:.3f} ms/step, {value:.1f} Mpix/s", file=sys.stderr, flush=True)

    render = stages["render"]
    render_ms = render["ms"] / max(render["launches"], 1)
    flops = info["n_contrib"] * FLOPS_PER_PAIR[use_floor]
    achieved = flops / (render_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP32_VECTOR_TFLOPS, "traffic": None,
                "kernel": "k_render (tile render)", "kernel_ms": render_ms,
                "units_per_launch": info["n_contrib"], "unit_name": "contributing pair",
                "flops_per_unit": FLOPS_PER_PAIR[use_floor], "transcendentals_per_unit": TRANSC_PER_PAIR[use_floor],
                "evaluated_per_contributing": info["n_evaluated"] / max(info["n_contrib"], 1),
                "full_per_contributing": info["n_full"] / max(info["n_contrib"], 1)}
    alg_bytes = info["n_pairs"] * BYTES_PER_PAIR + npx * BYTES_PER_PIXEL
    roofline["algorithmic_bytes"] = alg_bytes
    roofline["achieved_GBps"] = alg_bytes / (render_ms * 1e-3) / 1e9
    roofline["design_bytes"] = info["n_pairs"] * DESIGN_BYTES_PER_PAIR + npx * DESIGN_BYTES_PER_PIXEL
    tr = load_traffic()
    if tr is not None:
        roofline["traffic"] = tr["bytes_per_launch"]
    frame_ms, _, frame_bytes = frame_roofline_ms(scene.n, len(cams), info["n_pairs"], npx, info["n_contrib"])
    frame_roofline = {"ms": frame_ms, "frac": frame_ms / ms_per_step, "algorithmic_bytes": frame_bytes}
    ceiling = valu_ceiling(torch, R, device)
    roofline["measured_fp32_ceiling_tflops"] = ceiling["tflops"]
    roofline["frac_of_measured_ceiling"] = achieved / ceiling["tflops"]
    print(f"bench: VALU ceiling {ceiling['tflops']:.1f} TFLOP/s ({ceiling['inst_per_simd_per_clk']:.3f} "
          f"inst/SIMD/clk)", file=sys.stderr, flush=True)

    config2 = None
    if not args.no_config2:
        print("bench: pinhole workload at four resolutions", file=sys.stderr, flush=True)
        config2 = config2_bench(torch, R, synth, device, max(3, args.steps // 2), max(1, args.warmup))

    order_ray = None
    if not args.no_order:
        print("bench: per-ray compositing order", file=sys.stderr, flush=True)
        R.render_forward(scene, cams, opts, out=out)
        order_ray = order_ray_bench(torch, R, scene, cams, out.clone(), max(3, args.steps // 4),
                                    max(1, args.warmup // 2))
        print(f"bench: per-ray order {order_ray['ms_per_step']:.3f} ms/step, overflow "
              f"{order_ray['n_order_overflow']}", file=sys.stderr, flush=True)

    fwd_bwd = None
    if not args.no_train:
        print("bench: training step (fwd + L1 + bwd)", file=sys.stderr, flush=True)
        fwd_bwd = train_step_bench(torch, R, synth, device, max(3, args.steps // 4), max(1, args.warmup // 2))
        print(f"bench: fwd+bwd {fwd_bwd['ms_per_step']:.3f} ms/step, {fwd_bwd['value']:.1f} Mpix/s",
              file=sys.stderr, flush=True)

    serving_res = None
    if not args.no_serving:
        print("bench: serving", file=sys.stderr, flush=True)
        serving_res = serving_bench(torch, R, synth, device, n_requests=args.serving_requests)

    cpu = None
    if not args.no_cpu_baseline:
        print("bench: cpu baseline (oracle)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(scene_np, synth.orbit_views(), cams,
                           dict(filter_mode=1, use_floor=1), rows=args.cpu_rows)

    line = {
        "metric": "Mpix/s fwd & fwd+bwd at 1M Gaussians; serving p50/p99 ms vs per-view launch",
        "value": value, "unit": "Mpix/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "fisheye_1M", "gaussians": scene.n,
                   "views": "KB fisheye 1600x1600 (190 deg) + equirect 2048x1024, one batched call",
                   "filter": "anisotropic footprint + floor (marginal composition)", "colour": "SH degree 3",
                   "pixels_per_step": npx, "pairs": info["n_pairs"]},
        "roofline": roofline,
        "frame_roofline": frame_roofline,
        "valu_ceiling": ceiling,
        "cpu_baseline": cpu,
        "fwd_bwd": fwd_bwd,
        "config2": config2,
        "order_ray": order_ray,
        "serving": serving_res,
        "stages_ms_per_step": stage_ms,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
