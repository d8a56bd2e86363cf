"""Runs every entry point of the CPU oracle on small inputs, in a process that loads an
instrumented build of it (ASan + UBSan): started by test_sanitizers.py, which checks
that it ends cleanly.  argv[1]: path of the instrumented oracle library."""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

from oracle import build_oracle  # noqa: E402

build_oracle.LIB = sys.argv[1]  # load the instrumented build (newer than the source: no rebuild)

from oracle import oracle as O  # noqa: E402
from paper_2609_13397_amd import synth  # noqa: E402


def main():
    scene, cam = synth.tiny_config()
    scene = synth.subset_scene(scene, np.arange(64))
    cam = synth.scale_camera(cam, 0.5)
    sh = synth.make_scene(48, seed=5, layout="uniform", color="sh3", log_scale_mean=-2.5, log_scale_std=0.5)
    fish = synth.kb_camera(40, 40, 100.0, synth.draw_kb_coeffs(3, np.radians(100.0))[0], 16.0, np.eye(3),
                           (0.0, 0.0, -3.0))
    equi = synth.camera(synth.EQUIRECT, 48, 24, origin=(0.0, 0.0, -3.0))
    crop = synth.with_crop(cam, 3, 2, 17, 11)
    rho = O.bake_rho2(scene, [cam, fish], 0.2, n_threads=2)
    floored = dict(scene, rho2=rho.astype(np.float32))
    for sc in (scene, floored, sh):
        for c in (cam, fish, equi, crop):
            for f in (0, 1, 2):
                for floor in (0, 1):
                    for comp in (0, 1):
                        o = O.Opts(filter_mode=f, use_floor=floor, composition=comp)
                        O.render(sc, c, o, with_alt=True, n_threads=2)
            for om in (0, 1):
                for bb in (0, 1):
                    O.render(sc, c, O.Opts(order_mode=om, backbone=bb, use_floor=1), n_threads=2)
            O.render(sc, c, O.Opts(), mode="tiles", n_threads=2)
    empty = synth.subset_scene(scene, np.arange(0))
    O.render(empty, cam, O.Opts())
    O.render(scene, synth.with_crop(cam, 0, 0, 0, 0), O.Opts())
    O.render_supersampled(floored, cam, synth.mc_jitter(4, 1), O.Opts(use_floor=1), n_threads=2)
    gr = synth.seeded_image((cam["crop"][3], cam["crop"][2], 4), 9)
    for f in (0, 1, 2):
        O.grad(floored, [cam], [gr], O.Opts(filter_mode=f, use_floor=1), n_threads=2)
        O.grad(sh, [cam, fish], [gr, synth.seeded_image((40, 40, 4), 10)], O.Opts(filter_mode=f), n_threads=2)
    px = np.array([0.5, 3.25, 11.0]), np.array([0.5, 2.0, 7.75])
    for c in (cam, fish, equi):
        d, v = O.unproject(c, *px)
        O.project(c, d)
        O.pixel_rays(c)
    rays, _ = O.pixel_rays(cam)
    O.pair_batch(scene, 3, cam["origin"], rays.reshape(-1, rays.shape[-1])[:16], O.Opts())
    O.preprocess(sh, cam["origin"], O.Opts())
    O.sh_basis(np.array([0.0, 0.6, 0.8]))
    print("oracle entry points ran clean", flush=True)


if __name__ == "__main__":
    main()
