"""Offline oracle check of cameras served by the continuous-batching server.

`bench.py --serve-protocol OUT.json` keeps, for one camera in 50 served at
load 0.9, a few random 16x16 tiles of its image together with the camera
(OUT_checks.pkl, written by that run).  This script renders those tiles with
the FP64 oracle on the CPU and compares every pixel: within 1e-4 of the
oracle's primary render or of one of its single-decision alternatives (the
parity rule of tests/parity.py).  Test infrastructure: run it by hand on the
file a GPU run wrote, e.g.

    python tests/serve_oracle_check.py gpurun_out/serve_protocol_checks.pkl
"""
from __future__ import annotations

import json
import os
import pickle
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import gut_synth as G  # noqa: E402
import oracle as O  # noqa: E402

TOL = 1e-4


def check(path, limit=None):
    with open(path, "rb") as fh:
        d = pickle.load(fh)  # written by bench.py in this repository
    scene = O.OScene.from_scene(G.config3_scene(d["n_particles"]))
    p = O.default_params()
    checks = d["checks"][:limit] if limit else d["checks"]
    n_px = n_fail = n_alt = 0
    worst = 0.0
    fails = []
    t0 = time.perf_counter()
    for i, c in enumerate(checks):
        cam = c["cam"]
        pr = O.project(scene, cam, p)
        ob = O.bin_tiles(pr, cam, p)
        tiles = np.asarray(c["tiles"], np.int32)
        res = O.render(scene, pr, cam, ob, p, tiles=tiles)
        tx, _ = O.tiles_xy(cam, p)
        H, W = int(cam["height"]), int(cam["width"])
        for slot, t in enumerate(tiles):
            img = np.asarray(c["pixels"][slot], np.float64)
            y0, x0 = (int(t) // tx) * 16, (int(t) % tx) * 16
            for ly in range(img.shape[0]):
                for lx in range(img.shape[1]):
                    if y0 + ly >= H or x0 + lx >= W:
                        continue
                    k = slot * 256 + ly * 16 + lx
                    g = img[ly, lx]
                    err = np.abs(g - res["rgb"][k]).max()
                    n_px += 1
                    if err <= TOL:
                        worst = max(worst, err)
                        continue
                    if any(np.abs(g - res["alt_rgb"][k, a]).max() <= TOL for a in range(int(res["n_alt"][k]))):
                        n_alt += 1
                        continue
                    n_fail += 1
                    if len(fails) < 10:
                        fails.append(dict(camera=i, tile=int(t), px=x0 + lx, py=y0 + ly, err=float(err)))
        print(f"camera {i + 1}/{len(checks)} ({cam['model']} {W}x{H}): {n_fail} failing pixels so far, "
              f"{time.perf_counter() - t0:.0f} s", flush=True)
    return dict(cameras=len(checks), pixels=n_px, failing=n_fail, alternatives_used=n_alt,
                worst_primary_abs=worst, tolerance=TOL, load=d["load"], every=d["every"], fails=fails)


if __name__ == "__main__":
    out = check(sys.argv[1], int(sys.argv[2]) if len(sys.argv) > 2 else None)
    print(json.dumps(out))
