"""Continuous-batching server on the GPU: every request's images are bitwise
identical to rendering it alone, requests that can never fit are rejected,
and pair buffers grow when the estimate is short."""
import sys

import numpy as np
import pytest
import torch

import gut_synth as G
import oracle as O
from paper_2412_12507_amd import raster as R
from paper_2412_12507_amd.serve import Server, render_sequential
from paper_2412_12507_amd import _lib as L

from parity import compare_pixels

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def small_requests(n_req, seed, sizes=((160, 120), (320, 240), (200, 150))):
    rng = np.random.default_rng(seed)
    fish_k = G.config3_camera()["k"]
    reqs = []
    for _ in range(n_req):
        cams = []
        for _ in range(int(rng.integers(1, 5))):
            R_, t_ = G.look_at(G.random_eye(rng))
            if rng.random() < 0.5:
                w, h = sizes[int(rng.integers(0, len(sizes)))]
                cams.append(G.camera("pinhole", w, h, G.pinhole_focal(w), R0=R_, t0=t_))
            else:
                c = G.camera("fisheye", 200, 150, G.fisheye_focal(200), k=fish_k, R0=R_, t0=t_)
                cams.append(G.with_motion(c, 0.1, 0.3))
        reqs.append(cams)
    return reqs


def test_serve_mix_equals_alone():
    say("[serve mix vs alone]")
    scene = G.clustered_scene(40000, seed=1003)
    gs = R.GaussianScene.from_host(scene)
    reqs = small_requests(12, seed=3005)
    with Server(gs, mem_budget_bytes=2 << 30, max_slots=3, max_batch_cams=8) as srv:
        ids = [srv.submit(cams)[0] for cams in reqs]
        outs = {rid: srv.wait(rid) for rid in ids}
        st = srv.stats()
        say("  stats", st)
        assert st["completed"] == len(reqs) and st["batches"] >= 2
        assert st["batches"] < len(reqs), "requests were never merged into batches"
        assert st["p50_ms"] <= st["p99_ms"] and st["frames_per_s"] > 0
        for rid, cams in zip(ids, reqs):
            alone = render_sequential(gs, cams)
            for a, b in zip(outs[rid], alone):
                assert torch.equal(a, b)
    # one served camera against the oracle (sampled tiles)
    cam = reqs[0][0]
    p = O.default_params()
    pr, ob, res = O.render_full(scene, cam, p)
    img = outs[ids[0]][0].cpu().numpy().astype(np.float64)
    rgb_o = O.to_image(res, cam, p)
    amb = O.to_image(res, cam, p, key="n_alt") > 0
    assert np.abs(img - rgb_o)[~amb].max() <= 1e-4


def test_serve_full_size_mix_equals_alone():
    """The serving workload's own sizes: the 3M-particle scene and requests of
    the serving trace (pinhole 640x480 .. 3840x2160, rolling-shutter fisheye
    1600x1200, up to 8 cameras each), served together in merged batches; each
    image equals the request rendered alone, bit for bit."""
    say("[serve mix vs alone, full size]")
    scene = G.config3_scene()
    gs = R.GaussianScene.from_host(scene)
    reqs = G.config5_requests(5, seed=3007)
    say("  cameras", [[(c["model"], c["width"], c["height"]) for c in cams] for cams in reqs])
    with Server(gs, mem_budget_bytes=48 << 30, max_slots=4, max_batch_cams=8) as srv:
        ids = [srv.submit(cams)[0] for cams in reqs]
        outs = {rid: srv.wait(rid) for rid in ids}
        st = srv.stats()
        say("  stats", st)
        assert st["completed"] == len(reqs)
        for rid, cams in zip(ids, reqs):
            alone = render_sequential(gs, cams)
            for a, b in zip(outs[rid], alone):
                assert torch.equal(a, b)


def test_serve_admission_and_growth():
    say("[serve admission]")
    scene = G.clustered_scene(30000, seed=1003)
    gs = R.GaussianScene.from_host(scene)
    budget = 64 << 20
    with Server(gs, mem_budget_bytes=budget, max_slots=2, max_batch_cams=4) as srv:
        # 64 cameras x 30k particles: ~93 MB of per-entry buffers (48 B per entry),
        # above the 64 MB budget
        many = [G.camera("pinhole", 64, 48, 60.0, R0=np.eye(3), t0=np.array([0, 0, 8.0]))] * 64
        with pytest.raises(L.GutError) as ei:
            srv.submit(many)
        assert ei.value.status == L.GUT_E_ADMISSION
        # big particles close to the camera: far more pairs per entry than the initial estimate
        big = G.uniform_scene(3000, seed=7, log_scale_mean=-1.0)
        gb = R.GaussianScene.from_host(big)
    with Server(gb, mem_budget_bytes=512 << 20, max_slots=1, max_batch_cams=4) as srv:
        cam = G.camera("pinhole", 256, 256, 200.0, R0=np.eye(3), t0=np.array([0, 0, 3.0]))
        rid, out = srv.submit([cam])
        srv.wait(rid)
        alone = render_sequential(gb, [cam])
        assert torch.equal(out[0], alone[0])
        st = srv.stats()
        assert st["rejected"] == 0 and st["completed"] == 1


def test_serve_generalized_degree_equals_alone():
    """The server's batched kernels with a degree-4 response (Supp. A): each
    request bitwise equal to rendering it alone with the same parameters."""
    say("[serve degree 4 vs alone]")
    scene = G.clustered_scene(30000, seed=1003)
    gs = R.GaussianScene.from_host(scene)
    reqs = small_requests(6, seed=3006)
    params = dict(kernel_degree=4)
    with Server(gs, params, mem_budget_bytes=1 << 30, max_slots=2, max_batch_cams=8) as srv:
        ids = [srv.submit(cams)[0] for cams in reqs]
        outs = {rid: srv.wait(rid) for rid in ids}
        for rid, cams in zip(ids, reqs):
            alone = render_sequential(gs, cams, params)
            for a, b in zip(outs[rid], alone):
                assert torch.equal(a, b)
