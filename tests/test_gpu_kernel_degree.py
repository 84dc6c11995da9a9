"""Generalized Gaussian responses of degree n (Supp. A) on the HIP path
against the FP64 oracle: projection extents, tile lists, pixels and
gradients, under pinhole, fisheye and rolling-shutter cameras, to the same
bars as the Gaussian (pixels 1e-4, gradients 1e-3 relative per tensor and
per element, tile lists exact)."""
import sys

import numpy as np
import pytest
import torch

import gut_synth as G
import oracle as O
from paper_2412_12507_amd import raster as R
from parity import (compare_bins, compare_pixels, compare_projection, gpu_forward, grad_compare,
                    image_np)

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


CASES = {
    "c1": lambda: (G.config1()[0], G.config1()[1][0]),
    "c2-fisheye": lambda: (G.clustered_scene(20000, seed=1002), G.config2_cameras(320, 180)[1]),
    "c3-rolling": lambda: (G.clustered_scene(30000, seed=1003), G.config3_camera(400, 300)),
}


@pytest.mark.parametrize("case,n", [("c1", 4), ("c2-fisheye", 3), ("c2-fisheye", 8),
                                    ("c3-rolling", 4), ("c3-rolling", 5)])
def test_forward_parity_degree(case, n):
    say(f"[degree {n} forward parity] case={case}")
    scene, cam = CASES[case]()
    p = O.default_params(kernel_degree=n)
    gs, proj, bins, img = gpu_forward(scene, [cam], p)
    pr = O.project(scene, cam, p)
    rep = compare_projection(proj, pr, 0, scene.n)
    say("  projection", rep)
    assert rep["cull_mismatch_unexplained"] == 0
    assert rep["rect_mismatch_unexplained"] == 0
    assert rep["tiles_mismatch_unexplained"] == 0
    ob = O.bin_tiles(pr, cam, p)
    tx, ty = O.tiles_xy(cam, p)
    bad = compare_bins(bins, ob, pr, 0, scene.n, 0, tx * ty)
    say("  bins: pairs", bins.n_pairs, "bad tiles", bad[:5])
    assert not bad
    res = O.render(scene, pr, cam, ob, p)
    rep = compare_pixels(image_np(img), res, cam, p)
    say("  pixels", {k: v for k, v in rep.items() if k != "fails"}, rep["fails"][:3])
    assert rep["n_fail"] == 0


def test_degree_two_is_the_gaussian_path():
    """kernel_degree = 2 given explicitly takes the Gaussian kernels: same
    bits as the defaults."""
    scene, cam = CASES["c2-fisheye"]()
    _, _, _, a = gpu_forward(scene, [cam], None)
    _, _, _, b = gpu_forward(scene, [cam], O.default_params(kernel_degree=2))
    assert torch.equal(a.rgb, b.rgb) and torch.equal(a.T, b.T)


def test_degree_changes_the_image():
    """A degree-4 render differs from the Gaussian one (the option is live)."""
    scene, cam = CASES["c1"]()
    _, _, _, a = gpu_forward(scene, [cam], O.default_params(kernel_degree=2))
    _, _, _, b = gpu_forward(scene, [cam], O.default_params(kernel_degree=4))
    assert (a.rgb - b.rgb).abs().max().item() > 1e-2


def _zero_ambiguous(res, cam, p, wC, wT):
    amb = O.to_image(res, cam, p, key="n_alt") > 0
    wC, wT = wC.copy(), wT.copy()
    wC[amb] = 0
    wT[amb] = 0
    return wC, wT, int(amb.sum())


@pytest.mark.parametrize("kind,n", [("pinhole", 4), ("fisheye", 3), ("rolling", 8)])
def test_backward_parity_degree(kind, n):
    say(f"[degree {n} backward parity] {kind}")
    p = O.default_params(bg=(0.1, 0.3, 0.6), kernel_degree=n)
    scene, cam = G.config4_gradcheck(kind, log_scale_mean=-2.2)
    pr = O.project(scene, cam, p)
    ob = O.bin_tiles(pr, cam, p)
    res = O.render(scene, pr, cam, ob, p)
    rng = np.random.default_rng(12)
    H, W = cam["height"], cam["width"]
    wC, wT, n_amb = _zero_ambiguous(res, cam, p, rng.normal(size=(H, W, 3)), rng.normal(size=(H, W)))
    say("  ambiguous pixels zeroed:", n_amb)
    g_ora = O.backward(scene, pr, cam, ob, wC, wT, p)
    gs, proj, bins, img = gpu_forward(scene, [cam], p)
    d_rgb = torch.as_tensor(wC.reshape(-1, 3), dtype=torch.float32, device="cuda")
    d_T = torch.as_tensor(wT.reshape(-1), dtype=torch.float32, device="cuda")
    g = R.render_backward(gs, proj, bins, [cam], img, d_rgb, d_T, p)
    torch.cuda.synchronize()
    rep = grad_compare(g, g_ora)
    say("  grads", rep)
    for k, v in rep.items():
        assert v["rel"] <= 1e-3, (k, v)
        assert v["elem_fail"] == 0, (k, v)


def test_full_size_two_view_batch_degree4_sampled():
    """The benchmark's degree-4 step at full size: 1M particles, pinhole +
    fisheye 1920x1080 in one call (one merged render launch); every
    particle's projection and sampled tiles of both views (the longest lists
    plus random ones) against the oracle."""
    say("[degree 4 full size] two-view batch")
    scene, cams = G.config2_scene(), G.config2_cameras()
    p = O.default_params(kernel_degree=4)
    gs, proj, bins, img = gpu_forward(scene, cams, p)
    for c, cam in enumerate(cams):
        pr = O.project(scene, cam, p)
        rep = compare_projection(proj, pr, c, scene.n, params=p)
        say("  projection", c, rep)
        assert rep["cull_mismatch_unexplained"] == 0 and rep["rect_mismatch_unexplained"] == 0
        ob = O.bin_tiles(pr, cam, p)
        tx, ty = O.tiles_xy(cam, p)
        lens = np.diff(ob[0])
        rng = np.random.default_rng(70 + c)
        tiles = np.unique(np.concatenate([np.argsort(lens)[-5:], rng.choice(tx * ty, 12, replace=False)]))
        res = O.render(scene, pr, cam, ob, p, tiles=tiles.astype(np.int32))
        rep = compare_pixels(image_np(img, c), res, cam, p)
        say("  pixels", c, {k: v for k, v in rep.items() if k != "fails"}, rep["fails"][:3])
        assert rep["n_fail"] == 0


def test_full_size_backward_degree4_sampled():
    """Degree-4 backward at full size (1M particles, fisheye 1920x1080) on
    sampled tiles: every particle's gradient against the oracle."""
    from parity import sampled_backward_check
    say("[degree 4 full size backward] fisheye")
    rep = sampled_backward_check(G.config2_scene(), G.config2_cameras()[1],
                                 O.default_params(kernel_degree=4), seed=27)
    say("  grads", {k: (v["rel"], v["elem_fail"]) for k, v in rep.items()})
    for k, v in rep.items():
        assert v["rel"] <= 1e-3 and v["elem_fail"] == 0, (k, v)
