"""Hybrid-rendering depth clip (Sec. 6.2) on the HIP path against the FP64
oracle: hits whose maximum-response point lies beyond a pixel's clip
distance are discarded, in the forward (every pixel, 1e-4) and the backward
(gradients 1e-3), under pinhole, fisheye and rolling-shutter cameras."""
import sys

import numpy as np
import pytest
import torch

import gut_synth as G
import oracle as O
from paper_2412_12507_amd import raster as R
from parity import compare_pixels, gpu_forward, grad_compare, image_np

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def clip_map(cam, lo, hi, seed, inf_frac=0.1):
    """Per-pixel clip distances U[lo, hi], a fraction of them +inf."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(lo, hi, size=(cam["height"], cam["width"]))
    c[rng.random(c.shape) < inf_frac] = np.inf
    return c


CASES = {
    "c1": lambda: (G.config1()[0], G.config1()[1][0], 2.6, 3.4),
    "c2-fisheye": lambda: (G.clustered_scene(20000, seed=1002), G.config2_cameras(320, 180)[1], 5.0, 11.0),
    "c3-rolling": lambda: (G.clustered_scene(30000, seed=1003), G.config3_camera(400, 300), 5.0, 11.0),
}


@pytest.mark.parametrize("case", list(CASES))
def test_forward_parity_with_clip(case):
    say(f"[depth clip forward] {case}")
    scene, cam, lo, hi = CASES[case]()
    clip = clip_map(cam, lo, hi, seed=4001)
    p = O.default_params()
    gs = R.GaussianScene.from_host(scene)
    proj = R.project(gs, [cam], p)
    bins = R.bin_tiles(proj, [cam], p)
    ct = torch.as_tensor(clip.reshape(-1), dtype=torch.float32, device="cuda")
    img = R.render(proj, bins, [cam], p, with_eval=True, clip=ct)
    full = R.render(proj, bins, [cam], p)
    torch.cuda.synchronize()
    pr = O.project(scene, cam, p)
    ob = O.bin_tiles(pr, cam, p)
    # the oracle clips at the FP32 values the GPU reads
    res = O.render(scene, pr, cam, ob, p, clip=clip.astype(np.float32).astype(np.float64))
    rep = compare_pixels(image_np(img), res, cam, p)
    say("  pixels", {k: v for k, v in rep.items() if k != "fails"}, rep["fails"][:3])
    assert rep["n_fail"] == 0
    changed = (img.rgb - full.rgb).abs().amax(1).gt(1e-3).float().mean().item()
    say("  fraction of pixels the clip changes:", changed)
    assert changed > 0.05


def test_clip_at_infinity_is_bitwise_no_clip():
    scene, cam, _, _ = CASES["c2-fisheye"]()
    gs, proj, bins, a = gpu_forward(scene, [cam], None, with_eval=False)
    ct = torch.full((cam["height"] * cam["width"],), float("inf"), device="cuda")
    b = R.render(proj, bins, [cam], None, clip=ct)
    torch.cuda.synchronize()
    assert torch.equal(a.rgb, b.rgb) and torch.equal(a.T, b.T) and torch.equal(a.n_contrib, b.n_contrib)


@pytest.mark.parametrize("kind", ["pinhole", "fisheye", "rolling"])
def test_backward_parity_with_clip(kind):
    say(f"[depth clip backward] {kind}")
    p = O.default_params(bg=(0.1, 0.3, 0.6))
    scene, cam = G.config4_gradcheck(kind, log_scale_mean=-2.2)
    clip = clip_map(cam, 2.6, 3.4, seed=4002).astype(np.float32).astype(np.float64)
    pr = O.project(scene, cam, p)
    ob = O.bin_tiles(pr, cam, p)
    res = O.render(scene, pr, cam, ob, p, clip=clip)
    rng = np.random.default_rng(13)
    H, W = cam["height"], cam["width"]
    amb = O.to_image(res, cam, p, key="n_alt") > 0
    wC, wT = rng.normal(size=(H, W, 3)), rng.normal(size=(H, W))
    wC[amb] = 0
    wT[amb] = 0
    say("  ambiguous pixels zeroed:", int(amb.sum()))
    g_ora = O.backward(scene, pr, cam, ob, wC, wT, p, clip=clip)
    gs = R.GaussianScene.from_host(scene)
    proj = R.project(gs, [cam], p)
    bins = R.bin_tiles(proj, [cam], p)
    ct = torch.as_tensor(clip.reshape(-1), dtype=torch.float32, device="cuda")
    img = R.render(proj, bins, [cam], p, clip=ct)
    d_rgb = torch.as_tensor(wC.reshape(-1, 3), dtype=torch.float32, device="cuda")
    d_T = torch.as_tensor(wT.reshape(-1), dtype=torch.float32, device="cuda")
    g = R.render_backward(gs, proj, bins, [cam], img, d_rgb, d_T, p, clip=ct)
    torch.cuda.synchronize()
    rep = grad_compare(g, g_ora)
    say("  grads", rep)
    for k, v in rep.items():
        assert v["rel"] <= 1e-3, (k, v)
        assert v["elem_fail"] == 0, (k, v)


def test_multi_camera_clip_equals_single_calls():
    """A two-camera call (one merged launch) reads each camera's clip values
    at its own pixel offset: equal to clipping each camera alone."""
    scene = G.clustered_scene(20000, seed=1002)
    pin = G.config2_cameras(320, 180)[0]
    R2, t2 = G.look_at((1.5, 0.8, -7.5))
    cams = [pin, dict(pin, R0=R2, t0=t2, R1=R2, t1=t2)]  # two pinholes of one size: one launch
    clips = [clip_map(c, 5.0, 11.0, seed=4010 + i) for i, c in enumerate(cams)]
    gs = R.GaussianScene.from_host(scene)
    proj = R.project(gs, cams)
    bins = R.bin_tiles(proj, cams)
    ct = torch.as_tensor(np.concatenate([c.reshape(-1) for c in clips]), dtype=torch.float32,
                         device="cuda")
    both = R.render(proj, bins, cams, clip=ct)
    torch.cuda.synchronize()
    off = 0
    for cam, c in zip(cams, clips):
        _, pj1, b1, _ = gpu_forward(scene, [cam], None, with_eval=False)
        one = R.render(pj1, b1, [cam], clip=torch.as_tensor(c.reshape(-1), dtype=torch.float32,
                                                            device="cuda"))
        torch.cuda.synchronize()
        npx = cam["width"] * cam["height"]
        assert torch.equal(both.rgb[off:off + npx], one.rgb)
        assert torch.equal(both.T[off:off + npx], one.T)
        off += npx


def test_full_size_two_view_batch_clip_sampled():
    """The benchmark's depth-clip step at full size: 1M particles, pinhole +
    fisheye 1920x1080 in one call, the same per-pixel clip map (U[6, 10] from
    the same generator); sampled tiles of both views against the oracle."""
    say("[depth clip full size] two-view batch")
    scene, cams = G.config2_scene(), G.config2_cameras()
    p = O.default_params()
    gs = R.GaussianScene.from_host(scene)
    proj = R.project(gs, cams, p)
    bins = R.bin_tiles(proj, cams, p)
    npx = sum(c["width"] * c["height"] for c in cams)
    g = torch.Generator(device="cuda").manual_seed(4003)
    clip = 6.0 + 4.0 * torch.rand(npx, device="cuda", generator=g)
    img = R.render(proj, bins, cams, p, with_eval=True, clip=clip)
    torch.cuda.synchronize()
    clip_h = clip.cpu().numpy().astype(np.float64)
    off = 0
    for c, cam in enumerate(cams):
        n1 = cam["width"] * cam["height"]
        cm = clip_h[off:off + n1].reshape(cam["height"], cam["width"])
        off += n1
        pr = O.project(scene, cam, p)
        ob = O.bin_tiles(pr, cam, p)
        tx, ty = O.tiles_xy(cam, p)
        lens = np.diff(ob[0])
        rng = np.random.default_rng(90 + c)
        tiles = np.unique(np.concatenate([np.argsort(lens)[-5:], rng.choice(tx * ty, 12, replace=False)]))
        res = O.render(scene, pr, cam, ob, p, tiles=tiles.astype(np.int32), clip=cm)
        rep = compare_pixels(image_np(img, c), res, cam, p)
        say("  pixels", c, {k: v for k, v in rep.items() if k != "fails"}, rep["fails"][:3])
        assert rep["n_fail"] == 0


def test_autograd_with_clip_and_degree_matches_direct_calls():
    """render_gaussians with a clip map and a degree-4 response: the images
    and the gradients torch computes equal the direct gut_render /
    gut_render_bwd calls with the same clip and parameters."""
    scene, cam = G.config4_gradcheck("rolling", log_scale_mean=-2.2)
    p = O.default_params(kernel_degree=4)
    clip = torch.as_tensor(clip_map(cam, 2.6, 3.4, seed=4020).reshape(-1), dtype=torch.float32,
                           device="cuda")
    gs = R.GaussianScene.from_host(scene)
    leaves = [t.clone().requires_grad_(True) for t in (gs.means, gs.scales, gs.quats, gs.opacities, gs.sh)]
    imgs, Ts = R.render_gaussians(*leaves, gs.sh_degree, [cam], p, clip=clip)
    w = torch.randn_like(imgs[0])
    ((imgs[0] * w).sum() + Ts[0].sum()).backward()
    proj, bins, img = R.forward(gs, [cam], p, clip=clip)
    assert torch.equal(imgs[0].reshape(-1, 3), img.rgb)
    g = R.render_backward(gs, proj, bins, [cam], img, w.reshape(-1, 3), torch.ones_like(img.T), p,
                          clip=clip)
    torch.cuda.synchronize()
    for leaf, k in zip(leaves, ("means", "scales", "quats", "opacities", "sh")):
        assert torch.allclose(leaf.grad, g[k], rtol=1e-6, atol=1e-9 * float(g[k].abs().max()) + 1e-12), k


def test_full_size_backward_clip_sampled():
    """Clipped backward at full size (1M particles, fisheye 1920x1080, clip
    U[6, 10]) on sampled tiles: every particle's gradient against the oracle."""
    from parity import sampled_backward_check
    say("[depth clip full size backward] fisheye")
    cam = G.config2_cameras()[1]
    rep = sampled_backward_check(G.config2_scene(), cam, O.default_params(),
                                 clip=clip_map(cam, 6.0, 10.0, seed=4030, inf_frac=0.0), seed=37)
    say("  grads", {k: (v["rel"], v["elem_fail"]) for k, v in rep.items()})
    for k, v in rep.items():
        assert v["rel"] <= 1e-3 and v["elem_fail"] == 0, (k, v)
