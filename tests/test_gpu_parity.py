"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances (derived from FP32 arithmetic, see the design notes):
  pixels and T_final     1e-4 absolute, matching the oracle's render or one of
                         its single-decision alternatives; n_contrib and
                         n_eval exactly equal to the matched render's
  projection             depth 4e-6 relative, colour 1e-5, UT mean 2e-3 px,
                         UT covariance 1e-2 relative to its largest variance;
                         rectangles and culling exact except within 2e-3 px
                         of a tile edge / 1e-5 of a validity boundary
  tile lists             exact membership of decided entries, (depth, id)
                         order up to 1e-6 relative depth ties
  gradients              1e-3 of the largest oracle gradient per tensor, and
                         element-wise 1e-3 relative above 1e-3 of that max
"""
import sys

import numpy as np
import pytest
import torch

import gut_synth as G
import oracle as O
from paper_2412_12507_amd import raster as R

from parity import (compare_bins, compare_pixels, compare_projection, gpu_forward,
                    grad_compare, image_np, to_torch_scene)

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def small_c2(kind, n=20000, w=320, h=180):
    scene = G.clustered_scene(n, seed=1002)
    pin, fish = G.config2_cameras(w, h)
    return scene, (pin if kind == "pinhole" else fish)


def small_c3(n=30000, w=400, h=300):
    return G.clustered_scene(n, seed=1003), G.config3_camera(w, h)


CASES = {
    "c1": lambda: (G.config1()[0], G.config1()[1][0]),
    "c2-pinhole": lambda: small_c2("pinhole"),
    "c2-fisheye": lambda: small_c2("fisheye"),
    "c3-rolling": lambda: small_c3(),
    "ragged-37x23": lambda: (G.config1(n=300)[0],
                             G.camera("pinhole", 37, 23, 40.0, R0=np.eye(3), t0=np.array([0, 0, 3.0]))),
}


@pytest.mark.parametrize("case", list(CASES))
def test_forward_parity(case):
    say(f"[forward parity] case={case}")
    scene, cam = CASES[case]()
    p = O.default_params()
    gs, proj, bins, img = gpu_forward(scene, [cam])
    pr = O.project(scene, cam, p)
    rep = compare_projection(proj, pr, 0, scene.n)
    say("  projection", rep)
    assert rep["cull_mismatch_unexplained"] == 0
    assert rep["rect_mismatch_unexplained"] == 0
    assert rep["tiles_mismatch_unexplained"] == 0
    assert rep["depth_rel_err"] <= 4e-6
    assert rep["rgb_abs_err"] <= 1e-5
    assert rep["mean_abs_err_px"] <= 2e-3
    assert rep["cov_rel_err"] <= 1e-2
    ob = O.bin_tiles(pr, cam, p)
    tx, ty = O.tiles_xy(cam, p)
    bad = compare_bins(bins, ob, pr, 0, scene.n, 0, tx * ty)
    say("  bins: pairs", bins.n_pairs, "bad tiles", bad[:5])
    assert not bad
    res = O.render(scene, pr, cam, ob, p)
    rep = compare_pixels(image_np(img), res, cam, p)
    say("  pixels", {k: v for k, v in rep.items() if k != "fails"}, rep["fails"][:3])
    assert rep["n_fail"] == 0


@pytest.mark.parametrize("which", ["c2-pinhole", "c2-fisheye", "c3-rolling"])
def test_full_size_sampled(which):
    """The full workloads (1M / 3M particles, 1920x1080 / 1600x1200) in the
    launch configuration the benchmark times, checked on every particle's
    projection and on sampled tiles: the longest lists plus random ones."""
    say(f"[full size] {which}")
    if which == "c3-rolling":
        scene, cam = G.config3_scene(), G.config3_camera()
    else:
        scene = G.config2_scene()
        cam = G.config2_cameras()[0 if which == "c2-pinhole" else 1]
    p = O.default_params()
    gs, proj, bins, img = gpu_forward(scene, [cam])
    pr = O.project(scene, cam, p)
    rep = compare_projection(proj, pr, 0, scene.n)
    say("  projection", rep)
    assert rep["cull_mismatch_unexplained"] == 0 and rep["rect_mismatch_unexplained"] == 0
    assert rep["depth_rel_err"] <= 4e-6 and rep["rgb_abs_err"] <= 1e-5
    ob = O.bin_tiles(pr, cam, p)
    tx, ty = O.tiles_xy(cam, p)
    lens = np.diff(ob[0])
    rng = np.random.default_rng(7)
    tiles = np.unique(np.concatenate([np.argsort(lens)[-6:], rng.choice(tx * ty, 18, replace=False)]))
    ranges = bins.ranges.cpu().numpy().astype(np.int64)
    assert int(np.diff(ranges, axis=1).sum()) == bins.n_pairs
    res = O.render(scene, pr, cam, ob, p, tiles=tiles.astype(np.int32))
    rep = compare_pixels(image_np(img), res, cam, p)
    say("  pixels", {k: v for k, v in rep.items() if k != "fails"}, rep["fails"][:3])
    assert rep["n_fail"] == 0


def test_full_size_timed_launch():
    """The benchmark's exact step: the 1M-particle scene, both 1920x1080 views
    in one gut_render call, Gaussian response, no n_eval (the
    render_multi_kernel<false, false, false, false> instance the benchmark
    times).  Every particle's projection in both views, every tile list, and
    sampled tiles of both views (the longest lists plus random ones) against
    the oracle; n_eval comes from a second call with n_eval on, whose colour,
    T and n_contrib must equal the timed call's bit for bit.  The share of
    checked pixels that match only one of the oracle's single-decision
    alternatives is reported and bounded."""
    say("[full size, timed launch] 1M particles, pinhole + fisheye 1920x1080 in one call")
    scene = G.config2_scene()
    cams = G.config2_cameras()
    p = O.default_params()
    gs = to_torch_scene(scene)
    proj = R.project(gs, cams, p, debug=True)
    bins = R.bin_tiles(proj, cams, p)
    img = R.render(proj, bins, cams, p, with_eval=False)
    img_e = R.render(proj, bins, cams, p, with_eval=True)
    torch.cuda.synchronize()
    assert img.n_eval is None
    for key in ("rgb", "T", "n_contrib"):
        assert torch.equal(getattr(img, key), getattr(img_e, key)), key
    n = scene.n
    tile_base = 0
    checked = alt = 0
    for ci, cam in enumerate(cams):
        pr = O.project(scene, cam, p)
        rep = compare_projection(proj, pr, ci, n)
        say(f"  view {ci} projection", rep)
        assert rep["cull_mismatch_unexplained"] == 0 and rep["rect_mismatch_unexplained"] == 0
        assert rep["tiles_mismatch_unexplained"] == 0
        assert rep["depth_rel_err"] <= 4e-6 and rep["rgb_abs_err"] <= 1e-5
        assert rep["mean_abs_err_px"] <= 2e-3 and rep["cov_rel_err"] <= 1e-2
        ob = O.bin_tiles(pr, cam, p)
        tx, ty = O.tiles_xy(cam, p)
        bad = compare_bins(bins, ob, pr, ci, n, tile_base, tx * ty)
        say(f"  view {ci} bins: bad tiles", bad[:5])
        assert not bad
        lens = np.diff(ob[0])
        rng = np.random.default_rng(11 + ci)
        tiles = np.unique(np.concatenate([np.argsort(lens)[-6:], rng.choice(tx * ty, 18, replace=False)]))
        res = O.render(scene, pr, cam, ob, p, tiles=tiles.astype(np.int32))
        rep = compare_pixels(image_np(img_e, ci), res, cam, p)
        say(f"  view {ci} pixels", {k: v for k, v in rep.items() if k != "fails"}, rep["fails"][:3])
        assert rep["n_fail"] == 0
        checked += rep["n_checked"]
        alt += rep["n_alt_used"]
        tile_base += tx * ty
    say(f"  alternatives used on {alt} of {checked} checked pixels ({100.0 * alt / checked:.3f}%)")
    assert alt <= 0.01 * checked


@pytest.mark.parametrize("which", ["c2-pinhole", "c2-fisheye", "c3-rolling"])
def test_full_size_backward_sampled(which):
    """Backward parity on the full workloads in the benchmark's launch
    configuration: the loss weights are random on sampled tiles (the longest
    lists plus random ones) and zero elsewhere, so the oracle's backward only
    has those pixels to differentiate; every particle's gradient is compared."""
    say(f"[full size backward] {which}")
    if which == "c3-rolling":
        scene, cam = G.config3_scene(), G.config3_camera()
    else:
        scene = G.config2_scene()
        cam = G.config2_cameras()[0 if which == "c2-pinhole" else 1]
    p = O.default_params()
    gs, proj, bins, img = gpu_forward(scene, [cam])
    pr = O.project(scene, cam, p)
    ob = O.bin_tiles(pr, cam, p)
    tx, ty = O.tiles_xy(cam, p)
    ts = p["tile"]
    lens = np.diff(ob[0])
    rng = np.random.default_rng(17)
    tiles = np.unique(np.concatenate([np.argsort(lens)[-4:], rng.choice(tx * ty, 12, replace=False)]))
    res = O.render(scene, pr, cam, ob, p, tiles=tiles.astype(np.int32))
    H, W = cam["height"], cam["width"]
    wC = np.zeros((H, W, 3))
    n_amb = 0
    for slot, t in enumerate(tiles):
        y0, x0 = (int(t) // tx) * ts, (int(t) % tx) * ts
        for ly in range(ts):
            for lx in range(ts):
                py, px = y0 + ly, x0 + lx
                if py >= H or px >= W:
                    continue
                if res["n_alt"][slot * ts * ts + ly * ts + lx] > 0:
                    n_amb += 1  # a flipped decision changes which particles get gradient
                    continue
                wC[py, px] = rng.normal(size=3)
    say("  sampled tiles", len(tiles), "ambiguous pixels zeroed", n_amb)
    g_ora = O.backward(scene, pr, cam, ob, wC, None, p)
    d_rgb = torch.as_tensor(wC.reshape(-1, 3), dtype=torch.float32, device="cuda")
    g = R.render_backward(gs, proj, bins, [cam], img, d_rgb, None, p)
    torch.cuda.synchronize()
    rep = grad_compare(g, g_ora)
    say("  grads", {k: (v["rel"], v["elem_fail"]) for k, v in rep.items()})
    for k, v in rep.items():
        assert v["rel"] <= 1e-3, (k, v)
        assert v["elem_fail"] == 0, (k, v)


def test_forward_deterministic_and_zero_motion():
    say("[determinism]")
    scene, cam = small_c3()
    _, _, _, a = gpu_forward(scene, [cam])
    _, _, _, b = gpu_forward(scene, [cam])
    assert torch.equal(a.rgb, b.rgb) and torch.equal(a.n_contrib, b.n_contrib)
    still = G.with_motion(dict(cam, shutter="global"), 0.0, 0.0)
    glob = dict(still, shutter="global")
    _, pa, _, ia = gpu_forward(scene, [still])
    _, pb, _, ib = gpu_forward(scene, [glob])
    assert torch.equal(pa.rect, pb.rect) and torch.equal(pa.depth, pb.depth)
    assert torch.equal(ia.rgb, ib.rgb) and torch.equal(ia.T, ib.T)


def test_multi_camera_call_equals_single_calls():
    say("[multi camera]")
    scene = G.clustered_scene(20000, seed=1002)
    cams = G.config2_cameras(320, 180) + [G.config3_camera(200, 150)]
    _, _, _, multi = gpu_forward(scene, cams)
    for c, cam in enumerate(cams):
        _, _, _, one = gpu_forward(scene, [cam])
        assert torch.equal(multi.images("rgb")[c], one.images("rgb")[0])
        assert torch.equal(multi.images("n_contrib")[c], one.images("n_contrib")[0])


def test_render_order_is_longest_first():
    """gut_bin's render order: per camera a permutation of its tiles whose
    list lengths have non-increasing bit length."""
    say("[render order]")
    scene = G.clustered_scene(20000, seed=1002)
    cams = G.config2_cameras(320, 180) + [G.config3_camera(200, 150)]
    _, _, bins, _ = gpu_forward(scene, cams)
    rng = bins.ranges.cpu().numpy().astype(np.int64)
    order = bins.order.cpu().numpy().astype(np.int64)
    base = 0
    for cam in cams:
        tx, ty = O.tiles_xy(cam, O.default_params())
        o = order[base:base + tx * ty]
        assert np.array_equal(np.sort(o), np.arange(tx * ty))
        lens = rng[base + o, 1] - rng[base + o, 0]
        bits = np.array([int(v).bit_length() for v in lens])
        assert (np.diff(bits) <= 0).all()
        base += tx * ty


def test_edge_cases():
    say("[edge cases]")
    p = O.default_params()
    # empty scene
    sc = G.uniform_scene(0, seed=1)
    cam = G.camera("pinhole", 40, 30, 40.0, R0=np.eye(3), t0=np.array([0, 0, 3.0]))
    _, _, bins, img = gpu_forward(sc, [cam])
    assert bins.n_pairs == 0
    assert torch.all(img.T == 1) and torch.all(img.rgb == 0)
    # everything culled (opacity below alpha_min)
    sc = G.uniform_scene(500, seed=2)
    sc.opacities[:] = 1e-3
    _, proj, bins, img = gpu_forward(sc, [cam])
    assert bins.n_pairs == 0 and int(proj.tiles.sum()) == 0 and torch.all(img.T == 1)
    # a 1x1 camera and a single particle
    sc = G.uniform_scene(1, seed=3)
    sc.means[:] = 0.0
    sc.scales[:] = 0.3
    sc.opacities[:] = 0.8
    one = G.camera("pinhole", 1, 1, 2.0, R0=np.eye(3), t0=np.array([0, 0, 3.0]))
    _, _, _, img = gpu_forward(sc, [one])
    pr, ob, res = O.render_full(sc, one, p)
    rep = compare_pixels(image_np(img), res, one, p)
    assert rep["n_fail"] == 0 and rep["n_checked"] == 1
    # pair-capacity error path: too-small buffer reports the size, retry succeeds
    scene, cam2 = small_c2("pinhole", n=5000, w=160, h=90)
    gs = to_torch_scene(scene)
    proj = R.project(gs, [cam2])
    import ctypes as C
    from paper_2412_12507_amd import _lib as L
    lib = L.load()
    arr, ps = L.camera_array([cam2]), L.params_struct()
    ranges = torch.empty(3 * R.num_tiles([cam2]), dtype=torch.int32, device="cuda")
    ids = torch.empty(1, dtype=torch.int32, device="cuda")
    need = lib.gut_bin_workspace_bytes(gs.n, arr, 1, 1)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    npairs = C.c_int64(0)
    pj = proj.struct()
    st = lib.gut_bin(L.ref(pj), gs.n, arr, 1, L.ref(ps), C.c_void_p(ws.data_ptr()), need, 1,
                     C.c_void_p(ranges.data_ptr()), C.c_void_p(ids.data_ptr()), C.byref(npairs),
                     C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == L.GUT_E_CAPACITY and npairs.value > 1
    bins_small = R.bin_tiles(proj, [cam2], capacity=1)   # grows and retries internally
    bins_ok = R.bin_tiles(proj, [cam2])
    assert bins_small.n_pairs == bins_ok.n_pairs > 0
    assert torch.equal(bins_small.ids[: bins_ok.n_pairs], bins_ok.ids[: bins_ok.n_pairs])


def _zero_ambiguous(res, cam, p, wC, wT):
    amb = O.to_image(res, cam, p, key="n_alt") > 0
    wC = wC.copy()
    wT = wT.copy()
    wC[amb] = 0
    wT[amb] = 0
    return wC, wT, int(amb.sum())


@pytest.mark.parametrize("case", ["pinhole", "fisheye", "rolling", "dense-pinhole",
                                  "dense-rolling", "c2-fisheye"])
def test_backward_parity(case):
    say(f"[backward parity] {case}")
    p = O.default_params(bg=(0.1, 0.3, 0.6))
    if case.startswith("dense"):
        scene, cam = G.config4_gradcheck(case.split("-")[1], log_scale_mean=-2.2)
    elif case == "c2-fisheye":
        scene, cam = small_c2("fisheye", n=20000, w=240, h=136)
    else:
        scene, cam = G.config4_gradcheck(case)
    pr = O.project(scene, cam, p)
    ob = O.bin_tiles(pr, cam, p)
    res = O.render(scene, pr, cam, ob, p)
    rng = np.random.default_rng(11)
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


def test_autograd_function_matches_direct_call():
    say("[autograd]")
    scene, cam = G.config4_gradcheck("fisheye", log_scale_mean=-2.2)
    gs = to_torch_scene(scene)
    leaves = [t.clone().requires_grad_(True) for t in (gs.means, gs.scales, gs.quats, gs.opacities, gs.sh)]
    imgs, Ts = R.render_gaussians(*leaves, gs.sh_degree, [cam])
    w = torch.randn_like(imgs[0])
    loss = (imgs[0] * w).sum() + Ts[0].sum()
    loss.backward()
    proj, bins, img = R.forward(gs, [cam])
    g = R.render_backward(gs, proj, bins, [cam], img, w.reshape(-1, 3), torch.ones_like(img.T))
    # per-particle sums are FP64 atomics: their order varies from run to run,
    # which can move a result by one FP32 ulp at most
    def close(a, b):
        return torch.allclose(a, b, rtol=1e-6, atol=1e-9 * float(b.abs().max()) + 1e-12)
    for leaf, k in zip(leaves, ("means", "scales", "quats", "opacities", "sh")):
        assert close(leaf.grad, g[k]), k
    # recompute_projection gives the same gradients
    leaves2 = [t.clone().requires_grad_(True) for t in (gs.means, gs.scales, gs.quats, gs.opacities, gs.sh)]
    imgs2, Ts2 = R.render_gaussians(*leaves2, gs.sh_degree, [cam], recompute_projection=True)
    ((imgs2[0] * w).sum() + Ts2[0].sum()).backward()
    for a, b in zip(leaves, leaves2):
        assert close(a.grad, b.grad)
    # the returned images are saved for the backward: editing one in place
    # must be caught by autograd's version check, not change the gradients
    leaves3 = [t.clone().requires_grad_(True) for t in (gs.means, gs.scales, gs.quats, gs.opacities, gs.sh)]
    imgs3, Ts3 = R.render_gaussians(*leaves3, gs.sh_degree, [cam])
    loss3 = (imgs3[0] * w).sum()
    with torch.no_grad():
        imgs3[0].clamp_(0.0, 0.5)
    with pytest.raises(RuntimeError):
        loss3.backward()
