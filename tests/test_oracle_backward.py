"""Pins of the oracle's backward pass (Supp. B).

1. The closed form the paper derives for d alpha / d mu (Supp. B) against the
   oracle's chain, on single-contributor pixels.
2. Central finite differences (h = 1e-6) of a linear image loss with every
   discrete decision frozen (tile lists, skip masks, stop index, clamps)
   against the oracle's analytic gradient, for all 59 parameters of 64
   particles, under pinhole, fisheye and rolling-shutter cameras, with the
   Gaussian response and with generalized responses of degree 3, 4 and 8.
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import gut_synth as G
import oracle as O


def test_dalpha_dmu_closed_form():
    """d alpha/d mu = (-1/2 sigma e^{-w^2/2}) (2 o_g + 2 tau_g d_g/|d_g|)^T (-S^-1 R^T)
    with tau_g = -o_g . d_g/|d_g| (Supp. B), on pixels a lone particle covers."""
    cam = G.camera("pinhole", 32, 32, 40.0, R0=np.eye(3), t0=np.array([0.0, 0.0, 3.0]))
    mu = np.array([0.05, -0.08, 0.1])
    q = np.array([0.8, 0.3, -0.2, 0.4])
    s = np.array([0.12, 0.07, 0.2])
    sig = 0.8
    sh = np.full((1, 1, 3), 0.5 / G.SH_C0)  # white, degree 0: no view dependence
    sc = O.OScene(mu[None], s[None], q[None], np.array([sig]), sh, 0)
    p = O.default_params()
    pr = O.project(sc, cam, p)
    bins = O.bin_tiles(pr, cam, p)
    R = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
    M = np.diag(1 / s) @ R.T
    o = np.array([0, 0, -3.0])
    checked = 0
    for py in range(4, 28, 3):
        for px in range(4, 28, 3):
            d = np.array([(px + 0.5 - 16) / 40, (py + 0.5 - 16) / 40, 1.0])
            og, dg = M @ (o - mu), M @ d
            dgh = dg / np.linalg.norm(dg)
            tau_g = -og @ dgh
            om2 = np.linalg.norm(og + tau_g * dgh) ** 2
            a = sig * math.exp(-0.5 * om2)
            if not (1 / 255 + 1e-4 < a < 0.99):
                continue
            expect = (-0.5 * sig * math.exp(-0.5 * om2)) * (2 * og + 2 * tau_g * dgh) @ (-M)
            dC = np.zeros((32, 32, 3))
            dC[py, px, 0] = 1.0
            g = O.backward(sc, pr, cam, bins, dC, None, p)
            np.testing.assert_allclose(g["means"][0], expect, rtol=1e-10, atol=1e-12)
            checked += 1
    assert checked >= 10


def _fd_check(scene, cam, seed, h=1e-6, bg=(0.0, 0.0, 0.0), use_dT=True, kernel_degree=2, clip=None,
              kbuffer=0):
    p = O.default_params(bg=bg, kernel_degree=kernel_degree, kbuffer=kbuffer)
    sc = O.as_oscene(scene)
    pr = O.project(sc, cam, p)
    bins = O.bin_tiles(pr, cam, p)
    rec = O.record(sc, pr, cam, bins, p, clip=clip)
    rng = np.random.default_rng(seed)
    H, W = cam["height"], cam["width"]
    wC = rng.normal(size=(H, W, 3))
    wT = rng.normal(size=(H, W)) if use_dT else None
    g = O.backward(sc, pr, cam, bins, wC, wT, p, clip=clip)
    assert len(rec[1]) > 50  # the check must exercise compositing
    L0 = O.loss_frozen(sc, pr, cam, rec, wC, wT, p)
    # the analytic render must agree with the frozen loss at theta_0
    res = O.render(sc, pr, cam, bins, p, alternatives=False, clip=clip)
    img, T = O.to_image(res, cam), O.to_image(res, cam, key="T")
    L_render = (wC * img).sum() + ((wT * T).sum() if use_dT else 0.0)
    assert abs(L_render - L0) < 1e-10 * max(1, abs(L0))
    worst = {}
    for name in ("means", "scales", "quats", "opacities", "sh"):
        arr = getattr(sc, name)
        fd = np.zeros_like(arr)
        flat = arr.reshape(-1)
        fdf = fd.reshape(-1)
        for j in range(flat.size):
            v = flat[j]
            flat[j] = v + h
            lp = O.loss_frozen(sc, pr, cam, rec, wC, wT, p)
            flat[j] = v - h
            lm = O.loss_frozen(sc, pr, cam, rec, wC, wT, p)
            flat[j] = v
            fdf[j] = (lp - lm) / (2 * h)
        an = g[name].reshape(fd.shape)
        scale = np.abs(fd).max()
        assert scale > 0, name
        worst[name] = np.abs(an - fd).max() / scale
    return worst


@pytest.mark.parametrize("kind", ["pinhole", "fisheye", "rolling"])
def test_backward_matches_central_differences(kind):
    scene, cam = G.config4_gradcheck(kind)
    worst = _fd_check(scene, cam, seed=3004)
    for k, v in worst.items():
        assert v < 1e-6, (kind, k, v)


@pytest.mark.parametrize("kind", ["pinhole", "rolling"])
def test_backward_central_differences_dense_overlap(kind):
    """Larger particles (log-scale mean -2.2): many contributors per pixel,
    early termination and alpha clamps all occur."""
    scene, cam = G.config4_gradcheck(kind, log_scale_mean=-2.2)
    worst = _fd_check(scene, cam, seed=3014, bg=(0.2, 0.5, 0.9))
    for k, v in worst.items():
        assert v < 1e-6, (kind, k, v)


@pytest.mark.parametrize("kind,n", [("pinhole", 4), ("fisheye", 3), ("rolling", 8)])
def test_backward_central_differences_generalized_kernel(kind, n):
    """The degree-n response of Supp. A: its chain d rho / d omega^2 against
    central differences, with dense overlap so clamps and stops occur."""
    scene, cam = G.config4_gradcheck(kind, log_scale_mean=-2.2)
    worst = _fd_check(scene, cam, seed=3024 + n, bg=(0.1, 0.3, 0.6), kernel_degree=n)
    for k, v in worst.items():
        assert v < 1e-6, (kind, n, k, v)


@pytest.mark.parametrize("kind", ["pinhole", "rolling"])
def test_backward_central_differences_with_depth_clip(kind):
    """A per-pixel clip distance (Sec. 6.2's hybrid rendering) inside the
    particles' depth range: the clipped contributors get their gradients, the
    clipped-away ones none, consistently with the frozen clipped loss."""
    scene, cam = G.config4_gradcheck(kind, log_scale_mean=-2.2)
    rng = np.random.default_rng(3030)
    clip = rng.uniform(2.6, 3.4, size=(cam["height"], cam["width"]))
    worst = _fd_check(scene, cam, seed=3031, bg=(0.1, 0.3, 0.6), clip=clip)
    for k, v in worst.items():
        assert v < 1e-6, (kind, k, v)


@pytest.mark.parametrize("kind,k", [("pinhole", 16), ("fisheye", 2), ("rolling", 4)])
def test_backward_central_differences_kbuffer(kind, k):
    """The k-buffer ("Ours (sorted)", Sec. 4.3): the contributors in blend
    order (a second implementation of the buffer, which must reproduce the
    render), their gradients against central differences of the frozen loss."""
    scene, cam = G.config4_gradcheck(kind, log_scale_mean=-2.2)
    worst = _fd_check(scene, cam, seed=3040 + k, bg=(0.1, 0.3, 0.6), kbuffer=k)
    for key, v in worst.items():
        assert v < 1e-6, (kind, k, key, v)
