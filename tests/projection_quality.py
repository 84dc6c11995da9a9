"""Gaussian projection quality (Supp. C): how well a projected 2D Gaussian
matches the distribution of the particle's points pushed through the camera.

For each visible particle, 500 points are drawn from N(mu, Sigma) (Eq. 2) and
projected exactly, each as a sigma point is (rolling-shutter time solved per
point); their sample mean and covariance are the Monte-Carlo reference P.
An approximation Q -- the UT projection (Eq. 9-10) of the HIP path or of the
oracle, or the EWA linearisation (Eq. 3) at one exposure time -- is scored by
KL(P || Q) between the two 2D Gaussians.  Lower is better; with 500 samples
even an exact Q scores about chi2_5 / 1000 (the reference's own sampling
error: 5 fitted parameters), median 4.35e-3.

Test infrastructure: uses the oracle for the reference projections.  Run as a
script for the camera sweeps (pinhole, equidistant fisheye over its field of
view, OpenCV fisheye with k2 distortion, rolling-shutter translations):

    python tests/projection_quality.py [--gpu]
"""
from __future__ import annotations

import math
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

import gut_synth as G  # noqa: E402
import oracle as O  # noqa: E402

N_SAMPLES = 500


def kl_gauss2(mp, cp, mq, cq):
    """KL(N(mp, cp) || N(mq, cq)) for 2D Gaussians (arrays [..., 2], [..., 2, 2])."""
    iq = np.linalg.inv(cq)
    d = mq - mp
    tr = np.einsum("...ij,...ji->...", iq, cp)
    quad = np.einsum("...i,...ij,...j->...", d, iq, d)
    return 0.5 * (tr + quad - 2.0 + np.log(np.linalg.det(cq) / np.linalg.det(cp)))


def mc_reference(scene, idx, cam, n_samples=N_SAMPLES, seed=0, params=None):
    """Monte-Carlo moments of particles idx: (ok[k], mean[k,2], cov[k,2,2])."""
    rng = np.random.default_rng(seed)
    k = len(idx)
    mu = scene.means[idx]
    R = np.stack([O.quat_to_rot(q / np.linalg.norm(q)) for q in scene.quats[idx]])
    L = R * scene.scales[idx][:, None, :]          # R diag(s): Sigma = L L^T
    z = rng.normal(size=(k, n_samples, 3))
    x = mu[:, None, :] + np.einsum("kij,ksj->ksi", L, z)
    v, ok = O.project_samples(cam, x.reshape(-1, 3), params=params)
    v = v.reshape(k, n_samples, 2)
    ok = ok.reshape(k, n_samples).all(1)
    mean = v.mean(1)
    dv = v - mean[:, None, :]
    cov = np.einsum("ksi,ksj->kij", dv, dv) / (n_samples - 1)
    return ok, mean, cov


def ewa_moments(scene, idx, cam, t=0.0, params=None):
    """EWA (Eq. 3) at one exposure time t (no rolling-shutter awareness)."""
    out_ok, out_m, out_c = [], [], []
    for i in idx:
        s = scene.scales[i]
        ok, m, c = O.ewa(cam, scene.means[i], scene.quats[i], s, t=t, h=1e-6 * max(1.0, float(np.abs(scene.means[i]).max())), params=params)
        out_ok.append(ok)
        out_m.append(m)
        out_c.append(c)
    return np.array(out_ok), np.array(out_m), np.array(out_c)


def ut_oracle(scene, cam, params=None):
    """The oracle's UT projection (Eq. 9-10) of every particle: (visible, mean, cov)."""
    pr = O.project(scene, cam, params)
    c = pr["cov2d"]
    cov = np.stack([np.stack([c[:, 0], c[:, 1]], -1), np.stack([c[:, 1], c[:, 2]], -1)], -2)
    return pr["cull"] == 0, pr["mean2d"], cov


def ut_gpu(scene, cam, params=None):
    """The HIP path's UT projection (gut_project's mean2d / cov2d outputs)."""
    import torch
    from paper_2412_12507_amd import raster as R
    gs = R.GaussianScene.from_host(scene)
    pr = R.project(gs, [cam], params, debug=True)
    torch.cuda.synchronize()
    m = pr.mean2d.double().cpu().numpy().reshape(-1, 2)
    c = pr.cov2d.double().cpu().numpy().reshape(-1, 3)
    cov = np.stack([np.stack([c[:, 0], c[:, 1]], -1), np.stack([c[:, 1], c[:, 2]], -1)], -2)
    return pr.tiles.cpu().numpy() > 0, m, cov


def evaluate(scene, cam, n_max=400, seed=0, gpu=False, ewa_t=0.0):
    """Median and 90th-percentile KL of UT and EWA against the MC reference
    over up to n_max visible particles (the same particles for both)."""
    vis, um, uc = (ut_gpu if gpu else ut_oracle)(scene, cam)
    idx = np.nonzero(vis)[0]
    rng = np.random.default_rng(seed)
    if idx.size > n_max:
        idx = np.sort(rng.choice(idx, n_max, replace=False))
    ok_mc, mm, mc = mc_reference(scene, idx, cam, seed=seed + 1)
    ok_e, em, ec = ewa_moments(scene, idx, cam, t=ewa_t)
    good = ok_mc & ok_e & (np.linalg.det(mc) > 0) & (np.linalg.det(ec) > 0) & (np.linalg.det(uc[idx]) > 0)
    kl_ut = kl_gauss2(mm[good], mc[good], um[idx][good], uc[idx][good])
    kl_ewa = kl_gauss2(mm[good], mc[good], em[good], ec[good])
    # the other direction, KL(Q || P_MC) (the paper does not say which it uses)
    kl_ut_r = kl_gauss2(um[idx][good], uc[idx][good], mm[good], mc[good])
    kl_ewa_r = kl_gauss2(em[good], ec[good], mm[good], mc[good])
    return dict(n=int(good.sum()), ut_median=float(np.median(kl_ut)), ut_p90=float(np.percentile(kl_ut, 90)),
                ewa_median=float(np.median(kl_ewa)), ewa_p90=float(np.percentile(kl_ewa, 90)),
                ut_median_rev=float(np.median(kl_ut_r)), ewa_median_rev=float(np.median(kl_ewa_r)))


def cone_scene(half_angle_deg, n=1500, seed=1007, dist=1.5, log_scale_mean=-2.7):
    """Particles at distance ~dist from the origin along directions whose angle
    to +z lies in [0.5, 1] x half_angle (the outer part of a field of view,
    where a wide lens bends most), sizes log-normal around e^-2.7 = 0.067."""
    rng = np.random.default_rng(seed)
    th = np.radians(half_angle_deg) * rng.uniform(0.5, 1.0, n)
    ph = rng.uniform(0, 2 * np.pi, n)
    r = dist * rng.uniform(0.9, 1.1, n)
    means = np.stack([r * np.sin(th) * np.cos(ph), r * np.sin(th) * np.sin(ph), r * np.cos(th)], -1)
    log_s = rng.normal(log_scale_mean, 0.3, size=(n, 3))
    q = rng.normal(size=(n, 4))
    logit = rng.normal(0.0, 1.0, size=n)
    sh = np.full((n, 1, 3), 0.5 / G.SH_C0)
    return G.scene_from_raw(means, log_s, q / np.linalg.norm(q, axis=1, keepdims=True), logit, sh, 0)


def sweep(w=800, h=800):
    """(name, scene, camera) triples: a camera at the origin looking along +z."""
    out = []
    eye = dict(R0=np.eye(3), t0=np.zeros(3))
    out.append(("pinhole, 60 deg FOV", cone_scene(30),
                G.camera("pinhole", w, h, G.pinhole_focal(w, 60.0), **eye)))
    for fov in (60, 120, 180, 220):
        out.append((f"equidistant fisheye, {fov} deg FOV", cone_scene(fov / 2),
                    G.camera("fisheye", w, h, G.fisheye_focal(w, fov), **eye)))
    for k2 in (0.0, 0.5):
        out.append((f"OpenCV fisheye 180 deg, k2 = {k2}", cone_scene(90),
                    G.camera("fisheye", w, h, G.fisheye_focal(w, 180), k=(0, k2, 0, 0), **eye)))
    base = G.camera("fisheye", w, h, G.fisheye_focal(w, 180), **eye)
    for shift in (0.0, 0.35):
        out.append((f"rolling-shutter fisheye 180 deg, shift {shift}", cone_scene(90),
                    G.with_motion(base, 0.0, shift)))
    return out


def noise_floor_median(n_samples=N_SAMPLES):
    from scipy.stats import chi2
    return chi2.median(5) / (2 * n_samples)


def main():
    gpu = "--gpu" in sys.argv
    print(f"UT from {'the HIP path (gut_project)' if gpu else 'the oracle'}; EWA at exposure time 0")
    print(f"MC noise floor (median KL of an exact projection): {noise_floor_median():.2e}")
    print(f"{'camera':42s} {'n':>5s} {'UT median':>10s} {'UT p90':>9s} {'EWA median':>11s} {'EWA p90':>9s}"
          f" {'UT med Q||P':>12s} {'EWA med Q||P':>13s}")
    for name, scene, cam in sweep():
        r = evaluate(scene, cam, gpu=gpu)
        print(f"{name:42s} {r['n']:5d} {r['ut_median']:10.2e} {r['ut_p90']:9.2e} {r['ewa_median']:11.2e} "
              f"{r['ewa_p90']:9.2e} {r['ut_median_rev']:12.2e} {r['ewa_median_rev']:13.2e}", flush=True)


if __name__ == "__main__":
    main()
