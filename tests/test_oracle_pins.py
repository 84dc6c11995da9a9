"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these retypes the oracle's own formula: each compares the oracle with
a closed form, a library routine (scipy), a brute-force search, or an
identity the method must satisfy, chosen so that a dropped term, a wrong sign
or index, or a transposed operand in the oracle fails at least one of them.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.spatial.transform import Rotation, Slerp

import gut_synth as G
import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def rot_scipy(q_wxyz):
    q = np.asarray(q_wxyz, np.float64)
    return Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()


# ---------------------------------------------------------------------------
# Unscented transform (Eq. 6-10)
# ---------------------------------------------------------------------------

def test_ut_weights_golden():
    """Eq. 7-8 at alpha=1, beta=2, kappa=0 (Sec. 4.4) give fixed constants."""
    g = json.load(open(os.path.join(GOLD, "ut_weights.json")))
    lam, wm, wc = O.ut_weights(g["alpha"], g["beta"], g["kappa"])
    assert lam == g["lambda"]
    np.testing.assert_allclose(wm, g["w_mu"], rtol=0, atol=1e-15)
    np.testing.assert_allclose(wc, g["w_sigma"], rtol=0, atol=1e-15)


@pytest.mark.parametrize("a,b,k", [(0.5, 2.0, 0.0), (1.0, 0.0, 1.0), (1e-3, 2.0, 0.0)])
def test_ut_weights_identities(a, b, k):
    """For any spread the mean weights sum to one, and the covariance weights
    differ from them only at the centre point, by 1 - alpha^2 + beta."""
    lam, wm, wc = O.ut_weights(a, b, k)
    assert abs(lam - (a * a * (3 + k) - 3)) < 1e-12
    assert abs(wm.sum() - 1.0) < 1e-9
    np.testing.assert_allclose(wc[1:], wm[1:], rtol=0, atol=0)
    assert abs((wc[0] - wm[0]) - (1 - a * a + b)) < 1e-9


@pytest.mark.parametrize("seed", range(6))
def test_ut_exact_for_affine_maps(seed):
    """The UT reproduces (A mu + b, A Sigma A^T) exactly for affine g, with
    Sigma = R S S^T R^T (Eq. 2) and R from scipy's quaternion convention."""
    rng = np.random.default_rng(seed)
    mu = rng.normal(size=3)
    q = rng.normal(size=4)
    s = np.exp(rng.normal(-1, 0.5, size=3))
    A = rng.normal(size=(2, 3))
    b = rng.normal(size=2)
    R = rot_scipy(q / np.linalg.norm(q))
    Sigma = R @ np.diag(s ** 2) @ R.T
    m, cov = O.ut_affine(mu, q, s, A, b)
    np.testing.assert_allclose(m, A @ mu + b, rtol=0, atol=1e-12)
    np.testing.assert_allclose(cov, A @ Sigma @ A.T, rtol=1e-12, atol=1e-12)


def test_ut_affine_general_spread():
    """Exactness for affine maps holds for any (alpha, beta, kappa) with
    alpha^2 (3 + kappa) > 0 whenever beta = 0 adds no extra centre weight...
    here beta = 1 - alpha^2 keeps the covariance weights summing to one."""
    rng = np.random.default_rng(7)
    mu, q, s = rng.normal(size=3), rng.normal(size=4), np.array([0.2, 0.5, 0.1])
    A, b = rng.normal(size=(2, 3)), rng.normal(size=2)
    R = rot_scipy(q / np.linalg.norm(q))
    for a, k in [(0.7, 0.0), (1.3, 1.0)]:
        p = O.default_params(ut_alpha=a, ut_beta=1 - a * a, ut_kappa=k)
        m, cov = O.ut_affine(mu, q, s, A, b, p)
        np.testing.assert_allclose(m, A @ mu + b, atol=1e-12)
        np.testing.assert_allclose(cov, A @ R @ np.diag(s ** 2) @ R.T @ A.T, atol=1e-12)


@pytest.mark.parametrize("z,s,f", [(3.0, 0.1, 150.0), (8.0, 0.02, 1662.77), (1.5, 0.3, 37.5)])
def test_ut_on_axis_pinhole_closed_form(z, s, f):
    """An isotropic particle on the optical axis, its frame rotated only about
    that axis, projects to the principal point with covariance (f s / z)^2 I
    exactly (the two z-axis sigma points land on the centre; the other four at
    distance sqrt(3) f s / z with weight 1/6)."""
    cam = G.camera("pinhole", 200, 100, f, cx=100.0, cy=50.0)
    ang = 0.7
    q = np.array([[math.cos(ang / 2), 0.0, 0.0, math.sin(ang / 2)]])
    sc = O.OScene(np.array([[0.0, 0.0, z]]), np.full((1, 3), s), q, np.array([0.9]),
                  np.zeros((1, 1, 3)), 0)
    pr = O.project(sc, cam)
    np.testing.assert_allclose(pr["mean2d"][0], [100.0, 50.0], atol=1e-9)
    e = (f * s / z) ** 2
    np.testing.assert_allclose(pr["cov2d"][0], [e, 0.0, e], rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("a,b,k", [(1.0, 2.0, 0.0), (0.8, 0.5, 1.0), (1.0, 0.0, 0.0)])
def test_ut_off_axis_centre_weight_closed_form(a, b, k):
    """Eq. 9-10 worked by hand for an axis-aligned isotropic particle at
    (x0, 0, z0) in front of a pinhole at the origin.  With g^2 = 3 + lambda the
    seven sigma points are the centre and x0 +/- g s along x, y and z.  Along
    x and y they project symmetrically about the centre's u = c + f x0 / z0;
    along z they land at c + f x0 / (z0 -/+ g s), which pulls the UT mean off
    the centre point by D = a s^2 / (z0^2 - g^2 s^2), a = f x0 / z0.  The
    centre point therefore carries covariance weight into Sigma'_xx through
    its w0^Sigma = lambda/(3+lambda) + (1 - alpha^2 + beta) (Eq. 8): using the
    mean weight there instead drops (1 - alpha^2 + beta) D^2, about 5% here.
    v is symmetric about c_y, so Sigma'_yy = 2 w (f g s / z0)^2 and
    Sigma'_xy = 0."""
    f, cx, cy = 100.0, 200.0, 50.0
    x0, z0, s = 2.0, 3.0, 0.6
    cam = G.camera("pinhole", 400, 100, f, cx=cx, cy=cy)
    p = O.default_params(ut_alpha=a, ut_beta=b, ut_kappa=k)
    sc = O.OScene(np.array([[x0, 0.0, z0]]), np.full((1, 3), s), np.array([[1.0, 0, 0, 0]]),
                  np.array([0.9]), np.zeros((1, 1, 3)), 0)
    pr = O.project(sc, cam, p)
    assert pr["cull"][0] == 0

    lam = a * a * (3 + k) - 3
    g = math.sqrt(3 + lam)
    w = 1.0 / (2 * (3 + lam))                      # every non-centre point
    w0s = lam / (3 + lam) + (1 - a * a + b)        # centre, covariance
    aa = f * x0 / z0
    D = aa * s * s / (z0 * z0 - g * g * s * s)     # UT mean minus the centre's u
    e = f * g * s / z0                             # x- and y-pair offsets
    dz_p = -aa * g * s / (z0 + g * s)              # u(z0 + g s) - u(centre)
    dz_m = aa * g * s / (z0 - g * s)               # u(z0 - g s) - u(centre)
    cov_xx = w0s * D * D + w * ((e - D) ** 2 + (e + D) ** 2 + 2 * D * D
                                + (dz_p - D) ** 2 + (dz_m - D) ** 2)
    cov_yy = 2 * w * e * e
    np.testing.assert_allclose(pr["mean2d"][0], [cx + aa + D, cy], rtol=0, atol=1e-9)
    np.testing.assert_allclose(pr["cov2d"][0], [cov_xx, 0.0, cov_yy], rtol=1e-12, atol=1e-9)
    # the centre term is large enough to matter at this size
    assert (1 - a * a + b) * D * D > 1e-3 * cov_xx or b == a * a - 1


def test_ut_vs_ewa_converges_quadratically():
    """Off axis, the UT covariance approaches the linearised (EWA, Eq. 3)
    covariance J Sigma J^T as the particle shrinks, with error O((s/z)^2)."""
    f, c = 500.0, 0.0
    cam = G.camera("pinhole", 1000, 1000, f, cx=c, cy=c)
    mu = np.array([0.7, -0.4, 2.5])
    q = np.array([0.9, 0.2, -0.3, 0.1])
    R = rot_scipy(q / np.linalg.norm(q))
    errs = []
    for s in [0.04, 0.02, 0.01]:
        sc = O.OScene(mu[None], np.array([[s, 0.5 * s, 0.8 * s]]), q[None], np.array([0.9]),
                      np.zeros((1, 1, 3)), 0)
        pr = O.project(sc, cam)
        x, y, zz = mu
        J = np.array([[f / zz, 0, -f * x / zz ** 2], [0, f / zz, -f * y / zz ** 2]])
        S = R @ np.diag(np.array([s, 0.5 * s, 0.8 * s]) ** 2) @ R.T
        ewa = J @ S @ J.T
        cv = pr["cov2d"][0]
        ut = np.array([[cv[0], cv[1]], [cv[1], cv[2]]])
        errs.append(np.linalg.norm(ut - ewa) / np.linalg.norm(ewa))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.5 < r1 < 4.5 and 3.5 < r2 < 4.5, errs


# ---------------------------------------------------------------------------
# Camera models
# ---------------------------------------------------------------------------

def _fisheye(k, w=400, h=300, f=None):
    return G.camera("fisheye", w, h, f or G.fisheye_focal(w), k=k)


@pytest.mark.parametrize("model", ["pinhole", "fisheye"])
def test_projection_round_trip(model):
    """project(unproject(u)) = u for pixel centres across the image."""
    if model == "pinhole":
        cam = G.camera("pinhole", 320, 240, 300.0, cx=157.3, cy=121.9)
    else:
        cam = _fisheye([0.03, -0.02, 0.01, -0.004])
    rng = np.random.default_rng(0)
    checked = 0
    for _ in range(200):
        u, v = rng.uniform(0, cam["width"]), rng.uniform(0, cam["height"])
        ok, o, d, _ = O.pixel_ray(cam, u, v)
        if not ok:
            continue
        x = o + rng.uniform(0.5, 20) * d / np.linalg.norm(d)
        ok2, uv, _ = O.project_point(cam, x)
        assert ok2
        np.testing.assert_allclose(uv, [u, v], atol=1e-9)
        checked += 1
    assert checked > 100


def test_fisheye_k0_is_equidistant():
    """With k = 0 the OpenCV fisheye model is the equidistant model r = f theta."""
    cam = _fisheye([0, 0, 0, 0], f=250.0)
    for th in [0.01, 0.3, 1.0, 1.5]:
        for ph in [0.0, 0.7, 2.5]:
            x = np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)]) * 3
            ok, uv, _ = O.project_point(cam, x)
            assert ok
            r = np.hypot(uv[0] - cam["cx"], uv[1] - cam["cy"])
            assert abs(r - 250.0 * th) < 1e-9


def test_fisheye_small_angle_matches_pinhole():
    fish = _fisheye([0.04, 0.01, -0.02, 0.005], f=300.0)
    pin = G.camera("pinhole", 400, 300, 300.0)
    for eps in [1e-3, 1e-4]:
        x = np.array([eps, -0.5 * eps, 1.0])
        _, a, _ = O.project_point(fish, x)
        _, b, _ = O.project_point(pin, x)
        assert np.abs(a - b).max() < 300.0 * eps ** 3 * 10


@pytest.mark.parametrize("j,kv", [(0, -0.5), (1, -0.3), (2, -0.2), (3, -0.1)])
def test_theta_lim_single_coefficient_closed_form(j, kv):
    """With one coefficient k_j < 0 the validity limit is the root of
    1 + (2j+3) k_j theta^(2j+2) = 0 when it lies below pi/2."""
    k = [0.0] * 4
    k[j] = kv
    root = (-1.0 / ((2 * j + 3) * kv)) ** (1.0 / (2 * j + 2))
    expect = min(root, math.pi / 2)
    assert abs(O.theta_lim(k) - expect) < 1e-12


def test_theta_lim_is_the_image_radius_maximum():
    """The validity angle is where the projected radius stops growing: a dense
    scan of the projected radius (through project_point) peaks there."""
    k = [-0.05, -0.05, -0.05, -0.05]
    tl = O.theta_lim(k)
    assert tl < math.pi / 2
    cam = _fisheye(k, f=100.0)
    ths = np.linspace(0.5, math.pi / 2, 20001)
    radii = []
    p = O.default_params(near_plane=0.0)
    for th in ths:
        x = np.array([math.sin(th), 0.0, math.cos(th)]) * 2
        _, uv, _ = O.project_point(cam, x, params=p)
        radii.append(uv[0] - cam["cx"])
    th_max = ths[int(np.argmax(radii))]
    assert abs(th_max - tl) < 2 * (ths[1] - ths[0])


def test_fisheye_validity_and_image_circle():
    k = [-0.05, -0.05, -0.05, -0.05]
    cam = _fisheye(k, w=200, h=200, f=60.0)
    tl = O.theta_lim(k)
    ok_in, _, m_in = O.project_point(cam, np.array([math.sin(tl - 1e-3), 0, math.cos(tl - 1e-3)]))
    ok_out, _, m_out = O.project_point(cam, np.array([math.sin(tl + 1e-3), 0, math.cos(tl + 1e-3)]))
    assert ok_in and not ok_out and m_in > 0 > m_out
    ok, _, _, _ = O.pixel_ray(cam, 199.5, 199.5)  # a corner beyond the image circle
    assert not ok


# ---------------------------------------------------------------------------
# Rolling shutter
# ---------------------------------------------------------------------------

def _rs_cam(model="pinhole", pan=0.1, shift=0.3, w=320, h=240):
    R, t = G.look_at((0.5, -0.3, -6.0))
    if model == "pinhole":
        cam = G.camera("pinhole", w, h, G.pinhole_focal(w), R0=R, t0=t)
    else:
        cam = G.camera("fisheye", w, h, G.fisheye_focal(w), k=[0.02, -0.01, 0.0, 0.0], R0=R, t0=t)
    return G.with_motion(cam, pan, shift)


def test_pose_interpolation_matches_scipy_slerp():
    cam = _rs_cam(pan=0.4, shift=0.7)
    Q0, Q1 = cam["R0"].T, cam["R1"].T
    sl = Slerp([0, 1], Rotation.from_matrix([Q0, Q1]))
    c0, c1 = -cam["R0"].T @ cam["t0"], -cam["R1"].T @ cam["t1"]
    for t in [0.0, 0.25, 0.5, 0.9, 1.0]:
        Rwc, cen = O.pose(cam, t)
        np.testing.assert_allclose(Rwc.T, sl([t]).as_matrix()[0], atol=1e-12)
        np.testing.assert_allclose(cen, (1 - t) * c0 + t * c1, atol=1e-12)


def test_zero_motion_rolling_equals_global():
    sc, cams = G.config1()
    cam = cams[0]
    rs = G.with_motion(cam, 0.0, 0.0)
    a = O.project(sc, cam)
    b = O.project(sc, rs)
    for k in ("mean2d", "cov2d", "depth", "rgb"):
        np.testing.assert_allclose(a[k], b[k], atol=1e-10)
    np.testing.assert_array_equal(a["rect"], b["rect"])


@pytest.mark.parametrize("model", ["pinhole", "fisheye"])
def test_rolling_time_matches_bruteforce_root(model):
    """The solved exposure time approaches the row-consistency root
    t = (v_y(x, pose(t)) - 1/2)/(H - 1), found by a dense scan of t."""
    cam = _rs_cam(model)
    rng = np.random.default_rng(3)
    H = cam["height"]
    ts = np.linspace(0, 1, 100001)
    for _ in range(5):
        x = rng.normal(size=3) * np.array([1.5, 1.5, 1.0])
        ok, t3, _, _ = O.solve_time(cam, x, iters=3)
        ok20, t20, _, _ = O.solve_time(cam, x, iters=20)
        if not ok:
            continue
        F = []
        for t in ts[::100]:
            _, v, _ = O.project_point(cam, x, t)
            F.append(np.clip((v[1] - 0.5) / (H - 1), 0, 1) - t)
        F = np.array(F)
        i = np.nonzero(np.diff(np.sign(F)))[0]
        assert len(i) == 1
        lo, hi = ts[::100][i[0]], ts[::100][i[0] + 1]
        for _ in range(60):
            mid = 0.5 * (lo + hi)
            _, v, _ = O.project_point(cam, x, mid)
            f = np.clip((v[1] - 0.5) / (H - 1), 0, 1) - mid
            if np.sign(f) == np.sign(F[i[0]]):
                lo = mid
            else:
                hi = mid
        root = 0.5 * (lo + hi)
        assert abs(t20 - root) < 1e-10
        assert abs(t3 - root) < 1e-3


def test_rolling_pixel_ray_hits_its_row_at_its_time():
    """A point on the ray of pixel (u, v) projects back to (u, v) at the
    exposure time of row floor(v)."""
    cam = _rs_cam("fisheye")
    for u, v in [(60.5, 50.5), (160.5, 120.5), (280.5, 180.5)]:
        ok, o, d, _ = O.pixel_ray(cam, u, v)
        assert ok
        t = math.floor(v) / (cam["height"] - 1)
        _, uv, _ = O.project_point(cam, o + 5.0 * d / np.linalg.norm(d), t)
        np.testing.assert_allclose(uv, [u, v], atol=1e-8)


# ---------------------------------------------------------------------------
# Particle response (Eq. 1, Eq. 11)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(4))
def test_tau_max_forms_and_argmax(seed):
    """Eq. 11: the world-space form (mu-o)^T Sigma^-1 d / d^T Sigma^-1 d equals
    the canonical form, and it maximises the response along the ray."""
    rng = np.random.default_rng(seed)
    mu, q, s = rng.normal(size=3), rng.normal(size=4), np.exp(rng.normal(-1, 0.4, 3))
    o, d = rng.normal(size=3) * 3, rng.normal(size=3)
    R = rot_scipy(q / np.linalg.norm(q))
    Si = np.linalg.inv(R @ np.diag(s ** 2) @ R.T)
    tau_world = (mu - o) @ Si @ d / (d @ Si @ d)
    _, tau, om2, _ = O.particle_alpha(mu, q, s, 0.8, o, d)
    assert abs(tau - tau_world) < 1e-12 * max(1, abs(tau))
    taus = tau + np.linspace(-3, 3, 60001) * (1 + abs(tau))
    x = o[None] + taus[:, None] * d[None]
    rho = np.exp(-0.5 * np.einsum("ni,ij,nj->n", x - mu, Si, x - mu))
    assert abs(taus[np.argmax(rho)] - tau) <= (taus[1] - taus[0])
    assert abs(rho.max() - math.exp(-0.5 * om2)) < 1e-8


def test_single_isotropic_particle_closed_form():
    """One isotropic particle: pixel = c sigma exp(-d_perp^2 / (2 s^2)) with
    d_perp the distance from the centre to the pixel ray (vector geometry)."""
    cam = G.camera("pinhole", 64, 64, 80.0, R0=np.eye(3), t0=np.array([0.0, 0.0, 4.0]))
    s, sig, col = 0.15, 0.8, np.array([0.9, 0.4, 0.1])
    mu = np.array([0.1, -0.05, 0.2])
    sh = ((col - 0.5) / G.SH_C0)[None, None, :]
    sc = O.OScene(mu[None], np.full((1, 3), s), np.array([[0.3, 0.1, 0.7, -0.2]]),
                  np.array([sig]), sh, 0)
    pr, b, res = O.render_full(sc, cam)
    img = O.to_image(res, cam)
    o = np.array([0.0, 0.0, -4.0])
    worst = 0.0
    n_checked = 0
    for py in range(64):
        for px in range(64):
            d = np.array([(px + 0.5 - 32) / 80.0, (py + 0.5 - 32) / 80.0, 1.0])
            dperp = np.linalg.norm(np.cross(mu - o, d / np.linalg.norm(d)))
            a = sig * math.exp(-dperp ** 2 / (2 * s * s))
            if a < 1 / 255 + 1e-6 or a > 0.99:
                continue
            worst = max(worst, np.abs(img[py, px] - col * a).max())
            n_checked += 1
    assert n_checked > 50 and worst < 1e-12


# ---------------------------------------------------------------------------
# Generalized Gaussian response of degree n (Supp. A)
# ---------------------------------------------------------------------------

def _lambda_from_definition(n):
    """The scale that gives the degree-n kernel the reference Gaussian's
    response at canonical distance r = 3: lambda 3^n = 3^2 / 2."""
    return 4.5 / 3.0 ** n


@pytest.mark.parametrize("n", [2, 3, 4, 5, 8])
@pytest.mark.parametrize("seed", range(3))
def test_generalized_response_equals_gaussian_at_r3(n, seed):
    """Supp. A defines lambda so that every degree has the Gaussian's
    response at distance r = 3: a ray passing 3 s from an isotropic
    particle's centre sees sigma exp(-9/2) whatever n."""
    rng = np.random.default_rng(seed)
    mu, s, sig = rng.normal(size=3), math.exp(rng.normal(-1, 0.3)), 0.7
    q = rng.normal(size=4)
    d = rng.normal(size=3)
    d /= np.linalg.norm(d)
    perp = np.cross(d, rng.normal(size=3))
    perp /= np.linalg.norm(perp)
    o = mu + 3.0 * s * perp - 5.0 * d  # closest approach 3 s, in front of the origin
    ok, tau, om2, a = O.particle_alpha(mu, q, np.full(3, s), sig, o, d, n)
    assert ok and abs(om2 - 9.0) < 1e-9
    assert abs(a - sig * math.exp(-4.5)) < 1e-12


@pytest.mark.parametrize("w", [0.0, 0.5, 1.7, 2.9, 3.1, 4.0])
def test_generalized_response_denser_inside_steeper_outside(w):
    """Higher degrees are denser inside r = 3 and fall off faster outside
    (Supp. A, Fig. of the generalized particle); degree 2 is exp(-w^2/2)."""
    mu, q, s = np.zeros(3), np.array([1.0, 0, 0, 0]), np.ones(3)
    o, d = np.array([w, 0.0, -6.0]), np.array([0.0, 0.0, 1.0])
    vals = [O.particle_alpha(mu, q, s, 1.0, o, d, n)[3] for n in (2, 3, 4, 5, 8)]
    assert abs(vals[0] - math.exp(-0.5 * w * w)) < 1e-15
    steps = np.diff(vals)
    if w == 0.0:
        assert np.all(np.abs(np.array(vals) - 1.0) < 1e-15)
    elif w < 3.0:
        assert np.all(steps > 0)
    else:
        assert np.all(steps < 0)


@pytest.mark.parametrize("n", [3, 4, 8])
def test_generalized_single_particle_closed_form_and_extent(n):
    """One isotropic particle of low opacity rendered with the degree-n
    response: every pixel equals c sigma exp(-lambda (d_perp / s)^n) with
    lambda from Supp. A's definition and d_perp from vector geometry.  The
    particle sits so that its degree-n alpha_min circle crosses into a tile
    column that the Gaussian's (smaller, for this opacity) circle does not
    reach: an extent computed for the Gaussian would leave those pixels black.
    Rendered with the whole rectangle (no tile culling); with tile culling the
    pixels inside the UT extent ellipse keep these values and the others keep
    them or lose the particle entirely (the UT ellipse of this near particle,
    s/z = 0.12, undershoots its exact silhouette by O((s/z)^2), so tiles that
    only the silhouette reaches are culled: the approximation the rectangle
    itself makes at its edges)."""
    cam = G.camera("pinhole", 128, 128, 80.0, R0=np.eye(3), t0=np.array([0.0, 0.0, 4.0]))
    s, sig, col = 0.5, 0.1, np.array([0.9, 0.4, 0.1])
    mu = np.array([9.2 * 4.2 / 80.0, 0.0, 0.2])  # centre 9.2 px right of the principal point
    sh = ((col - 0.5) / G.SH_C0)[None, None, :]
    sc = O.OScene(mu[None], np.full((1, 3), s), np.array([[0.3, 0.1, 0.7, -0.2]]),
                  np.array([sig]), sh, 0)
    p = O.default_params(kernel_degree=n, tile_cull=0)
    pr, b, res = O.render_full(sc, cam, p)
    img = O.to_image(res, cam, p)
    pc = O.default_params(kernel_degree=n)
    _, _, resc = O.render_full(sc, cam, pc)
    imc = O.to_image(resc, cam, pc)
    A = pr["kext"][0] ** 2 * pr["cov2d"][0]
    Q = np.linalg.inv(np.array([[A[0], A[1]], [A[1], A[2]]]))
    lam = _lambda_from_definition(n)
    k_gauss = math.sqrt(2 * math.log(sig * 255))
    o = np.array([0.0, 0.0, -4.0])
    worst, n_checked, ring = 0.0, 0, 0
    for py in range(128):
        for px in range(128):
            d = np.array([(px + 0.5 - 64) / 80.0, (py + 0.5 - 64) / 80.0, 1.0])
            w = np.linalg.norm(np.cross(mu - o, d / np.linalg.norm(d))) / s
            a = sig * math.exp(-lam * w ** n)
            if abs(a - 1 / 255) < 1e-6:
                continue
            expect = col * a if a >= 1 / 255 else np.zeros(3)
            worst = max(worst, np.abs(img[py, px] - expect).max())
            dv = np.array([px + 0.5, py + 0.5]) - pr["mean2d"][0]
            if dv @ Q @ dv <= 1.0:
                worst_c = np.abs(imc[py, px] - expect).max()
            else:
                worst_c = min(np.abs(imc[py, px] - expect).max(), np.abs(imc[py, px]).max())
            worst = max(worst, worst_c)
            n_checked += 1
            if a >= 1 / 255 and w > k_gauss and px < 48:
                ring += 1
    assert n_checked > 16000 and ring > 0
    assert worst < 1e-12


# ---------------------------------------------------------------------------
# Hybrid-rendering depth clip (Sec. 6.2)
# ---------------------------------------------------------------------------

def test_clip_at_infinity_changes_nothing():
    sc, cams = G.config1()
    cam = cams[0]
    pr, b, res = O.render_full(sc, cam)
    clip = np.full((cam["height"], cam["width"]), np.inf)
    res2 = O.render(sc, pr, cam, b, clip=clip)
    for k in ("rgb", "T", "n_contrib", "n_eval"):
        np.testing.assert_array_equal(res[k], res2[k])


@pytest.mark.parametrize("clipd,which", [(3.0, "none"), (4.6, "front"), (20.0, "both")])
def test_clip_two_particles_closed_form(clipd, which):
    """Two isotropic particles in front of each other: a clip distance before
    both, between them, or past both keeps no hit, the front one, or both.
    Each hit's distance is the centre's projection on the ray and its alpha
    sigma exp(-d_perp^2 / 2 s^2) (vector geometry)."""
    cam = G.camera("pinhole", 32, 32, 40.0, R0=np.eye(3), t0=np.array([0.0, 0.0, 4.0]))
    mus = np.array([[0.02, -0.01, 0.0], [-0.03, 0.02, 1.2]])
    s = np.array([0.15, 0.2])
    sig = np.array([0.6, 0.8])
    cols = np.array([[0.9, 0.2, 0.1], [0.1, 0.3, 0.95]])
    sh = ((cols - 0.5) / G.SH_C0)[:, None, :]
    sc = O.OScene(mus, np.repeat(s[:, None], 3, 1), np.array([[1.0, 0, 0, 0], [0.6, 0.2, -0.3, 0.7]]),
                  sig, sh, 0)
    p = O.default_params()
    pr = O.project(sc, cam, p)
    b = O.bin_tiles(pr, cam, p)
    clip = np.full((32, 32), clipd)
    img = O.to_image(O.render(sc, pr, cam, b, p, clip=clip), cam, p)
    o = np.array([0.0, 0.0, -4.0])
    n_checked = 0
    for py in range(8, 24, 2):
        for px in range(8, 24, 2):
            d = np.array([(px + 0.5 - 16) / 40.0, (py + 0.5 - 16) / 40.0, 1.0])
            dh = d / np.linalg.norm(d)
            expect, T = np.zeros(3), 1.0
            for k in range(2):  # front to back (sorted depth order is 0, 1)
                dist = (mus[k] - o) @ dh
                a = sig[k] * math.exp(-np.linalg.norm(np.cross(mus[k] - o, dh)) ** 2 / (2 * s[k] ** 2))
                if a < 1 / 255 or dist > clipd:
                    continue
                expect += T * a * cols[k]
                T *= 1 - a
            np.testing.assert_allclose(img[py, px], expect, atol=1e-12)
            n_checked += 1
    assert n_checked == 64
    centre = img[16, 16]
    if which == "none":
        assert np.all(centre == 0)
    elif which == "front":
        assert centre[0] > centre[2]   # the red front particle alone
    else:
        assert centre[2] > 0.2          # the blue one behind shows through


# ---------------------------------------------------------------------------
# "Ours (sorted)": the per-ray k-buffer (Sec. 4.3)
# ---------------------------------------------------------------------------

def _iso_scene(mus, s, sig, cols):
    n = len(mus)
    sh = ((np.asarray(cols) - 0.5) / G.SH_C0)[:, None, :]
    q = np.tile([1.0, 0.0, 0.0, 0.0], (n, 1))
    return O.OScene(np.asarray(mus, float), np.repeat(np.asarray(s, float)[:, None], 3, 1), q,
                    np.asarray(sig, float), sh, 0)


def _composite(hits, p):
    """Eq. 5 over (alpha, colour) in the given order, stopping before a hit
    that would take T below t_min."""
    T, C = 1.0, np.zeros(3)
    for a, c in hits:
        if T * (1 - a) < p["t_min"]:
            break
        C += T * a * np.asarray(c)
        T *= 1 - a
    return C, T


def test_kbuffer_worked_example_three_hits():
    """Three particles listed A, B, C (by centre distance 5.0, 5.51, 5.66) whose
    hits on the axis ray lie at 5.0, 5.5 and 4.8: tile order composites A, B,
    C; a buffer of one blends A (B arrives farther), then C (nearer than the
    buffered B), then B at the end; a buffer of three blends them sorted,
    C, A, B."""
    cam = G.camera("pinhole", 33, 33, 40.0, cx=16.5, cy=16.5)  # pixel (16, 16) looks along +z
    mus = [[0, 0, 5.0], [0, 0.3, 5.5], [0, 3.0, 4.8]]
    sig = [0.7, 0.8, 0.9]
    s = [0.6, 0.6, 1.5]
    cols = [[1, 0, 0], [0, 1, 0], [0, 0, 1]]
    sc = _iso_scene(mus, s, sig, cols)
    o, d = np.zeros(3), np.array([0.0, 0.0, 1.0])
    hit = {}
    for name, i in zip("ABC", range(3)):
        ok, tau, om2, a = O.particle_alpha(mus[i], [1, 0, 0, 0], [s[i]] * 3, sig[i], o, d)
        assert ok and a > 1 / 255
        hit[name] = (min(a, 0.99), cols[i], tau)
    assert hit["C"][2] < hit["A"][2] < hit["B"][2]
    base = O.default_params()
    for k, order in ((0, "ABC"), (1, "ACB"), (3, "CAB"), (16, "CAB")):
        p = O.default_params(kbuffer=k)
        pr = O.project(sc, cam, p)
        assert (pr["cull"] == 0).all()
        b = O.bin_tiles(pr, cam, p)
        img = O.to_image(O.render(sc, pr, cam, b, p), cam, p)
        C, T = _composite([hit[x][:2] for x in order], base)
        np.testing.assert_allclose(img[16, 16], C, atol=1e-12, err_msg=f"k={k}")


def test_kbuffer_large_k_is_per_ray_sorted_compositing():
    """With a buffer larger than any pixel's hit count, every pixel composites
    its hits in exact distance order (brute force per pixel); tile order
    differs on many pixels of this overlapping scene."""
    rng = np.random.default_rng(31)
    n = 30
    mus = np.column_stack([rng.uniform(-0.6, 0.6, (n, 2)), rng.uniform(-0.8, 0.8, n)])
    s = np.exp(rng.normal(-1.3, 0.2, n))
    sig = rng.uniform(0.2, 0.6, n)
    cols = rng.uniform(0, 1, (n, 3))
    sc = _iso_scene(mus, s, sig, cols)
    cam = G.camera("pinhole", 24, 24, 20.0, R0=np.eye(3), t0=np.array([0.0, 0.0, 4.0]))
    p = O.default_params(kbuffer=64)
    pr = O.project(sc, cam, p)
    b = O.bin_tiles(pr, cam, p)
    vis = pr["cull"] == 0
    img = O.to_image(O.render(sc, pr, cam, b, p), cam, p)
    img0 = O.to_image(O.render(sc, pr, cam, b, O.default_params()), cam)
    o = np.array([0.0, 0.0, -4.0])
    tx, _ = O.tiles_xy(cam, p)
    worst, n_diff = 0.0, 0
    for py in range(24):
        for px in range(24):
            d = np.array([(px + 0.5 - 12) / 20.0, (py + 0.5 - 12) / 20.0, 1.0])
            t = (py // 16) * tx + px // 16
            hits = []
            for i in range(n):
                r = pr["rect"][i]
                if not vis[i] or not (r[0] <= px // 16 <= r[2] and r[1] <= py // 16 <= r[3]):
                    continue
                ok, tau, om2, a = O.particle_alpha(mus[i], [1, 0, 0, 0], [s[i]] * 3, sig[i], o, d)
                a = min(a, p["alpha_max"])
                if ok and a >= p["alpha_min"]:
                    hits.append((tau * np.linalg.norm(d), a, cols[i]))
            hits.sort(key=lambda h: h[0])
            C, T = _composite([(a, c) for _, a, c in hits], p)
            worst = max(worst, np.abs(img[py, px] - C).max())
            n_diff += np.abs(img0[py, px] - C).max() > 1e-3
    assert worst < 1e-12
    assert n_diff > 50


def test_kbuffer_in_list_order_equals_tile_order():
    """Hits that arrive already in distance order (particles strung along the
    axis, far apart in depth) blend in list order for any buffer size."""
    mus = [[0.02 * i, -0.01 * i, -1.0 + 0.5 * i] for i in range(6)]
    sc = _iso_scene(mus, [0.3] * 6, [0.5] * 6, np.eye(3)[[0, 1, 2, 0, 1, 2]])
    cam = G.camera("pinhole", 32, 32, 40.0, R0=np.eye(3), t0=np.array([0.0, 0.0, 4.0]))
    ref = None
    for k in (0, 1, 2, 16):
        p = O.default_params(kbuffer=k)
        pr, b, res = O.render_full(sc, cam, p)
        img = O.to_image(res, cam, p)
        if ref is None:
            ref = img
        np.testing.assert_allclose(img, ref, atol=1e-13, err_msg=f"k={k}")


# ---------------------------------------------------------------------------
# Compositing (Eq. 5)
# ---------------------------------------------------------------------------

def _white(scene):
    sh = np.zeros_like(scene.sh)
    sh[:, 0, :] = 0.5 / G.SH_C0
    return O.OScene(scene.means, scene.scales, scene.quats, scene.opacities, sh, scene.sh_degree)


def test_weights_plus_transmittance_sum_to_one():
    """With unit colour and black background, C = sum_i alpha_i T_i, so
    C + T_final = 1 telescopes exactly."""
    sc, cams = G.config1()
    w = _white(sc)
    pr, b, res = O.render_full(w, cams[0])
    m = res["inside"] == 1
    np.testing.assert_allclose(res["rgb"][m, 0] + res["T"][m], 1.0, atol=1e-12)


def test_two_particle_order_closed_form():
    """Front particle first: C = c1 a1 + c2 a2 (1 - a1) on the line of sight."""
    cam = G.camera("pinhole", 16, 16, 20.0, R0=np.eye(3), t0=np.array([0.0, 0.0, 5.0]))
    cols = np.array([[0.9, 0.1, 0.2], [0.2, 0.8, 0.6]])
    mu = np.array([[0.0, 0.0, -1.0], [0.0, 0.0, 1.0]])  # depth 4 and 6
    sh = ((cols - 0.5) / G.SH_C0)[:, None, :]
    sc = O.OScene(mu, np.full((2, 3), 0.5), np.tile([1.0, 0, 0, 0], (2, 1)), np.array([0.7, 0.6]),
                  sh, 0)
    pr, b, res = O.render_full(sc, cam)
    img = O.to_image(res, cam)
    o = np.array([0, 0, -5.0])
    d = np.array([(8.5 - 8) / 20, (8.5 - 8) / 20, 1.0])
    a = [sg * math.exp(-np.linalg.norm(np.cross(m - o, d / np.linalg.norm(d))) ** 2 / 0.5)
         for m, sg in zip(mu, [0.7, 0.6])]
    expect = cols[0] * a[0] + cols[1] * a[1] * (1 - a[0])
    np.testing.assert_allclose(img[8, 8], expect, atol=1e-12)


def test_early_termination_closed_form():
    """Ten stacked particles of alpha 0.9 on the axis: T falls 10x per layer;
    with T_min = 5e-5 the fifth would take T below it, so it is not added and
    T_final = 1e-4."""
    cam = G.camera("pinhole", 16, 16, 20.0, R0=np.eye(3), t0=np.array([0.0, 0.0, 5.0]))
    n = 10
    mu = np.stack([np.zeros(n), np.zeros(n), np.linspace(-1, 1, n)], 1)
    sh = np.full((n, 1, 3), 0.5 / G.SH_C0)
    p = O.default_params(alpha_max=1.0, t_min=5e-5)
    # opacity chosen so alpha at the exact centre ray is 0.9: put the pixel ray through the axis
    cam["cx"] = cam["cy"] = 8.5
    sc = O.OScene(mu, np.full((n, 3), 0.2), np.tile([1.0, 0, 0, 0], (n, 1)), np.full(n, 0.9), sh, 0)
    pr, b, res = O.render_full(sc, cam, params=p)
    px = (8 // 16) * 256 + 8 * 16 + 8
    assert res["n_contrib"][px] == 4
    assert res["n_eval"][px] == 5
    assert abs(res["T"][px] - 0.1 ** 4) < 1e-15
    np.testing.assert_allclose(res["rgb"][px] + res["T"][px], 1.0, atol=1e-15)
    assert abs(res["rgb"][px, 0] - (1 - 0.1 ** 4)) < 1e-14


def test_alpha_min_skip():
    """A particle whose alpha at the pixel is below 1/255 is skipped entirely."""
    cam = G.camera("pinhole", 16, 16, 20.0, R0=np.eye(3), t0=np.array([0.0, 0.0, 5.0]))
    cam["cx"] = cam["cy"] = 8.5
    sh = np.full((1, 1, 3), 0.5 / G.SH_C0)
    for sig, expect_contrib in [(0.0039, 0), (0.004, 1)]:
        sc = O.OScene(np.zeros((1, 3)), np.full((1, 3), 0.2), np.array([[1.0, 0, 0, 0]]),
                      np.array([sig]), sh, 0)
        p = O.default_params(alpha_min=1 / 255)
        pr, b, res = O.render_full(sc, cam, params=p)
        px = 8 * 16 + 8
        assert res["n_contrib"][px] == expect_contrib


# ---------------------------------------------------------------------------
# Culling and tiling
# ---------------------------------------------------------------------------

def test_tiled_equals_bruteforce_when_rects_cover_everything():
    """Large particles whose rectangles cover every tile: the tiled render and
    the no-culling brute-force render (every particle, every pixel) agree."""
    rng = np.random.default_rng(5)
    n = 40
    cam = G.camera("pinhole", 48, 48, 30.0, R0=np.eye(3), t0=np.array([0.0, 0.0, 4.0]))
    sc = O.OScene(rng.uniform(-0.3, 0.3, (n, 3)), np.exp(rng.normal(0.3, 0.1, (n, 3))),
                  rng.normal(size=(n, 4)), rng.uniform(0.05, 0.2, n),
                  rng.normal(0, 1, (n, 1, 3)), 0)
    p = O.default_params(tile_cull=0)
    pr = O.project(sc, cam, p)
    assert (pr["cull"] == 0).all() and (pr["tiles"] == 9).all()
    b = O.bin_tiles(pr, cam, p)
    tiled = O.render(sc, pr, cam, b, p)
    brute = O.render(sc, pr, cam, None, p, brute_force=True)
    np.testing.assert_allclose(tiled["rgb"], brute["rgb"], atol=1e-15)
    np.testing.assert_array_equal(tiled["n_contrib"], brute["n_contrib"])


def test_tiled_close_to_bruteforce_config1():
    """In general the tiled render drops only response outside each
    particle's extent box, so it stays close to the brute-force render."""
    sc, cams = G.config1()
    cam = cams[0]
    pr = O.project(sc, cam)
    b = O.bin_tiles(pr, cam)
    tiled = O.render(sc, pr, cam, b, alternatives=False)
    brute = O.render(sc, pr, cam, None, brute_force=True, alternatives=False)
    d = np.abs(tiled["rgb"] - brute["rgb"]).max()
    assert d < 0.05
    assert np.mean(np.abs(tiled["rgb"] - brute["rgb"]).max(1) < 1e-9) > 0.9


def test_tile_lists_bruteforce():
    """Without tile culling each tile's list holds exactly the visible
    particles whose rectangle covers it, ordered by (depth, id)."""
    sc, cams = G.config1()
    cam = cams[0]
    pr = O.project(sc, cam)
    ts, ids, fl = O.bin_tiles(pr, cam, O.default_params(tile_cull=0))
    prim = fl & 1 == 1
    tx, ty = O.tiles_xy(cam, O.default_params())
    vis = np.nonzero(pr["cull"] == 0)[0]
    for t in range(tx * ty):
        x, y = t % tx, t // tx
        r = pr["rect"][vis]
        cov = vis[(r[:, 0] <= x) & (x <= r[:, 2]) & (r[:, 1] <= y) & (y <= r[:, 3])]
        order = sorted(cov, key=lambda i: (pr["depth"][i], i))
        seg = slice(ts[t], ts[t + 1])
        got = ids[seg][prim[seg]]
        assert list(got) == list(order)


def test_opacity_and_near_culls():
    sc, cams = G.config1()
    cam = cams[0]
    pr = O.project(sc, cam)
    low = sc.opacities < np.float32(1 / 255)
    assert (pr["cull"][low] == 1).all()
    # a particle straddling the near plane of a camera placed inside the cloud
    cam2 = G.camera("pinhole", 64, 64, 60.0, R0=np.eye(3), t0=np.array([0.0, 0.0, -0.1]))
    sc2 = O.OScene(np.array([[0.0, 0.0, 0.3]]), np.full((1, 3), 0.1), np.array([[1.0, 0, 0, 0]]),
                   np.array([0.9]), np.zeros((1, 1, 3)), 0)
    pr2 = O.project(sc2, cam2)
    assert pr2["cull"][0] == 2


def test_depth_and_degree0_colour():
    sc, cams = G.config1()
    cam = cams[0]
    pr = O.project(sc, cam)
    eye = np.array([0, 0, -3.0])
    vis = pr["cull"] != 1
    np.testing.assert_allclose(pr["depth"][vis], np.linalg.norm(sc.means[vis] - eye, axis=1),
                               rtol=1e-12)
    dc = 0.5 + G.SH_C0 * sc.sh[:, 0, :].astype(np.float64)
    np.testing.assert_allclose(pr["rgb"][vis], np.maximum(dc[vis], 0), atol=1e-12)


# ---------------------------------------------------------------------------
# Spherical harmonics
# ---------------------------------------------------------------------------

def test_sh_matches_scipy():
    """Real SH with the Condon-Shortley phase: sqrt2 Re Y_l^m (m>0),
    sqrt2 Im Y_l^|m| (m<0), Y_l^0, from scipy's complex harmonics."""
    from scipy.special import sph_harm_y
    rng = np.random.default_rng(0)
    for _ in range(20):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        th, ph = math.acos(d[2]), math.atan2(d[1], d[0])
        Y = O.sh_basis(3, d)
        for l in range(4):
            for m in range(-l, l + 1):
                y = sph_harm_y(l, abs(m), th, ph)
                ref = y.real if m == 0 else (math.sqrt(2) * (y.real if m > 0 else y.imag))
                assert abs(Y[l * l + l + m] - ref) < 1e-12, (l, m)


def test_sh_orthonormal_by_quadrature():
    x, w = np.polynomial.legendre.leggauss(16)
    phis = np.arange(32) * 2 * np.pi / 32
    G_ = np.zeros((16, 16))
    for zi, wi in zip(x, w):
        for ph in phis:
            r = math.sqrt(1 - zi * zi)
            Y = O.sh_basis(3, [r * math.cos(ph), r * math.sin(ph), zi])
            G_ += wi * (2 * np.pi / 32) * np.outer(Y, Y)
    np.testing.assert_allclose(G_, np.eye(16), atol=1e-12)


def test_sh_gradient_tangential_matches_differences():
    rng = np.random.default_rng(1)
    for _ in range(5):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        dY = O.sh_basis_grad(3, d)
        P = np.eye(3) - np.outer(d, d)
        for j in range(3):
            e = np.zeros(3)
            e[j] = 1e-6
            f = lambda v: O.sh_basis(3, v / np.linalg.norm(v))
            fd = (f(d + e) - f(d - e)) / 2e-6
            np.testing.assert_allclose(fd, (dY @ P)[:, j], atol=1e-8)
