"""gut_bin against a plain sort of its own inputs.

Given the projected rectangles, tiles-touched counts, FP32 depths and (with
tile culling) the extent ellipses, the tile lists are fixed: every (tile,
entry) pair of the rectangles whose tile box meets the ellipse
(v - m)^T A^-1 (v - m) <= 1 (A = k^2 Sigma', as the projection wrote it),
ordered by (global tile id, depth bits, entry id) -- the per-tile depth order
of Sec. 4.3 with the id tie-break.  This test expands the pairs with numpy
from the same projection outputs the kernels read, decides each tile by the
minimum of the quadratic form over the tile's box (a different computation
from the kernels' per-row ellipse extents), sorts with np.lexsort, and
requires identical lists, ranges and pair count; only pairs whose box lies
within 1e-9 of the ellipse's boundary may go either way.  At the full
benchmark sizes, with lists above 4096 and 8192 entries, cameras counted in
LDS and in global memory, and both tile rules.
"""
import sys

import numpy as np
import pytest
import torch

import gut_synth as G
from paper_2412_12507_amd import raster as R

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def box_qmin(mx, my, a, b, c, x0, y0, x1, y1):
    """Minimum of (v-m)^T A^-1 (v-m), A = [[a, b], [b, c]], over the boxes
    [x0, x1] x [y0, y1] (arrays): 0 inside, else the smallest of the four
    edges' clamped one-dimensional minima."""
    det = a * c - b * b
    Qxx, Qxy, Qyy = c / det, -b / det, a / det
    best = np.full(mx.shape, np.inf)
    for X in (x0, x1):
        dx = X - mx
        y = np.clip(my - Qxy * dx / Qyy, y0, y1)
        dy = y - my
        best = np.minimum(best, Qxx * dx * dx + 2 * Qxy * dx * dy + Qyy * dy * dy)
    for Y in (y0, y1):
        dy = Y - my
        x = np.clip(mx - Qxy * dy / Qxx, x0, x1)
        dx = x - mx
        best = np.minimum(best, Qxx * dx * dx + 2 * Qxy * dx * dy + Qyy * dy * dy)
    inside = (mx >= x0) & (mx <= x1) & (my >= y0) & (my <= y1)
    return np.where(inside, 0.0, best)


def expected_bins(proj, cams, n, cull):
    """Pairs in (tile, depth bits, entry) order, and which are undecided."""
    rect = proj.rect.cpu().numpy().astype(np.int64)
    tiles = proj.tiles.cpu().numpy().astype(np.int64)
    dbits = proj.depth.cpu().numpy().view(np.uint32).astype(np.int64)
    base, tx = [], []
    b = 0
    for cam in cams:
        txc = -(-int(cam["width"]) // 16)
        tyc = -(-int(cam["height"]) // 16)
        base.append(b)
        tx.append(txc)
        b += txc * tyc
    T = b
    ent = np.nonzero(tiles > 0)[0]
    r = rect[ent]
    w = r[:, 2] - r[:, 0] + 1
    h = r[:, 3] - r[:, 1] + 1
    assert np.array_equal(w * h, tiles[ent]), "tiles touched != rectangle area"
    cnt = tiles[ent]
    P = int(cnt.sum())
    start = np.cumsum(cnt) - cnt
    e_rep = np.repeat(ent, cnt)
    k = np.arange(P, dtype=np.int64) - np.repeat(start, cnt)
    w_rep = np.repeat(w, cnt)
    y, x = k // w_rep, k % w_rep
    ty = np.repeat(r[:, 1], cnt) + y
    txl = np.repeat(r[:, 0], cnt) + x
    cam = e_rep // n
    tile = np.asarray(base)[cam] + ty * np.asarray(tx)[cam] + txl
    amb = np.zeros(P, bool)
    if cull:
        m = proj.mean2d.cpu().numpy().astype(np.float64)[e_rep]
        A = proj.extent.cpu().numpy().astype(np.float64)[e_rep]
        a, bb, c = A[:, 0], A[:, 1], A[:, 2]
        det = a * c - bb * bb
        ok = (det > 0) & (a > 0) & (c > 0)  # degenerate ellipses keep the rectangle
        with np.errstate(divide="ignore", invalid="ignore"):
            q = box_qmin(m[:, 0], m[:, 1], a, bb, c, 16.0 * txl, 16.0 * ty, 16.0 * txl + 16, 16.0 * ty + 16)
        keep = ~ok | (q <= 1.0)
        amb = ok & (np.abs(np.sqrt(np.abs(q)) - 1.0) <= 1e-9)
        e_rep, tile, amb = e_rep[keep | amb], tile[keep | amb], amb[keep | amb]
    order = np.lexsort((e_rep, dbits[e_rep], tile))
    return e_rep[order], tile[order], amb[order], T


def check(scene, cams, capacity=None, params=None):
    gs = R.GaussianScene.from_host(scene)
    proj = R.project(gs, cams, params)
    bins = R.bin_tiles(proj, cams, params, capacity=capacity)
    torch.cuda.synchronize()
    cull = (params or {}).get("tile_cull", 1) != 0
    ids, tile, amb, T = expected_bins(proj, cams, gs.n, cull)
    P = bins.n_pairs
    say(f"  n={gs.n} cams={len(cams)} T={T} P={P} expected {len(ids) - amb.sum()}..{len(ids)}"
        f" (rectangles {int(proj.tiles.to(torch.int64).sum().item())})")
    got_ids = bins.ids[:P].cpu().numpy().astype(np.int64)
    got_ranges = bins.ranges.cpu().numpy().astype(np.int64)
    assert got_ranges.shape == (T, 2)
    # ranges partition [0, P) in tile order
    lens = got_ranges[:, 1] - got_ranges[:, 0]
    assert (lens >= 0).all() and lens.sum() == P
    nz = lens > 0
    assert (got_ranges[nz, 0] == (np.cumsum(lens) - lens)[nz]).all()
    if not amb.any():
        exp_lens = np.bincount(tile, minlength=T)
        assert P == len(ids)
        badr = np.nonzero(lens != exp_lens)[0]
        assert badr.size == 0, f"{badr.size} list lengths differ, first tiles {badr[:5]}"
        bad = np.nonzero(got_ids != ids)[0]
        assert bad.size == 0, f"{bad.size} ids differ, first at {bad[:5]}"
        return bins
    say(f"  {int(amb.sum())} undecided pairs")
    gt = np.repeat(np.arange(T), lens)
    dec = ~amb
    # every decided pair present, undecided ones optional, order exact
    exp_keys = set(zip(tile[dec].tolist(), ids[dec].tolist()))
    all_keys = set(zip(tile.tolist(), ids.tolist()))
    got_keys = list(zip(gt.tolist(), got_ids.tolist()))
    assert len(set(got_keys)) == P
    assert exp_keys <= set(got_keys) and set(got_keys) <= all_keys
    drop = set(zip(tile[amb].tolist(), ids[amb].tolist())) - set(got_keys)
    keepm = np.array([(t, i) not in drop for t, i in zip(tile.tolist(), ids.tolist())])
    assert np.array_equal(got_ids, ids[keepm])
    return bins


def test_bin_exact_c1():
    say("[bin exact] c1, 64 tiles")
    scene, cams = G.config1()
    check(scene, cams[:1])


def test_bin_exact_c2_full():
    say("[bin exact] 1M Gaussians, pinhole + fisheye 1920x1080, tile culling")
    check(G.config2_scene(), G.config2_cameras())


def test_bin_exact_c2_full_rectangles():
    say("[bin exact] 1M Gaussians, pinhole + fisheye 1920x1080, whole rectangles")
    check(G.config2_scene(), G.config2_cameras(), params=dict(tile_cull=0))


def test_bin_exact_c3_full_long_lists():
    say("[bin exact] 3M Gaussians, rolling-shutter fisheye 1600x1200: lists over 4096 and 8192")
    bins = check(G.config3_scene(), [G.config3_camera()])
    lens = np.diff(bins.ranges.cpu().numpy().astype(np.int64), axis=1)
    assert (lens >= 4096).sum() > 0 and (lens > 8192).sum() > 0


def test_bin_exact_nine_views():
    say("[bin exact] nine 1920x1080 views (73440 tiles)")
    scene = G.clustered_scene(40000, seed=1002)
    pin, fish = G.config2_cameras()
    cams = [pin, fish] * 4 + [G.config3_camera(1920, 1080)]
    check(scene, cams)


def test_bin_exact_after_capacity_retry():
    say("[bin exact] pair buffer too small: GUT_E_CAPACITY, then retry")
    scene = G.clustered_scene(20000, seed=1002)
    check(scene, G.config2_cameras(320, 180), capacity=4096)


def test_bin_nothing_visible():
    say("[bin exact] every particle behind the camera")
    scene, cams = G.config1()
    cam = G.camera("pinhole", 64, 48, 60.0, R0=np.eye(3), t0=np.array([0.0, 0.0, -10.0]))
    bins = check(scene, [cam])
    assert bins.n_pairs == 0
    assert (bins.ranges.cpu().numpy() == 0).all()


def test_bin_exact_8k_camera_counted_in_global_memory():
    say("[bin exact] one 7680x4320 view (480x270 tiles, beyond the LDS histogram)")
    scene = G.clustered_scene(40000, seed=1002)
    cam = G.camera("pinhole", 7680, 4320, G.pinhole_focal(7680), R0=np.eye(3), t0=np.array([0, 0, 8.0]))
    check(scene, [cam])
    check(scene, [cam], params=dict(tile_cull=0))
