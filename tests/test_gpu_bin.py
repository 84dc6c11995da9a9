"""gut_bin against a plain sort of its own inputs, bit for bit.

Binning is integer work: given the projected rectangles, tiles-touched counts
and FP32 depths, the tile lists are fixed exactly -- every (tile, entry) pair
the rectangles define, ordered by (global tile id, depth bits, entry id)
(the per-tile depth order of Sec. 4.3 with the id tie-break).  This test
expands the pairs with numpy from the same projection outputs the kernels
read, sorts them with np.lexsort, and requires identical sorted ids, ranges
and pair count, at the full benchmark sizes and at tile counts that take
one, two and three radix passes over the tile bits.
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


def expected_bins(proj, cams, n):
    """Pairs of the projected rectangles in (tile, depth bits, entry) order."""
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
    cam = e_rep // n
    tile = np.asarray(base)[cam] + (np.repeat(r[:, 1], cnt) + y) * np.asarray(tx)[cam] + \
        np.repeat(r[:, 0], cnt) + x
    order = np.lexsort((e_rep, dbits[e_rep], tile))
    ids = e_rep[order]
    st = tile[order]
    first = np.searchsorted(st, np.arange(T), side="left")
    last = np.searchsorted(st, np.arange(T), side="right")
    ranges = np.stack([np.where(last > first, first, 0), np.where(last > first, last, 0)], axis=1)
    return P, ids, ranges, T


def check(scene, cams, capacity=None):
    gs = R.GaussianScene.from_host(scene)
    proj = R.project(gs, cams)
    bins = R.bin_tiles(proj, cams, capacity=capacity)
    torch.cuda.synchronize()
    P, ids, ranges, T = expected_bins(proj, cams, gs.n)
    say(f"  n={gs.n} cams={len(cams)} T={T} P={P} gpu_P={bins.n_pairs}")
    assert bins.n_pairs == P
    got_ids = bins.ids[:P].cpu().numpy().astype(np.int64)
    got_ranges = bins.ranges.cpu().numpy().astype(np.int64)
    assert got_ranges.shape == (T, 2)
    bad = np.nonzero(got_ids != ids)[0]
    assert bad.size == 0, f"{bad.size} ids differ, first at {bad[:5]}"
    badr = np.nonzero((got_ranges != ranges).any(axis=1))[0]
    assert badr.size == 0, f"{badr.size} ranges differ, first tiles {badr[:5]}"
    return bins


def test_bin_exact_c1_single_pass():
    say("[bin exact] c1, 64 tiles: one tile pass")
    scene, cams = G.config1()
    check(scene, cams[:1])


def test_bin_exact_c2_full():
    say("[bin exact] 1M Gaussians, pinhole + fisheye 1920x1080: two tile passes")
    check(G.config2_scene(), G.config2_cameras())


def test_bin_exact_c3_full():
    say("[bin exact] 3M Gaussians, rolling-shutter fisheye 1600x1200")
    check(G.config3_scene(), [G.config3_camera()])


def test_bin_exact_three_tile_passes():
    say("[bin exact] nine 1920x1080 views (73440 tiles, 17 bits): three tile passes")
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
    cam = dict(cams[0])
    cam = G.camera("pinhole", 64, 48, 60.0, R0=np.eye(3), t0=np.array([0.0, 0.0, -10.0]))
    bins = check(scene, [cam])
    assert bins.n_pairs == 0
    assert (bins.ranges.cpu().numpy() == 0).all()


def test_bin_exact_8k_camera_gathered_rectangles():
    say("[bin exact] one 7680x4320 view (480x270 tiles): rectangles gathered, not packed")
    scene = G.clustered_scene(40000, seed=1002)
    cam = G.camera("pinhole", 7680, 4320, G.pinhole_focal(7680), R0=np.eye(3), t0=np.array([0, 0, 8.0]))
    check(scene, [cam])
