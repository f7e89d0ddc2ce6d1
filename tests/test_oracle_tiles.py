"""Pins of the oracle's tile arithmetic: hand-worked wrap examples of App. A (golden fixture),
brute force over dense sample points on tiny grids (every covered sample lands in a listed tile,
every listed tile touches the box), and the FP32 stage emulation agreeing with FP64 away from
tile borders."""
import json
import math
import os

import numpy as np
import pytest

from oracle import tiles as tl
from scenes import synthetic as S

HERE = os.path.dirname(os.path.abspath(__file__))


def _lid(n_az, tile_az=32, n_beams=16, tile_el=4):
    return S.make_lidar((0, 0, 0), 0.0, n_beams, -15.0, 15.0, n_az, tile_az=tile_az, tile_el=tile_el,
                        rolling_shutter=False)


def _az_tiles(start, n, M):
    return sorted({(int(start) + k) % M for k in range(int(n))})


def test_lidar_wrap_golden():
    gold = json.load(open(os.path.join(HERE, "golden", "lidar_azimuth_wrap.json")))
    lid = _lid(gold["n_az"], gold["tile_az"])
    assert lid.n_az_tiles == 57
    for case in gold["cases"]:
        lo_d, hi_d = case["box_deg"]
        lo = np.array([[math.radians(lo_d), 0.0]])
        hi = np.array([[math.radians(hi_d), 0.01]])
        for fn in (tl.lidar_tile_rect, tl.lidar_tile_rect_f32):
            start, n, e0, e1 = fn(lo, hi, lid)
            got = _az_tiles(start[0], n[0], 57)
            want = list(range(57)) if case["tiles"] == "all" else sorted(case["tiles"])
            assert got == want, (case, fn.__name__)


def test_camera_tiles_brute_force():
    rng = np.random.default_rng(0)
    for (W, H, tw, th) in [(37, 29, 8, 8), (64, 40, 16, 16), (50, 33, 16, 8), (41, 17, 4, 8)]:
        cam = S.make_camera((0, 0, 0), 0.0, W, H, 50.0, tile=(tw, th))
        tx = -(-W // tw)
        n = 400
        c = rng.uniform(-10, max(W, H) + 10, size=(n, 2))
        e = rng.exponential(6.0, size=(n, 2))
        lo, hi = c - e, c + e
        # snap some edges exactly onto tile borders and pixel centres
        lo[::7, 0] = np.round(lo[::7, 0] / tw) * tw
        hi[::5, 1] = np.round(hi[::5, 1] / th) * th
        hi[::9, 0] = np.floor(hi[::9, 0]) + 0.5
        x0, x1, y0, y1 = tl.camera_tile_rect(lo, hi, cam)
        cols = np.arange(W) + 0.5
        rows = np.arange(H) + 0.5
        for i in range(n):
            listed = {(a, b) for b in range(y0[i], y1[i]) for a in range(x0[i], x1[i])}
            inx = (cols >= lo[i, 0]) & (cols < hi[i, 0])
            iny = (rows >= lo[i, 1]) & (rows < hi[i, 1])
            need = {(int(cx // tw), int(cy // th)) for cx in np.arange(W)[inx] for cy in np.arange(H)[iny]}
            assert need <= listed
            for (a, b) in listed:   # every listed tile touches the closed box
                assert a * tw <= hi[i, 0] and (a + 1) * tw >= lo[i, 0]
                assert b * th <= hi[i, 1] and (b + 1) * th >= lo[i, 1]
                assert 0 <= a < tx


def test_lidar_tiles_brute_force():
    rng = np.random.default_rng(1)
    for n_az, tile_az in [(1800, 32), (1024, 32), (360, 8), (100, 16)]:
        lid = _lid(n_az, tile_az)
        M = lid.n_az_tiles
        w = tile_az * 2 * math.pi / n_az
        b = lid.elev_bounds.astype(np.float64)
        n = 300
        c = np.stack([rng.uniform(0, 2 * math.pi, n), rng.uniform(b[0] - 0.1, b[-1] + 0.1, n)], 1)
        e = np.stack([rng.exponential(0.4, n), rng.exponential(0.05, n)], 1)
        e[::11, 0] = rng.uniform(3.0, 8.0, size=e[::11, 0].shape)       # wider than a turn
        lo, hi = c - e, c + e
        start, nz, e0, e1 = tl.lidar_tile_rect(lo, hi, lid)
        az_s = np.linspace(0, 2 * math.pi, 4001)[:-1] + 1e-7
        el_s = np.linspace(b[0], b[-1], 501)[:-1] + 1e-9
        for i in range(n):
            listed_az = set(_az_tiles(start[i], nz[i], M))
            inside = np.mod(az_s - lo[i, 0], 2 * math.pi) < (hi[i, 0] - lo[i, 0])
            need_az = {int(a // w) % M for a in az_s[inside]}
            assert need_az <= listed_az
            for a in listed_az:     # listed tiles touch the (modular) box
                t0, t1 = a * w, (a + 1) * w
                touches = any(lo[i, 0] - 1e-12 <= t1 + k * 2 * math.pi and hi[i, 0] + 1e-12 >= t0 + k * 2 * math.pi
                              for k in range(-3, 4))
                assert touches
            ine = (el_s >= lo[i, 1]) & (el_s < hi[i, 1])
            need_el = {int(np.searchsorted(b, x, side="right") - 1) for x in el_s[ine]}
            listed_el = set(range(e0[i], e1[i]))
            assert need_el <= listed_el
            for k in listed_el:
                assert b[k] <= hi[i, 1] and b[k + 1] >= lo[i, 1]


def test_fp32_stage_formula_agrees_away_from_borders():
    rng = np.random.default_rng(2)
    lid = _lid(2048, 32)
    n = 2000
    c = np.stack([rng.uniform(0, 2 * math.pi, n), rng.uniform(-0.2, 0.2, n)], 1)
    e = np.stack([rng.exponential(0.3, n), rng.exponential(0.03, n)], 1)
    lo = (c - e).astype(np.float32)
    hi = (c + e).astype(np.float32)
    a = tl.lidar_tile_rect(lo.astype(np.float64), hi.astype(np.float64), lid)
    f = tl.lidar_tile_rect_f32(lo, hi, lid)
    w = 32 * 2 * math.pi / 2048
    def near_border(x):
        x = np.where(x < 0, x + 2 * math.pi, np.where(x > 2 * math.pi, x - 2 * math.pi, x))
        r = x / w
        return np.abs(r - np.round(r)) < 1e-4
    ok = ~(near_border(lo[:, 0].astype(np.float64)) | near_border(hi[:, 0].astype(np.float64)))
    for u, v in zip(a, f):
        np.testing.assert_array_equal(u[ok], v[ok])
    cam = S.make_camera((0, 0, 0), 0.0, 1920, 1080, 1500.0)
    c = rng.uniform(-100, 2000, size=(n, 2))
    e = rng.exponential(30.0, size=(n, 2))
    lo = (c - e).astype(np.float32)
    hi = (c + e).astype(np.float32)
    for u, v in zip(tl.camera_tile_rect(lo, hi, cam), tl.camera_tile_rect_f32(lo, hi, cam)):
        np.testing.assert_array_equal(u, v)     # power-of-two tiles: exact in both


def test_ray_tiles_and_lists():
    lid = _lid(360, 8)
    a, e, valid = tl.lidar_ray_tiles(lid.ray_az, lid.ray_el, lid)
    assert valid.all()
    # 16 beams, 4 per tile: beam k is in elevation tile k // 4; azimuth step j in tile j // 8
    beams = np.repeat(np.arange(16), 360)
    steps = np.tile(np.arange(360), 16)
    np.testing.assert_array_equal(e, beams // 4)
    np.testing.assert_array_equal(a, steps // 8)
    a32, e32, v32 = tl.lidar_ray_tiles_f32(lid.ray_az, lid.ray_el, lid)
    np.testing.assert_array_equal(a, a32)
    np.testing.assert_array_equal(e, e32)
    # per-tile lists are ordered by (depth, id) with ties broken by id
    depth = np.array([3.0, 1.0, 3.0, 2.0])
    per = [[0, 1], [1], [0, 1], [1]]
    lists = tl.tile_lists(per, depth, np.array([True, True, True, False]), 2)
    assert lists == [[0, 2], [1, 0, 2]]
