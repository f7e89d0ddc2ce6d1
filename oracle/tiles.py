"""Oracle, step 8: tile ranges, ray tiles and per-tile depth-ordered lists.

Plain NumPy.  Test infrastructure only.

Camera (Sec. 3.2): tiles of tile_w x tile_h pixels; a Gaussian is duplicated into every tile
its rectangular box touches.  Lower tile bound floor(lo / T) (inclusive), upper bound
floor(hi / T) + 1 (exclusive), clamped to the grid.

Lidar (App. A, lidar tiling): N_phi azimuth steps by N_omega channels per tile.
  * azimuth: the piecewise Phi_low / Phi_high of App. A.  Reading: the upper bound uses
    floor(.) + 1 rather than ceil(.), so a box whose upper edge lies exactly on a tile border
    still reaches every ray it contains; the span is clamped to M_phi tiles and the start is
    wrapped into [0, M_phi).
  * elevation: Omega_low = the last boundary <= the lower edge (clamped to >= 0) and
    Omega_high = (the last boundary <= the upper edge) + 1 (clamped to <= M_omega); this is
    our reading of the garbled sentence at the end of App. A's tiling paragraph.

Training-time cap (App. A): `lidar_training_dropped` picks the rays a crowded tile drops, from
per-ray priorities (the shuffle, an input); pinned by a worked example and by invariants (kept
count per tile, priorities on either side of the cut, ties by ray index).

`*_f32` functions evaluate the same ranges in IEEE float32 in the exact order the GPU library
documents (include/splat.h), from the library's own float32 boxes: they are the bit-exact stage
check, not an independent derivation.  The FP64 functions follow the paper's formulas and are
pinned by brute force on tiny grids and by hand-worked wrap examples (tests).
"""
from __future__ import annotations

import math

import numpy as np

TWO_PI = 2.0 * math.pi


# --------------------------------------------------------------------------------------
# FP64, paper formulas
# --------------------------------------------------------------------------------------
def camera_tile_rect(lo, hi, cam):
    """[N,2] boxes -> (x0, x1, y0, y1) int64 arrays (half-open)."""
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    tx = -(-cam.width // cam.tile_w)
    ty = -(-cam.height // cam.tile_h)
    x0 = np.clip(np.floor(lo[:, 0] / cam.tile_w), 0, tx).astype(np.int64)
    x1 = np.clip(np.floor(hi[:, 0] / cam.tile_w) + 1, 0, tx).astype(np.int64)
    y0 = np.clip(np.floor(lo[:, 1] / cam.tile_h), 0, ty).astype(np.int64)
    y1 = np.clip(np.floor(hi[:, 1] / cam.tile_h) + 1, 0, ty).astype(np.int64)
    return x0, x1, y0, y1


def lidar_tile_rect(lo, hi, lid):
    """App. A.  Returns (az_start in [0, M_phi), n_az, el0, el1) int64 arrays."""
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    M = lid.n_az_tiles
    w = lid.tile_az * float(lid.az_res)           # tile azimuth size
    phi_max = M * w
    lo_a, hi_a = lo[:, 0], hi[:, 0]
    low = np.where(lo_a >= 0, np.floor(lo_a / w), np.floor((lo_a + TWO_PI - phi_max) / w))
    high = np.where(hi_a <= TWO_PI, np.floor(hi_a / w) + 1,
                    np.floor(np.mod(hi_a, TWO_PI) / w) + 1 + M)
    n_az = high - low
    full = n_az >= M
    start = np.where(full, 0, np.mod(low, M))
    n_az = np.where(full, M, np.maximum(n_az, 0))
    b = np.asarray(lid.elev_bounds, np.float64)
    Mw = b.shape[0] - 1
    el0 = np.clip(np.searchsorted(b, lo[:, 1], side="right") - 1, 0, Mw)
    el1 = np.clip(np.searchsorted(b, hi[:, 1], side="right"), 0, Mw)
    return start.astype(np.int64), n_az.astype(np.int64), el0.astype(np.int64), el1.astype(np.int64)


def lidar_ray_tiles(ray_az, ray_el, lid):
    """Tile of each ray (App. A, lidar points to rasterisation points: a ray is a box of
    zero extent).  Returns (az_tile, el_tile, valid)."""
    az = np.asarray(ray_az, np.float64)
    el = np.asarray(ray_el, np.float64)
    w = lid.tile_az * float(lid.az_res)
    a = np.mod(np.floor(az / w), lid.n_az_tiles).astype(np.int64)
    b = np.asarray(lid.elev_bounds, np.float64)
    e = np.searchsorted(b, el, side="right") - 1
    valid = (el >= b[0]) & (el < b[-1]) & (az >= 0) & (az < TWO_PI)
    return a, np.clip(e, 0, b.shape[0] - 2), valid


# --------------------------------------------------------------------------------------
# FP32 stage check: the library's documented float32 evaluation of the same ranges
# --------------------------------------------------------------------------------------
F = np.float32
TWO_PI_F = F(TWO_PI)


def _fl_floor_div(x, w):
    with np.errstate(over="ignore", invalid="ignore"):
        return np.floor((x.astype(F) / F(w)).astype(F))


def camera_tile_rect_f32(lo, hi, cam):
    lo = np.asarray(lo, F)
    hi = np.asarray(hi, F)
    tx = -(-cam.width // cam.tile_w)
    ty = -(-cam.height // cam.tile_h)
    x0 = np.clip(_fl_floor_div(lo[:, 0], cam.tile_w), 0, tx).astype(np.int64)
    x1 = np.clip(_fl_floor_div(hi[:, 0], cam.tile_w) + 1, 0, tx).astype(np.int64)
    y0 = np.clip(_fl_floor_div(lo[:, 1], cam.tile_h), 0, ty).astype(np.int64)
    y1 = np.clip(_fl_floor_div(hi[:, 1], cam.tile_h) + 1, 0, ty).astype(np.int64)
    return x0, x1, y0, y1


def lidar_tile_width_f32(lid):
    return F(F(lid.tile_az) * F(lid.az_res))


def lidar_tile_rect_f32(lo, hi, lid):
    """Float32: w = fl(N_phi * res); for lo < 0 the lower index is
    floor(fl(lo + 2pi) / w) - M_phi (equal to the paper's floor((lo + 2pi - phi_max) / w) in
    exact arithmetic); for hi > 2pi the upper index is floor(fl(hi - 2pi) / w) + 1 + M_phi.
    Integer parts are clamped to [-2^24, 2^24] before conversion."""
    lo = np.asarray(lo, F)
    hi = np.asarray(hi, F)
    M = lid.n_az_tiles
    w = lidar_tile_width_f32(lid)
    lo_a, hi_a = lo[:, 0], hi[:, 0]
    with np.errstate(over="ignore", invalid="ignore"):
        lo_w = np.where(lo_a < 0, (lo_a + TWO_PI_F).astype(F), lo_a)
        hi_w = np.where(hi_a > TWO_PI_F, (hi_a - TWO_PI_F).astype(F), hi_a)
    lim = float(1 << 24)
    low = np.clip(_fl_floor_div(lo_w, w), -lim, lim).astype(np.int64) - np.where(lo_a < 0, M, 0)
    high = np.clip(_fl_floor_div(hi_w, w), -lim, lim).astype(np.int64) + 1 + np.where(hi_a > TWO_PI_F, M, 0)
    n_az = high - low
    full = n_az >= M
    start = np.where(full, 0, np.mod(low, M))
    n_az = np.where(full, M, np.maximum(n_az, 0))
    b = np.asarray(lid.elev_bounds, F)
    Mw = b.shape[0] - 1
    el0 = np.clip(np.searchsorted(b, lo[:, 1], side="right") - 1, 0, Mw)
    el1 = np.clip(np.searchsorted(b, hi[:, 1], side="right"), 0, Mw)
    return start.astype(np.int64), n_az.astype(np.int64), el0.astype(np.int64), el1.astype(np.int64)


def lidar_ray_tiles_f32(ray_az, ray_el, lid):
    az = np.asarray(ray_az, F)
    el = np.asarray(ray_el, F)
    w = lidar_tile_width_f32(lid)
    a = np.mod(_fl_floor_div(az, w).astype(np.int64), lid.n_az_tiles)
    b = np.asarray(lid.elev_bounds, F)
    e = np.searchsorted(b, el, side="right") - 1
    valid = (el >= b[0]) & (el < b[-1]) & (az >= 0) & (az < TWO_PI_F)
    return a, np.clip(e, 0, b.shape[0] - 2), valid


# --------------------------------------------------------------------------------------
# per-tile lists: every (tile, Gaussian) pair ordered by (tile, depth, Gaussian id)
# --------------------------------------------------------------------------------------
def camera_tiles_of(rect, cam):
    x0, x1, y0, y1 = rect
    tx = -(-cam.width // cam.tile_w)
    out = []
    for i in range(x0.shape[0]):
        ts = [ty_ * tx + tx_ for ty_ in range(y0[i], y1[i]) for tx_ in range(x0[i], x1[i])]
        out.append(ts)
    return out


def lidar_tiles_of(rect, lid):
    start, n_az, el0, el1 = rect
    M = lid.n_az_tiles
    out = []
    for i in range(start.shape[0]):
        ts = [e * M + (start[i] + k) % M for e in range(el0[i], el1[i]) for k in range(n_az[i])]
        out.append(ts)
    return out


def tile_lists(tiles_per_gaussian, depth, valid, n_tiles):
    """Dict-free list-of-lists: lists[t] = Gaussian ids covering tile t, ordered by
    (depth, id).  `depth` is compared as given (float32 bits order for positive floats equals
    numeric order)."""
    lists = [[] for _ in range(n_tiles)]
    order = np.lexsort((np.arange(depth.shape[0]), depth))
    for g in order:
        if not valid[g]:
            continue
        for t in tiles_per_gaussian[g]:
            lists[t].append(int(g))
    return lists


# --------------------------------------------------------------------------------------
# training-time cap on the rays of a lidar tile (App. A, lidar points to rasterisation points)
# --------------------------------------------------------------------------------------
def lidar_training_dropped(az_tile, el_tile, valid, priority, n_az_tiles, cap=256):
    """During training a tile that receives more than `cap` lidar rays renders a random `cap` of
    them (the paper shuffles the points each iteration and discards those beyond 256).  The
    shuffle is an input: one priority per ray; a tile keeps its `cap` rays of smallest
    (priority, ray index) and drops the rest.  Returns `dropped` [R] bool (False for rays
    outside every tile).  Plain per-tile loop."""
    priority = np.asarray(priority)
    tile = np.asarray(el_tile, np.int64) * int(n_az_tiles) + np.asarray(az_tile, np.int64)
    valid = np.asarray(valid, bool)
    dropped = np.zeros(len(priority), bool)
    for t in np.unique(tile[valid]):
        members = np.nonzero(valid & (tile == t))[0]
        order = sorted(members.tolist(), key=lambda r: (int(priority[r]), r))
        for r in order[cap:]:
            dropped[r] = True
    return dropped
