"""Tile-shape autotuner.

Under the BOX candidate rule the rendered outputs do not depend on the tile shape (tiling only
accelerates the per-ray candidate search), so the shape is free to be chosen for speed.  For
each sensor this times one batched forward + backward step (project, bin/sort, persistent
forward and adjoint) of that sensor alone over the caller's Gaussians for every candidate shape
and keeps the fastest.

The caller's own layout is kept unless a candidate is more than KEEP_MARGIN faster.

Candidates:
  camera -- tiles of 256 pixels (one lane per pixel of a 256-lane workgroup): 16x16, 32x8, 8x32,
            64x4;
  lidar  -- azimuth widths tile_az / 2, tile_az, 2 tile_az, each with the given elevation tiles
            and with pairs of them merged (the elevation boundaries are the caller's, so tiles
            can be merged but not split).

This is a setup-time search: it allocates, synchronises the device and takes seconds.  Each
candidate is timed as the median of REPEATS runs of STEPS steps.  Results are kept in a JSON
file (autotune_cache.json beside this module, or the path in SPLAT_AUTOTUNE_CACHE), keyed by
the GPU architecture, the sensor class and shape (resolution / beams x azimuth steps, tile
layout, channel count) and the Gaussian count rounded to a power of two, so that later runs
take the stored layout without searching.
"""
from __future__ import annotations

import copy
import json
import math
import os
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import binding as B

CAMERA_TILES = [(16, 16), (32, 8), (8, 32), (64, 4)]
KEEP_MARGIN = 0.03   # another layout must be this much faster to replace the caller's
STEPS = 8            # steps per timing run of a candidate
REPEATS = 3          # timing runs per candidate (the median is kept)
CACHE_PATH = os.environ.get("SPLAT_AUTOTUNE_CACHE",
                            os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_cache.json"))

_cache: Dict[str, list] = {}
_loaded = False


def _arch() -> str:
    try:
        return torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]
    except Exception:   # no device: only the key's arch field is affected
        return "unknown"


def _load_cache():
    global _loaded
    if _loaded:
        return
    _loaded = True
    try:
        with open(CACHE_PATH) as f:
            data = json.load(f)
        if isinstance(data, dict):
            _cache.update({k: v for k, v in data.items() if isinstance(v, list)})
    except (OSError, ValueError):
        pass


def _store_cache():
    try:
        tmp = CACHE_PATH + ".tmp"
        with open(tmp, "w") as f:
            json.dump(dict(sorted(_cache.items())), f, indent=1)
        os.replace(tmp, CACHE_PATH)
    except OSError:   # a read-only tree keeps the results for this process only
        pass


def _key(parts) -> str:
    return "|".join(str(p) for p in (_arch(),) + tuple(parts))


def _camera_key(cam, n):
    return _key(("camera", f"{int(cam.width)}x{int(cam.height)}", f"tile{int(cam.tile_w)}x{int(cam.tile_h)}",
                 f"c{int(cam.n_channels)}", f"n{1 << max(0, int(n - 1).bit_length())}"))


def _lidar_key(lid, n):
    return _key(("lidar", f"rays{int(lid.n_rays)}", f"az{int(lid.tile_az)}x{int(lid.n_az_tiles)}",
                 f"el{len(lid.elev_bounds) - 1}", f"c{int(lid.n_channels)}",
                 f"n{1 << max(0, int(n - 1).bit_length())}"))


def camera_candidates(cam) -> List:
    out = []
    for tw, th in CAMERA_TILES:
        c = copy.copy(cam)
        c.tile_w, c.tile_h = tw, th
        out.append(c)
    return out


def _merge_bounds(b: np.ndarray, f: int) -> np.ndarray:
    idx = list(range(0, len(b) - 1, f)) + [len(b) - 1]
    return np.ascontiguousarray(b[idx], dtype=np.float32)


def lidar_candidates(lid) -> List:
    n_az = int(round(2.0 * math.pi / float(lid.az_res)))
    out = []
    for taz in sorted({max(4, int(lid.tile_az) // 2), int(lid.tile_az), 2 * int(lid.tile_az)}):
        for f in (1, 2):
            if f > 1 and len(lid.elev_bounds) <= 2:
                continue
            c = copy.copy(lid)
            c.tile_az = taz
            c.n_az_tiles = (n_az + taz - 1) // taz
            c.elev_bounds = _merge_bounds(np.asarray(lid.elev_bounds, np.float32), f)
            if hasattr(c, "tile_el"):
                c.tile_el = int(lid.tile_el) * f
            out.append(c)
    return out


def _time_step(sensor, is_camera: bool, g: B.GaussTensors, steps: int, warmup: int) -> float:
    rig = B.Rig([sensor], []) if is_camera else B.Rig([], [sensor])
    sp = B.SensorPass(rig, 0, 1, g.n, 1, batched=True)
    sp.fit_capacity(g, 1.15)
    up = np.random.default_rng(0)
    dF = torch.from_numpy(up.normal(size=max(1, sp.n_feat)).astype(np.float32)).cuda()
    dD = torch.from_numpy((0.1 * up.normal(size=sp.n_rays)).astype(np.float32)).cuda()
    dA = torch.from_numpy(up.normal(size=sp.n_rays).astype(np.float32)).cuda()
    grads = B.zeros_like_grads(g)
    pipe = B.Pipeline(sp, g, B.BOX, grads, dF, dD, dA)
    for _ in range(warmup):
        pipe.run()
    torch.cuda.synchronize()
    st = B.read_status(sp.status)
    if st.overflow:
        raise B.SplatError(f"autotune: intersection overflow ({st.n_isect} > {st.k_cap})")
    s = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    runs = []
    for _ in range(REPEATS):
        a.record(s)
        for _ in range(steps):
            pipe.run()
        b.record(s)
        torch.cuda.synchronize()
        runs.append(a.elapsed_time(b) / steps)
    pipe.close()
    return float(np.median(runs))


def tune_sensor(sensor, is_camera: bool, g: B.GaussTensors, steps: int = STEPS, warmup: int = 2,
                log=None) -> Tuple[object, List[Tuple[tuple, float]]]:
    """Fastest tile layout for one sensor; returns (sensor copy with that layout, timings; empty
    when the layout came from the cache)."""
    _load_cache()
    key = _camera_key(sensor, g.n) if is_camera else _lidar_key(sensor, g.n)
    cands = camera_candidates(sensor) if is_camera else lidar_candidates(sensor)
    if key in _cache:
        shape = tuple(_cache[key])
        for c in cands:
            if _shape(c, is_camera) == shape:
                return c, []
    timings = []
    best, best_ms = None, float("inf")
    for c in cands:
        ms = _time_step(c, is_camera, g, steps, warmup)
        timings.append((_shape(c, is_camera), ms))
        if log:
            log(f"autotune {'camera' if is_camera else 'lidar'} {_shape(c, is_camera)}: {ms:.3f} ms")
        if ms < best_ms:
            best, best_ms = c, ms
    # keep the caller's layout unless another is clearly faster (timing noise is a few percent)
    mine = _shape(sensor, is_camera)
    for c, (sh, ms) in zip(cands, timings):
        if sh == mine and ms <= best_ms * (1.0 + KEEP_MARGIN):
            best = c
    _cache[key] = list(_shape(best, is_camera))
    _store_cache()
    return best, timings


def _shape(s, is_camera: bool) -> tuple:
    if is_camera:
        return (int(s.tile_w), int(s.tile_h))
    return (int(s.tile_az), len(s.elev_bounds) - 1)


def tune_rig(cameras: Sequence, lidars: Sequence, g: B.GaussTensors, steps: int = STEPS, warmup: int = 2,
             log=None) -> Tuple[list, list, dict]:
    """Tile layouts for every sensor of a rig (each tuned alone).  Returns new camera and lidar
    lists and a report {sensor index: (chosen shape, [(shape, ms), ...])}."""
    report = {}
    cams, lids = [], []
    for i, c in enumerate(cameras):
        best, t = tune_sensor(c, True, g, steps, warmup, log)
        cams.append(best)
        report[i] = (_shape(best, True), t)
    for j, l in enumerate(lidars):
        best, t = tune_sensor(l, False, g, steps, warmup, log)
        lids.append(best)
        report[len(cameras) + j] = (_shape(best, False), t)
    return cams, lids, report
