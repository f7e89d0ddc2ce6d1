"""Helpers shared by the GPU parity tests: run the library through the binding and compare with
the oracle.  Nothing here computes the method; comparisons only."""
from __future__ import annotations

import numpy as np
import torch

from oracle import render as rd
from oracle import tiles as tl


def rtol_check(gpu, ref, rtol=1e-4, atol=1e-5, mask=None):
    """|gpu - ref| <= atol + rtol |ref| elementwise over rows selected by `mask`."""
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    if mask is not None:
        gpu, ref = gpu[mask], ref[mask]
    bad = np.abs(gpu - ref) > atol + rtol * np.abs(ref)
    return bad


def gpu_outputs(sp, k=0):
    """numpy outputs of sensor k of a SensorPass."""
    o = sp.outputs()
    rs, fs, C = sp.sensor_slices(k)
    F = o["feat"][fs].reshape(-1, C).cpu().numpy() if C > 0 else np.zeros((rs.stop - rs.start, 0))
    res = dict(F=F, D=o["depth"][rs].cpu().numpy(), A=o["alpha"][rs].cpu().numpy(),
               T=o["t_final"][rs].cpu().numpy(), last=o["last"][rs].cpu().numpy())
    if o["median"] is not None:
        res["median"] = o["median"][rs].cpu().numpy()
    return res


def tile_lists_gpu(sp):
    """Per-tile Gaussian id lists produced by the library."""
    tr = sp.tile_range.cpu().numpy()[:sp.n_tiles]
    ga = sp.gauss.cpu().numpy()
    return [ga[a:b].tolist() for a, b in tr]


def camera_ray_tiles(cam, pixel_idx):
    row = pixel_idx // cam.width
    col = pixel_idx % cam.width
    tx = -(-cam.width // cam.tile_w)
    return (row // cam.tile_h) * tx + col // cam.tile_w


def last_ids_gpu(sp, k, sensor, ray_idx, last):
    """Map the library's per-ray `last` (1 + list position) to a Gaussian id (-1: none)."""
    lists = tile_lists_gpu(sp)
    base = int(sp.rig.tile_base[sp.first + k] - sp.rig.tile_base[sp.first])
    if hasattr(sensor, "ray_az"):
        a, e, v = tl.lidar_ray_tiles_f32(sensor.ray_az[ray_idx], sensor.ray_el[ray_idx], sensor)
        tiles = np.where(v, e * sensor.n_az_tiles + a, -1)
    else:
        tiles = camera_ray_tiles(sensor, np.asarray(ray_idx))
    out = np.full(len(ray_idx), -1, np.int64)
    for i, (t, l) in enumerate(zip(tiles, last)):
        if t >= 0 and l > 0:
            out[i] = lists[base + t][l - 1]
    return out


def grad_mismatch(got, ref, rtol=1e-3, afloor=1e-5):
    """Elements outside the per-element gradient bar |g - g_ref| <= rtol |g_ref| + afloor max|g_ref|."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    return np.abs(got - ref) > rtol * np.abs(ref) + afloor * np.abs(ref).max(initial=0.0)


def assert_grad_close(got, ref, what, rtol=1e-3, norm_tol=1e-3, afloor=1e-5, require_nonzero=True,
                      per_element=True):
    """The gradient bar of the parity tests: ||g - g_ref|| <= norm_tol ||g_ref|| for the array,
    and |g - g_ref| <= rtol |g_ref| + afloor max|g_ref| for every element (unless per_element is
    False: the caller checks the elements itself).  On failure the message names the worst
    elements (flat index, GPU value, reference value)."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    nrm = float(np.linalg.norm(ref))
    if require_nonzero:
        assert nrm > 0, f"{what}: reference gradient is zero"
    rel = float(np.linalg.norm(got - ref)) / max(nrm, 1e-300)
    bad = grad_mismatch(got, ref, rtol, afloor) if per_element else np.zeros(got.shape, bool)
    if rel <= norm_tol and not bad.any():
        return
    err = (np.abs(got - ref) / (rtol * np.abs(ref) + afloor * np.abs(ref).max(initial=0.0) + 1e-300)).reshape(-1)
    worst = np.argsort(-err)[:8]
    rows = ", ".join(f"[{int(i)}] gpu {got.reshape(-1)[i]:.6g} ref {ref.reshape(-1)[i]:.6g}" for i in worst)
    raise AssertionError(f"{what}: relative norm error {rel:.3g}, {int(bad.sum())} of {bad.size} elements "
                         f"outside the bar; worst: {rows}")
