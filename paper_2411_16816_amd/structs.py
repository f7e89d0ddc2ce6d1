"""ctypes mirrors of the structs declared in include/splat.h, and converters from the scene
containers (scenes.synthetic.Camera / Lidar).  Argument marshalling only."""
from __future__ import annotations

import ctypes as C

import numpy as np

SPLAT_MAX_EL_TILES = 64
SPLAT_MAX_SENSORS = 1024
SUPPORT_BOX = 0
SUPPORT_TILE = 1


class SplatStatus(C.Structure):
    _fields_ = [("n_isect", C.c_ulonglong), ("k_cap", C.c_ulonglong), ("overflow", C.c_uint),
                ("n_nonfinite", C.c_uint), ("n_rays_invalid", C.c_uint), ("n_rays_time", C.c_uint),
                ("n_pairs", C.c_ulonglong), ("n_stopped", C.c_ulonglong)]


class SplatGaussians(C.Structure):
    _fields_ = [("n", C.c_int64), ("means", C.c_void_p), ("log_scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacities", C.c_void_p), ("velocities", C.c_void_p), ("features", C.c_void_p),
                ("c_total", C.c_int32)]


class SplatCamera(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("t", C.c_float * 3), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("width", C.c_int32), ("height", C.c_int32),
                ("lin_vel", C.c_float * 3), ("ang_vel", C.c_float * 3), ("t_rs", C.c_float),
                ("eps2d", C.c_float), ("near_plane", C.c_float), ("far_plane", C.c_float),
                ("jac_clamp", C.c_float), ("feat_offset", C.c_int32), ("n_channels", C.c_int32),
                ("tile_w", C.c_int32), ("tile_h", C.c_int32), ("time_offset", C.c_float)]


class SplatLidar(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("t", C.c_float * 3), ("lin_vel", C.c_float * 3),
                ("ang_vel", C.c_float * 3), ("t_rs", C.c_float), ("eps2d", C.c_float), ("r_min", C.c_float),
                ("r_max", C.c_float), ("az_res", C.c_float), ("tile_az", C.c_int32),
                ("n_az_tiles", C.c_int32), ("n_el_tiles", C.c_int32), ("elev_bounds", C.c_void_p),
                ("n_rays", C.c_int64), ("ray_az", C.c_void_p), ("ray_el", C.c_void_p), ("ray_t", C.c_void_p),
                ("feat_offset", C.c_int32), ("n_channels", C.c_int32), ("ray_range", C.c_void_p),
                ("los_eps", C.c_float), ("ray_priority", C.c_void_p)]


class SplatRigLayout(C.Structure):
    _fields_ = [("n_sensors", C.c_int32), ("n_cameras", C.c_int32),
                ("tile_base", C.c_int64 * (SPLAT_MAX_SENSORS + 1)),
                ("ray_base", C.c_int64 * (SPLAT_MAX_SENSORS + 1)),
                ("feat_base", C.c_int64 * (SPLAT_MAX_SENSORS + 1))]


class SplatProjected(C.Structure):
    _fields_ = [("n_records", C.c_int64), ("mv", C.c_void_p), ("cn", C.c_void_p), ("box", C.c_void_p),
                ("dv", C.c_void_p), ("dkey", C.c_void_p), ("rect", C.c_void_p), ("n_tiles", C.c_void_p)]


class SplatTileLists(C.Structure):
    _fields_ = [("k_cap", C.c_int64), ("gauss", C.c_void_p), ("tile_range", C.c_void_p),
                ("entry_base", C.c_void_p), ("ray_order", C.c_void_p), ("ray_range", C.c_void_p), ("work", C.c_void_p),
                ("n_work", C.c_void_p), ("work_cap", C.c_int64)]


class SplatRenderOut(C.Structure):
    _fields_ = [("feat", C.c_void_p), ("depth", C.c_void_p), ("alpha", C.c_void_p), ("t_final", C.c_void_p),
                ("last", C.c_void_p), ("median", C.c_void_p), ("sensor_done", C.c_void_p), ("los", C.c_void_p),
                ("d_los", C.c_void_p), ("dropped", C.c_void_p)]


class SplatGrads(C.Structure):
    _fields_ = [("means", C.c_void_p), ("log_scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacities", C.c_void_p), ("velocities", C.c_void_p), ("features", C.c_void_p),
                ("sensor_lin_vel", C.c_void_p), ("sensor_ang_vel", C.c_void_p), ("sensor_time_offset", C.c_void_p)]


def _arr(ctype, n, values):
    a = ctype * n
    return a(*[float(v) for v in np.asarray(values, np.float64).reshape(-1)])


def camera_struct(cam) -> SplatCamera:
    s = SplatCamera()
    s.R = _arr(C.c_float, 9, cam.R)
    s.t = _arr(C.c_float, 3, cam.t)
    s.fx, s.fy, s.cx, s.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    s.width, s.height = int(cam.width), int(cam.height)
    s.lin_vel = _arr(C.c_float, 3, cam.lin_vel)
    s.ang_vel = _arr(C.c_float, 3, cam.ang_vel)
    s.t_rs, s.eps2d = float(cam.t_rs), float(cam.eps2d)
    s.near_plane, s.far_plane, s.jac_clamp = float(cam.near), float(cam.far), float(cam.jac_clamp)
    s.feat_offset, s.n_channels = int(cam.feat_offset), int(cam.n_channels)
    s.tile_w, s.tile_h = int(cam.tile_w), int(cam.tile_h)
    s.time_offset = float(getattr(cam, "time_offset", 0.0))
    return s


def lidar_struct(lid, ray_ptrs=(None, None, None), bounds_keepalive=None) -> SplatLidar:
    """`ray_ptrs` are device pointers (ints) of the azimuth, elevation and time arrays, optionally
    followed by the measured ranges; or a dict with keys az, el, t and optionally range and
    priority (the training-time cap)."""
    s = SplatLidar()
    s.R = _arr(C.c_float, 9, lid.R)
    s.t = _arr(C.c_float, 3, lid.t)
    s.lin_vel = _arr(C.c_float, 3, lid.lin_vel)
    s.ang_vel = _arr(C.c_float, 3, lid.ang_vel)
    s.t_rs, s.eps2d = float(lid.t_rs), float(lid.eps2d)
    s.r_min, s.r_max, s.az_res = float(lid.r_min), float(lid.r_max), float(lid.az_res)
    s.tile_az, s.n_az_tiles, s.n_el_tiles = int(lid.tile_az), int(lid.n_az_tiles), int(lid.n_el_tiles)
    b = np.ascontiguousarray(lid.elev_bounds, dtype=np.float32)
    if bounds_keepalive is not None:
        bounds_keepalive.append(b)
    s.elev_bounds = b.ctypes.data
    s.n_rays = int(lid.n_rays)
    if isinstance(ray_ptrs, dict):
        s.ray_az, s.ray_el, s.ray_t = ray_ptrs["az"], ray_ptrs["el"], ray_ptrs["t"]
        s.ray_range, s.ray_priority = ray_ptrs.get("range"), ray_ptrs.get("priority")
    else:
        s.ray_az, s.ray_el, s.ray_t = ray_ptrs[:3]
        s.ray_range = ray_ptrs[3] if len(ray_ptrs) > 3 else None
    s.feat_offset, s.n_channels = int(lid.feat_offset), int(lid.n_channels)
    s.los_eps = float(getattr(lid, "los_eps", 0.8))
    return s


SPLAT_STEP_BACKWARD = 1
SPLAT_STEP_ZERO_GRADS = 2
SPLAT_STEP_COUNT_PAIRS = 4


class SplatStep(C.Structure):
    _fields_ = [("gaussians", SplatGaussians), ("proj", SplatProjected), ("lists", SplatTileLists),
                ("out", SplatRenderOut), ("support", C.c_int32), ("flags", C.c_int32),
                ("d_feat", C.c_void_p), ("d_depth", C.c_void_p), ("d_alpha", C.c_void_p),
                ("grads", SplatGrads), ("ws", C.c_void_p), ("ws_bytes", C.c_size_t), ("status", C.c_void_p)]


class SplatActors(C.Structure):
    _fields_ = [("n", C.c_int32), ("rot", C.c_void_p), ("trans", C.c_void_p), ("rot_offset", C.c_void_p),
                ("trans_offset", C.c_void_p), ("lin_vel", C.c_void_p), ("lin_vel_offset", C.c_void_p),
                ("ang_vel", C.c_void_p)]


class SplatActorGrads(C.Structure):
    _fields_ = [("rot_offset", C.c_void_p), ("trans_offset", C.c_void_p), ("lin_vel_offset", C.c_void_p),
                ("ang_vel", C.c_void_p)]


class SplatLidarMLP(C.Structure):
    _fields_ = [("n_feat", C.c_int32), ("w1", C.c_void_p), ("b1", C.c_void_p), ("w2", C.c_void_p), ("b2", C.c_void_p)]


class SplatLidarMLPGrads(C.Structure):
    _fields_ = [("w1", C.c_void_p), ("b1", C.c_void_p), ("w2", C.c_void_p), ("b2", C.c_void_p)]


class SplatCameraCNN(C.Structure):
    _fields_ = [("n_feat", C.c_int32), ("n_embed", C.c_int32), ("embed", C.c_void_p), ("w_in", C.c_void_p),
                ("b_in", C.c_void_p), ("w_block", C.c_void_p * 4), ("b_block", C.c_void_p * 4), ("w_out", C.c_void_p),
                ("b_out", C.c_void_p)]


class SplatCameraCNNGrads(C.Structure):
    _fields_ = [("embed", C.c_void_p), ("w_in", C.c_void_p), ("b_in", C.c_void_p), ("w_block", C.c_void_p * 4),
                ("b_block", C.c_void_p * 4), ("w_out", C.c_void_p), ("b_out", C.c_void_p)]


class SplatGaussianState(C.Structure):
    _fields_ = [("n", C.c_int64), ("means", C.c_void_p), ("log_scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacities", C.c_void_p), ("velocities", C.c_void_p), ("features", C.c_void_p), ("c_total", C.c_int32)]
