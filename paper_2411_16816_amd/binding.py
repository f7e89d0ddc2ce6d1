"""Thin ctypes binding of libsplat (include/splat.h).

Argument marshalling only: every step of projection, binning, sorting and compositing runs in
the library's HIP kernels.  PyTorch provides device memory and the stream.  Loading fails loudly
when the library has not been built; there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import structs as st

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsplat.so")

_lib = None

BOX = st.SUPPORT_BOX
TILE = st.SUPPORT_TILE
KIND_CAMERA = 0
KIND_LIDAR = 1

_P = C.c_void_p


def _declare(lib):
    vp = C.c_void_p
    i32, i64 = C.c_int32, C.c_int64
    sig = {
        "splat_status_string": (C.c_char_p, [C.c_int]),
        "splat_version": (C.c_int, []),
        "splat_check_camera": (C.c_int, [vp]),
        "splat_check_lidar": (C.c_int, [vp]),
        "splat_rig_create": (C.c_int, [i32, i32, C.POINTER(vp)]),
        "splat_rig_set": (C.c_int, [vp, vp, vp, vp]),
        "splat_rig_layout": (C.c_int, [vp, vp]),
        "splat_rig_destroy": (None, [vp]),
        "splat_workspace_bytes": (C.c_size_t, [vp, i32, i32, i64, i64]),
        "splat_set_adjoint_row_limit": (C.c_int, [i64]),
        "splat_project_camera": (C.c_int, [vp, vp, i32, i32, vp, vp, vp]),
        "splat_project_lidar": (C.c_int, [vp, vp, i32, i32, vp, vp, vp]),
        "splat_bin_sort_camera": (C.c_int, [vp, i32, i32, i64, vp, vp, vp, C.c_size_t, vp, vp]),
        "splat_bin_sort_lidar": (C.c_int, [vp, i32, i32, i64, vp, vp, vp, C.c_size_t, vp, vp]),
        "splat_rasterize_fwd_camera": (C.c_int, [vp, vp, i32, i32, vp, vp, i32, vp, vp, vp]),
        "splat_rasterize_fwd_lidar": (C.c_int, [vp, vp, i32, i32, vp, vp, i32, vp, vp, vp]),
        "splat_rasterize_bwd_camera": (C.c_int, [vp, vp, i32, i32, vp, vp, i32, vp, vp, vp, vp, vp, vp, C.c_size_t, vp]),
        "splat_rasterize_bwd_lidar": (C.c_int, [vp, vp, i32, i32, vp, vp, i32, vp, vp, vp, vp, vp, vp, C.c_size_t, vp]),
        "splat_project": (C.c_int, [vp, vp, i32, i32, vp, vp, vp]),
        "splat_bin_sort": (C.c_int, [vp, i32, i32, i64, vp, vp, vp, C.c_size_t, vp, vp]),
        "splat_rasterize_fwd": (C.c_int, [vp, vp, i32, i32, vp, vp, i32, vp, vp, vp]),
        "splat_rasterize_bwd": (C.c_int, [vp, vp, i32, i32, vp, vp, i32, vp, vp, vp, vp, vp, vp, C.c_size_t, vp]),
        "splat_time_next_raster": (C.c_int, [vp, vp]),
        "splat_pipeline_create": (C.c_int, [vp, i32, i32, vp, C.POINTER(vp)]),
        "splat_pipeline_run": (C.c_int, [vp, vp]),
        "splat_pipeline_destroy": (None, [vp]),
        "splat_device_clock": (C.c_int, [vp, vp]),
        "splat_device_clock_hz": (C.c_int, [C.POINTER(C.c_int64)]),
        "splat_compose": (C.c_int, [i64, vp, vp, vp, vp, vp, vp, vp, vp, vp]),
        "splat_compose_workspace_bytes": (C.c_size_t, [i32]),
        "splat_compose_bwd": (C.c_int, [i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, C.c_size_t, vp]),
        "splat_compose_bwd_noalloc": (C.c_int, [i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]),
        "splat_lidar_points_to_rays": (C.c_int, [i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]),
        "splat_mcmc_regularizer": (C.c_int, [vp, C.c_float, C.c_float, vp, vp, vp]),
        "splat_lidar_decode": (C.c_int, [i64, vp, vp, vp, vp, vp, vp, vp]),
        "splat_lidar_decode_workspace_bytes": (C.c_size_t, [i64, i32]),
        "splat_lidar_decode_bwd": (C.c_int, [i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, C.c_size_t, vp]),
        "splat_camera_decode_workspace_bytes": (C.c_size_t, [i32, i32]),
        "splat_mcmc_relocate_workspace_bytes": (C.c_size_t, [i64]),
        "splat_mcmc_relocate": (C.c_int, [vp, vp, C.c_float, i32, vp, vp, vp, C.c_size_t, vp]),
        "splat_camera_decode": (C.c_int, [vp, vp, vp, vp, vp, C.c_size_t, vp]),
        "splat_camera_decode_bwd": (C.c_int, [vp, vp, vp, vp, vp, vp, vp, C.c_size_t, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


def load(path: str = LIB_PATH):
    """Load libsplat.so (built by `python -m paper_2411_16816_amd.build`)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build it with `python -m paper_2411_16816_amd.build`")
        _lib = _declare(C.CDLL(path))
    return _lib


class SplatError(RuntimeError):
    pass


def check(rc: int, what: str):
    if rc != 0:
        raise SplatError(f"{what}: {load().splat_status_string(rc).decode()} ({rc})")


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream=None) -> C.c_void_p:
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


# ----------------------------------------------------------------------------------------
@dataclass
class GaussTensors:
    means: torch.Tensor
    log_scales: torch.Tensor
    quats: torch.Tensor
    opacities: torch.Tensor
    velocities: Optional[torch.Tensor]
    features: torch.Tensor

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    @staticmethod
    def from_numpy(g, device="cuda") -> "GaussTensors":
        f = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(device)
        return GaussTensors(f(g.means), f(g.log_scales), f(g.quats), f(g.opacities),
                            None if g.velocities is None else f(g.velocities), f(g.features))

    def struct(self) -> st.SplatGaussians:
        s = st.SplatGaussians()
        s.n = self.n
        s.means, s.log_scales, s.quats = _ptr(self.means), _ptr(self.log_scales), _ptr(self.quats)
        s.opacities, s.velocities, s.features = _ptr(self.opacities), _ptr(self.velocities), _ptr(self.features)
        s.c_total = int(self.features.shape[1])
        return s


class Rig:
    """A SplatRig: cameras first, then lidars; lidar ray arrays are uploaded and kept alive."""

    def __init__(self, cameras: Sequence, lidars: Sequence, device="cuda"):
        lib = load()
        self.lib = lib
        self.cameras = list(cameras)
        self.lidars = list(lidars)
        self.n_cam, self.n_lid = len(self.cameras), len(self.lidars)
        h = C.c_void_p()
        check(lib.splat_rig_create(self.n_cam, self.n_lid, C.byref(h)), "splat_rig_create")
        self.handle = h
        self.device = device
        self.ray_tensors = []
        self._upload()
        lay = st.SplatRigLayout()
        check(lib.splat_rig_layout(h, C.byref(lay)), "splat_rig_layout")
        n = self.n_cam + self.n_lid
        self.tile_base = np.array(lay.tile_base[:n + 1], np.int64)
        self.ray_base = np.array(lay.ray_base[:n + 1], np.int64)
        self.feat_base = np.array(lay.feat_base[:n + 1], np.int64)
        self.sensors = self.cameras + self.lidars

    def _upload(self):
        """Sensor structs -> splat_rig_set on the current stream.  Lidar ray arrays of unchanged
        length are copied into the existing device tensors (their addresses stay valid)."""
        keep = []
        cams = (st.SplatCamera * max(1, self.n_cam))()
        for i, c in enumerate(self.cameras):
            cams[i] = st.camera_struct(c)
        lids = (st.SplatLidar * max(1, self.n_lid))()
        for i, l in enumerate(self.lidars):
            f32 = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32))
            host = {"az": f32(l.ray_az), "el": f32(l.ray_el), "t": f32(l.ray_t)}
            if getattr(l, "ray_range", None) is not None:   # measured ranges: the line-of-sight sum
                host["range"] = f32(l.ray_range)
            if getattr(l, "ray_priority", None) is not None:   # the training-time cap
                # uint16 priorities travel as int16 bit patterns (torch has no uint16 copies)
                host["priority"] = torch.from_numpy(np.ascontiguousarray(l.ray_priority, np.uint16).view(np.int16))
            old = self.ray_tensors[i] if i < len(self.ray_tensors) else None
            if (old is not None and old.keys() == host.keys()
                    and all(old[k].numel() == h.numel() for k, h in host.items())):
                for k, h in host.items():
                    old[k].copy_(h)
            else:
                dev = {k: h.to(self.device) for k, h in host.items()}
                if old is not None:
                    self.ray_tensors[i] = dev
                else:
                    self.ray_tensors.append(dev)
            lids[i] = st.lidar_struct(l, {k: d.data_ptr() for k, d in self.ray_tensors[i].items()}, keep)
        self._cams, self._lids, self._keep = cams, lids, keep
        check(self.lib.splat_rig_set(self.handle, cams if self.n_cam else None, lids if self.n_lid else None,
                                     _stream()), "splat_rig_set")

    def update(self, cameras: Optional[Sequence] = None, lidars: Optional[Sequence] = None):
        """New sensor parameters (poses, motion, rays) for the same sensors; uploaded on the current
        stream.  Pipelines stay valid while tile, ray and channel counts are unchanged."""
        if cameras is not None:
            assert len(cameras) == self.n_cam
            self.cameras = list(cameras)
        if lidars is not None:
            assert len(lidars) == self.n_lid
            self.lidars = list(lidars)
        self._upload()
        self.sensors = self.cameras + self.lidars

    def kind(self, s: int) -> int:
        return KIND_CAMERA if s < self.n_cam else KIND_LIDAR

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                torch.cuda.synchronize()
                self.lib.splat_rig_destroy(self.handle)
                self.handle = None
        except Exception:
            pass


def _status_tensor(device) -> torch.Tensor:
    return torch.zeros(C.sizeof(st.SplatStatus), dtype=torch.uint8, device=device)


def read_status(t: torch.Tensor) -> st.SplatStatus:
    b = t.cpu().numpy().tobytes()
    return st.SplatStatus.from_buffer_copy(b)


class SensorPass:
    """All buffers of one call range [first, first + count) of a rig, and the four library calls.

    batched=False: the per-kind calls (all sensors of the range are cameras, or all lidars);
    count == 1 is the plain per-sensor form.  batched=True: the batched calls (any mix of
    cameras and lidars, one launch per step, persistent queue rasterisers)."""

    def __init__(self, rig: Rig, first: int, count: int, n_gauss: int, k_cap: int, device="cuda",
                 batched: bool = False):
        self.rig, self.first, self.count = rig, first, count
        self.lib = rig.lib
        self.batched = batched
        kinds = [rig.kind(s) for s in range(first, first + count)]
        if not batched:
            assert len(set(kinds)) == 1, "a per-kind call range holds one sensor kind"
        self.kind = kinds[0] if len(set(kinds)) == 1 else -1
        self.lidar = (not batched) and self.kind == KIND_LIDAR
        self.has_lidar = KIND_LIDAR in kinds
        self.device = device
        self.n_gauss = n_gauss
        tb, rb, fb = rig.tile_base, rig.ray_base, rig.feat_base
        self.n_tiles = int(tb[first + count] - tb[first])
        self.n_rays = int(rb[first + count] - rb[first])
        self.n_feat = int(fb[first + count] - fb[first])
        self.ray_off = rb[first:first + count + 1] - rb[first]
        self.feat_off = fb[first:first + count + 1] - fb[first]
        R = count * n_gauss
        i32 = dict(dtype=torch.int32, device=device)
        f32 = dict(dtype=torch.float32, device=device)
        self.mv = torch.empty((R, 4), **f32)
        self.cn = torch.empty((R, 4), **f32)
        self.box = torch.empty((R, 4), **f32)
        self.dv = torch.empty((R, 2), **f32)
        self.dkey = torch.empty((R,), dtype=torch.int64, device=device)
        self.rect = torch.empty((R, 4), **i32)
        self.ntiles = torch.empty((R,), **i32)
        self.tile_range = torch.empty((max(1, self.n_tiles), 2), dtype=torch.int64, device=device)
        self.entry_base = torch.empty((max(1, R),), dtype=torch.int64, device=device)
        if self.has_lidar or batched:
            self.work_cap = self.n_tiles + (self.n_rays + 255) // 256 + 1
            first_lidar = next((k for k in range(count) if rig.kind(first + k) == KIND_LIDAR), count)
            n_lidar_rays = self.n_rays - int(self.ray_off[first_lidar])
            self.ray_order = torch.empty((max(1, n_lidar_rays),), **i32)
            self.ray_range = torch.empty((self.n_tiles + 1, 2), **i32)
            self.work = torch.empty((self.work_cap, 2), **i32)
            self.n_work = torch.zeros((3,), **i32)
        else:
            self.work_cap = 0
            self.ray_order = self.ray_range = self.work = self.n_work = None
        self.feat = torch.empty((max(1, self.n_feat),), **f32)
        self.depth = torch.empty((max(1, self.n_rays),), **f32)
        self.alpha = torch.empty((max(1, self.n_rays),), **f32)
        self.t_final = torch.empty((max(1, self.n_rays),), **f32)
        self.last = torch.empty((max(1, self.n_rays),), **i32)
        self.median = torch.empty((max(1, self.n_rays),), **f32) if self.has_lidar else None
        self.los = torch.empty((max(1, self.n_rays),), **f32) if self.has_lidar else None
        self.dropped = torch.empty((max(1, self.n_rays),), dtype=torch.uint8, device=device) if self.has_lidar \
            else None
        self.status = _status_tensor(device)
        # bumped by every call that rewrites the forward state (records, lists, outputs,
        # capacity); SplatRenderFn.backward refuses state newer than its forward
        self.generation = 0
        self.set_capacity(k_cap)

    # ---- structs -------------------------------------------------------------------------
    def set_capacity(self, k_cap: int):
        self.generation += 1
        self.k_cap = int(k_cap)
        self.gauss = torch.empty((max(1, self.k_cap),), dtype=torch.int32, device=self.device)
        nbytes = int(self.lib.splat_workspace_bytes(self.rig.handle, self.first, self.count, self.n_gauss, self.k_cap))
        if nbytes == 0:
            raise SplatError("splat_workspace_bytes returned 0")
        self.ws = torch.empty((nbytes + 256,), dtype=torch.uint8, device=self.device)
        self.ws_ptr = (self.ws.data_ptr() + 255) // 256 * 256
        self.ws_bytes = nbytes

    def proj_struct(self):
        p = st.SplatProjected()
        p.n_records = self.count * self.n_gauss
        p.mv, p.cn, p.box, p.dv = _ptr(self.mv), _ptr(self.cn), _ptr(self.box), _ptr(self.dv)
        p.dkey = _ptr(self.dkey)
        p.rect, p.n_tiles = _ptr(self.rect), _ptr(self.ntiles)
        return p

    def lists_struct(self):
        L = st.SplatTileLists()
        L.k_cap = self.k_cap
        L.gauss, L.tile_range, L.entry_base = _ptr(self.gauss), _ptr(self.tile_range), _ptr(self.entry_base)
        L.ray_order, L.ray_range, L.work, L.n_work = (_ptr(self.ray_order), _ptr(self.ray_range),
                                                      _ptr(self.work), _ptr(self.n_work))
        L.work_cap = self.work_cap
        return L

    def out_struct(self, sensor_done: Optional[torch.Tensor] = None, d_los: Optional[torch.Tensor] = None):
        o = st.SplatRenderOut()
        o.feat, o.depth, o.alpha = _ptr(self.feat), _ptr(self.depth), _ptr(self.alpha)
        o.t_final, o.last, o.median = _ptr(self.t_final), _ptr(self.last), _ptr(self.median)
        o.sensor_done = _ptr(sensor_done)
        o.los, o.d_los = _ptr(self.los), _ptr(d_los)
        o.dropped = _ptr(self.dropped)
        return o

    # ---- the four calls -------------------------------------------------------------------
    def project(self, g: GaussTensors, stream=None):
        self.generation += 1
        fn = (self.lib.splat_project if self.batched else
              self.lib.splat_project_lidar if self.lidar else self.lib.splat_project_camera)
        check(fn(C.byref(g.struct()), self.rig.handle, self.first, self.count, C.byref(self.proj_struct()),
                 _ptr(self.status), _stream(stream)), "splat_project")

    def bin_sort(self, stream=None):
        self.generation += 1
        fn = (self.lib.splat_bin_sort if self.batched else
              self.lib.splat_bin_sort_lidar if self.lidar else self.lib.splat_bin_sort_camera)
        check(fn(self.rig.handle, self.first, self.count, self.n_gauss, C.byref(self.proj_struct()),
                 C.byref(self.lists_struct()), C.c_void_p(self.ws_ptr), self.ws_bytes, _ptr(self.status),
                 _stream(stream)), "splat_bin_sort")

    def _time(self, timer):
        """Ask the library to record timer = (start, stop) torch events around the next
        rasteriser kernel (splat_time_next_raster)."""
        if timer is not None:
            a, b = timer
            check(self.lib.splat_time_next_raster(C.c_void_p(a.cuda_event), C.c_void_p(b.cuda_event)),
                  "splat_time_next_raster")

    def raster_fwd(self, g: GaussTensors, support=BOX, stream=None, count_pairs: bool = False, timer=None,
                   sensor_done: Optional[torch.Tensor] = None):
        """sensor_done: optional int64 [count] device tensor of per-sensor completion clocks."""
        self.generation += 1
        st_ = _ptr(self.status) if count_pairs else None
        self._time(timer)
        out = self.out_struct(sensor_done)
        if self.batched:
            check(self.lib.splat_rasterize_fwd(C.byref(g.struct()), self.rig.handle, self.first, self.count,
                                               C.byref(self.proj_struct()), C.byref(self.lists_struct()), support,
                                               C.byref(out), st_, _stream(stream)),
                  "splat_rasterize_fwd")
        elif self.lidar:
            check(self.lib.splat_rasterize_fwd_lidar(C.byref(g.struct()), self.rig.handle, self.first, self.count,
                                                     C.byref(self.proj_struct()), C.byref(self.lists_struct()),
                                                     support, C.byref(out), st_,
                                                     _stream(stream)), "splat_rasterize_fwd_lidar")
        else:
            check(self.lib.splat_rasterize_fwd_camera(C.byref(g.struct()), self.rig.handle, self.first, self.count,
                                                      C.byref(self.proj_struct()), C.byref(self.lists_struct()),
                                                      support, C.byref(out), st_, _stream(stream)),
                  "splat_rasterize_fwd_camera")

    def raster_bwd(self, g: GaussTensors, dF, dD, dA, grads: GaussTensors, support=BOX, stream=None, timer=None,
                   sensor_done: Optional[torch.Tensor] = None, sensor_grads: Optional[dict] = None,
                   d_los: Optional[torch.Tensor] = None):
        """d_los: optional [n_rays] upstream gradient of the lidar line-of-sight sums."""
        gr = _grads_struct(grads, sensor_grads)
        self._time(timer)
        fn = (self.lib.splat_rasterize_bwd if self.batched else
              self.lib.splat_rasterize_bwd_lidar if self.lidar else self.lib.splat_rasterize_bwd_camera)
        check(fn(C.byref(g.struct()), self.rig.handle, self.first, self.count, C.byref(self.proj_struct()),
                 C.byref(self.lists_struct()), support, C.byref(self.out_struct(sensor_done, d_los)), _ptr(dF), _ptr(dD),
                 _ptr(dA),
                 C.byref(gr), C.c_void_p(self.ws_ptr), self.ws_bytes, _stream(stream)), "splat_rasterize_bwd")

    # ---- conveniences ---------------------------------------------------------------------
    def fit_capacity(self, g: GaussTensors, margin: float = 1.1, stream=None) -> int:
        """Project, bin with zero capacity to learn K, and size the lists (host sync)."""
        self.status.zero_()
        self.project(g, stream)
        old = self.k_cap
        if old != 0:
            self.set_capacity(0)
        self.bin_sort(stream)
        torch.cuda.synchronize()
        K = int(read_status(self.status).n_isect)
        self.set_capacity(max(1, int(K * margin) + 1024))
        self.status.zero_()
        return K

    def render(self, g: GaussTensors, support=BOX, stream=None):
        """project -> bin/sort -> rasterise (no host sync).  Returns the output tensors."""
        self.project(g, stream)
        self.bin_sort(stream)
        self.raster_fwd(g, support, stream)
        return self.outputs()

    def outputs(self):
        n = self.n_rays
        return dict(feat=self.feat[:self.n_feat], depth=self.depth[:n], alpha=self.alpha[:n],
                    t_final=self.t_final[:n], last=self.last[:n],
                    median=None if self.median is None else self.median[:n],
                    los=None if self.los is None else self.los[:n],
                    dropped=None if self.dropped is None else self.dropped[:n])

    def sensor_slices(self, k: int):
        """(ray slice, feature slice, channels) of the k-th sensor of the call."""
        s = self.rig.sensors[self.first + k]
        return (slice(int(self.ray_off[k]), int(self.ray_off[k + 1])),
                slice(int(self.feat_off[k]), int(self.feat_off[k + 1])), s.n_channels)


SENSOR_GRAD_FIELDS = ("sensor_lin_vel", "sensor_ang_vel", "sensor_time_offset")


def _grads_struct(grads: GaussTensors, sensor_grads: Optional[dict] = None) -> st.SplatGrads:
    """sensor_grads: optional {"sensor_lin_vel": [count,3], "sensor_ang_vel": [count,3],
    "sensor_time_offset": [count]} float32 device accumulators of the call's sensors."""
    gr = st.SplatGrads()
    gr.means, gr.log_scales, gr.quats = _ptr(grads.means), _ptr(grads.log_scales), _ptr(grads.quats)
    gr.opacities, gr.velocities, gr.features = _ptr(grads.opacities), _ptr(grads.velocities), _ptr(grads.features)
    for f in SENSOR_GRAD_FIELDS:
        setattr(gr, f, _ptr((sensor_grads or {}).get(f)))
    return gr


class Pipeline:
    """One step of a batched SensorPass captured as a hipGraph (splat_pipeline_*).  The tensors
    named here are captured by address and kept alive by this object; `run` replays the step."""

    def __init__(self, sp: SensorPass, g: GaussTensors, support=BOX, grads: Optional[GaussTensors] = None,
                 dF=None, dD=None, dA=None, zero_grads: bool = True, d_los=None, count_pairs: bool = False):
        if not sp.batched:
            raise ValueError("pipelines run the batched form")
        self.lib, self.sp, self.g = sp.lib, sp, g
        self.keep = (grads, dF, dD, dA, d_los)
        step = st.SplatStep()
        step.gaussians = g.struct()
        step.proj, step.lists, step.out = sp.proj_struct(), sp.lists_struct(), sp.out_struct(d_los=d_los)
        step.support = support
        step.flags = st.SPLAT_STEP_COUNT_PAIRS if count_pairs else 0
        if grads is not None:
            step.flags |= st.SPLAT_STEP_BACKWARD | (st.SPLAT_STEP_ZERO_GRADS if zero_grads else 0)
            step.d_feat, step.d_depth, step.d_alpha = _ptr(dF), _ptr(dD), _ptr(dA)
            step.grads = _grads_struct(grads)
        step.ws, step.ws_bytes = C.c_void_p(sp.ws_ptr), sp.ws_bytes
        step.status = _ptr(sp.status)
        self.handle = C.c_void_p()
        check(self.lib.splat_pipeline_create(sp.rig.handle, sp.first, sp.count, C.byref(step), C.byref(self.handle)),
              "splat_pipeline_create")

    def run(self, stream=None):
        check(self.lib.splat_pipeline_run(self.handle, _stream(stream)), "splat_pipeline_run")

    def close(self):
        if self.handle:
            self.lib.splat_pipeline_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def zeros_like_grads(g: GaussTensors) -> GaussTensors:
    z = torch.zeros_like
    return GaussTensors(z(g.means), z(g.log_scales), z(g.quats), z(g.opacities),
                        None if g.velocities is None else z(g.velocities), z(g.features))


def check_saved_state(sp, generation: int):
    """Raise unless `sp` still holds the forward state recorded at `generation`."""
    if sp.generation != generation:
        raise SplatError("SplatRenderFn.backward: the SensorPass was used again after this forward "
                         f"(state {sp.generation}, forward {generation}); run backward before the next "
                         "render through the same pass, or give each render its own pass")


class SplatRenderFn(torch.autograd.Function):
    """Differentiable render of one call range.  Inputs are the Gaussian tensors; outputs are the
    flat feature rows, depth and alpha of the call (see SensorPass.sensor_slices).  The pass's
    buffers hold the forward state, so backward must run before the pass renders again: a
    backward whose pass has projected, binned, rendered or been resized since its forward raises
    SplatError instead of differentiating the newer state."""

    @staticmethod
    def forward(ctx, sp: SensorPass, support: int, means, log_scales, quats, opacities, velocities, features):
        g = GaussTensors(means.contiguous(), log_scales.contiguous(), quats.contiguous(), opacities.contiguous(),
                         None if velocities is None else velocities.contiguous(), features.contiguous())
        sp.status.zero_()
        sp.project(g)
        sp.bin_sort()
        st_ = read_status(sp.status)
        if st_.overflow:
            sp.set_capacity(int(st_.n_isect * 1.1) + 1024)
            sp.bin_sort()
        sp.raster_fwd(g, support)
        ctx.sp, ctx.support, ctx.g = sp, support, g
        ctx.generation = sp.generation
        ctx.has_vel = velocities is not None
        o = sp.outputs()
        return o["feat"].clone(), o["depth"].clone(), o["alpha"].clone()

    @staticmethod
    def backward(ctx, dF, dD, dA):
        sp, g = ctx.sp, ctx.g
        check_saved_state(sp, ctx.generation)
        grads = zeros_like_grads(g)
        f32 = lambda t, n: torch.zeros(n, dtype=torch.float32, device=g.means.device) if t is None else t.contiguous()
        sp.raster_bwd(g, f32(dF, sp.n_feat), f32(dD, sp.n_rays), f32(dA, sp.n_rays), grads, ctx.support)
        return (None, None, grads.means, grads.log_scales, grads.quats, grads.opacities,
                grads.velocities if ctx.has_vel else None, grads.features)


# ----------------------------------------------------------------------------------------
# scene-graph composition (splat_compose / splat_compose_bwd)
# ----------------------------------------------------------------------------------------
ACTOR_FIELDS = ("rot", "trans", "rot_offset", "trans_offset", "lin_vel", "lin_vel_offset", "ang_vel")
ACTOR_GRAD_FIELDS = ("rot_offset", "trans_offset", "lin_vel_offset", "ang_vel")


@dataclass
class ActorTensors:
    """Actor poses and motions at a capture time (device float32; None = identity / zero)."""
    rot: torch.Tensor                               # [A,4] (w,x,y,z)
    trans: torch.Tensor                             # [A,3]
    rot_offset: Optional[torch.Tensor] = None       # [A,4]
    trans_offset: Optional[torch.Tensor] = None     # [A,3]
    lin_vel: Optional[torch.Tensor] = None          # [A,3]
    lin_vel_offset: Optional[torch.Tensor] = None   # [A,3]
    ang_vel: Optional[torch.Tensor] = None          # [A,3]

    @property
    def n(self) -> int:
        return int(self.rot.shape[0])

    def struct(self) -> st.SplatActors:
        a = st.SplatActors()
        a.n = self.n
        for f in ACTOR_FIELDS:
            setattr(a, f, _ptr(getattr(self, f)))
        return a


def _f32(t: torch.Tensor, cols: int, name: str) -> torch.Tensor:
    if t.dtype != torch.float32 or not t.is_contiguous() or t.dim() != 2 or t.shape[1] != cols:
        raise SplatError(f"{name}: expected a contiguous float32 [*, {cols}] tensor")
    return t


def compose(means: torch.Tensor, quats: torch.Tensor, actor_id: torch.Tensor, actors: ActorTensors,
            velocities: Optional[torch.Tensor] = None, stream=None):
    """World means, rotations and velocities of the scene composed at the actors' poses."""
    lib = load()
    n = int(means.shape[0])
    _f32(means, 3, "means"), _f32(quats, 4, "quats")
    if actor_id.dtype != torch.int32 or actor_id.numel() != n:
        raise SplatError("actor_id: expected int32 [n]")
    mw, qw, vw = torch.empty_like(means), torch.empty_like(quats), torch.empty_like(means)
    A = actors.struct()
    check(lib.splat_compose(n, _ptr(means), _ptr(quats), _ptr(velocities), _ptr(actor_id), C.byref(A), _ptr(mw),
                            _ptr(qw), _ptr(vw), _stream(stream)), "splat_compose")
    return mw, qw, vw


def compose_bwd(means, quats, actor_id, actors: ActorTensors, d_means_w, d_quats_w, d_vel_w, d_means, d_quats,
                d_velocities=None, d_actors: Optional[dict] = None, ws: Optional[torch.Tensor] = None, stream=None):
    """Accumulates (+=) the gradients of the local arrays and of the learnable actor arrays."""
    lib = load()
    n = int(means.shape[0])
    need = int(lib.splat_compose_workspace_bytes(actors.n))
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=means.device)
    G = st.SplatActorGrads()
    for f in ACTOR_GRAD_FIELDS:
        setattr(G, f, _ptr((d_actors or {}).get(f)))
    A = actors.struct()
    check(lib.splat_compose_bwd(n, _ptr(means), _ptr(quats), _ptr(actor_id), C.byref(A), _ptr(d_means_w),
                                _ptr(d_quats_w), _ptr(d_vel_w), _ptr(d_means), _ptr(d_quats), _ptr(d_velocities),
                                C.byref(G), _ptr(ws), ws.numel(), _stream(stream)), "splat_compose_bwd")
    return ws


COMPOSE_NOALLOC_MAX_ACTORS = 16384   # SPLAT_COMPOSE_NOALLOC_MAX_ACTORS


def compose_bwd_noalloc(means, quats, actor_id, actors: ActorTensors, d_means_w, d_quats_w, d_vel_w, d_means,
                        d_quats, d_velocities=None, d_actors: Optional[dict] = None, stream=None):
    """compose_bwd through the entry point that allocates nothing: the per-actor accumulators
    live in the library's own per-GPU array (at most COMPOSE_NOALLOC_MAX_ACTORS actors).  Calls
    that overlap on one GPU race."""
    lib = load()
    n = int(means.shape[0])
    G = st.SplatActorGrads()
    for f in ACTOR_GRAD_FIELDS:
        setattr(G, f, _ptr((d_actors or {}).get(f)))
    A = actors.struct()
    check(lib.splat_compose_bwd_noalloc(n, _ptr(means), _ptr(quats), _ptr(actor_id), C.byref(A), _ptr(d_means_w),
                                        _ptr(d_quats_w), _ptr(d_vel_w), _ptr(d_means), _ptr(d_quats),
                                        _ptr(d_velocities), C.byref(G), _stream(stream)),
          "splat_compose_bwd_noalloc")


class ComposeFn(torch.autograd.Function):
    """Differentiable composition: (means, quats, velocities, rot_offset, trans_offset,
    lin_vel_offset, ang_vel) -> (world means, world quats, world velocities).  The base rotation,
    translation and linear velocity of the actors are constants."""

    @staticmethod
    def forward(ctx, actor_id, rot, trans, lin_vel, means, quats, velocities, rot_offset, trans_offset,
                lin_vel_offset, ang_vel):
        actors = ActorTensors(rot, trans, rot_offset, trans_offset, lin_vel, lin_vel_offset, ang_vel)
        mw, qw, vw = compose(means, quats, actor_id, actors, velocities)
        ctx.actors = actors
        ctx.save_for_backward(actor_id, means, quats)
        ctx.has_vel = velocities is not None
        return mw, qw, vw

    @staticmethod
    def backward(ctx, gm, gq, gv):
        actor_id, means, quats = ctx.saved_tensors
        A = ctx.actors
        z = lambda t: None if t is None else torch.zeros_like(t)
        dm, dq = torch.zeros_like(means), torch.zeros_like(quats)
        dv = torch.zeros_like(means) if ctx.has_vel else None
        da = {f: z(getattr(A, f)) for f in ACTOR_GRAD_FIELDS}
        compose_bwd(means, quats, actor_id, A, gm.contiguous(), gq.contiguous(), gv.contiguous(), dm, dq, dv, da)
        return (None, None, None, None, dm, dq, dv, da["rot_offset"], da["trans_offset"], da["lin_vel_offset"],
                da["ang_vel"])


# ----------------------------------------------------------------------------------------
# device clock (latency measurement)
# ----------------------------------------------------------------------------------------
def device_clock(dst: torch.Tensor, index: int = 0, stream=None):
    """Writes the device wall clock into dst[index] (int64 device tensor) in stream order."""
    check(load().splat_device_clock(C.c_void_p(dst.data_ptr() + 8 * index), _stream(stream)), "splat_device_clock")


def device_clock_hz() -> int:
    hz = C.c_int64()
    check(load().splat_device_clock_hz(C.byref(hz)), "splat_device_clock_hz")
    return int(hz.value)


ADJOINT_ROW_LIMIT = 1 << 29   # splat.h SPLAT_ADJOINT_ROW_LIMIT


def set_adjoint_row_limit(max_entries: int = ADJOINT_ROW_LIMIT):
    """Largest list capacity whose adjoint keeps per-entry gradient rows (splat_set_adjoint_row_limit);
    larger calls add every work item's sums atomically.  Process-wide: set it before sizing the
    workspaces it applies to."""
    check(load().splat_set_adjoint_row_limit(int(max_entries)), "splat_set_adjoint_row_limit")


# ----------------------------------------------------------------------------------------
# lidar points to rasterisation rays (splat_lidar_points_to_rays)
# ----------------------------------------------------------------------------------------
def points_to_rays(points: torch.Tensor, times: torch.Tensor, R, t, lin_vel=None, ang_vel=None,
                   with_range: bool = True, out=None, stream=None):
    """World points [n,3] (ego motion compensated) and capture times [n] -> (ray_az, ray_el,
    ray_range or None), float32 device tensors.  R (3x3 or 9), t, lin_vel, ang_vel: host arrays of
    the lidar (x_l = R x_w + t; velocities in the sensor frame).  `out` = (az, el, range) writes
    into existing tensors."""
    lib = load()
    n = int(points.shape[0])
    if points.dtype != torch.float32 or times.dtype != torch.float32 or not points.is_contiguous() \
            or not times.is_contiguous() or tuple(points.shape) != (n, 3) or times.numel() != n:
        raise ValueError("points [n,3] and times [n] must be contiguous float32")
    if out is None:
        az, el = torch.empty(n, dtype=torch.float32, device=points.device), torch.empty(n, dtype=torch.float32,
                                                                                       device=points.device)
        rg = torch.empty(n, dtype=torch.float32, device=points.device) if with_range else None
    else:
        az, el, rg = out
    h = lambda a, k: None if a is None else (C.c_float * k)(*np.asarray(a, np.float32).reshape(-1)[:k])
    Rh, th, vh, wh = h(R, 9), h(t, 3), h(lin_vel, 3), h(ang_vel, 3)
    check(lib.splat_lidar_points_to_rays(n, _ptr(points), _ptr(times), C.cast(Rh, C.c_void_p), C.cast(th, C.c_void_p),
                                         None if vh is None else C.cast(vh, C.c_void_p),
                                         None if wh is None else C.cast(wh, C.c_void_p), _ptr(az), _ptr(el), _ptr(rg),
                                         _stream(stream)), "splat_lidar_points_to_rays")
    return az, el, rg


# ----------------------------------------------------------------------------------------
# MCMC regulariser (splat_mcmc_regularizer)
# ----------------------------------------------------------------------------------------
MCMC_LAMBDA_O = 0.005
MCMC_LAMBDA_S = 0.001


def mcmc_regularizer(g: GaussTensors, value: Optional[torch.Tensor] = None, grads: Optional[GaussTensors] = None,
                     lambda_o: float = MCMC_LAMBDA_O, lambda_s: float = MCMC_LAMBDA_S, stream=None):
    """Adds the regulariser's value to `value` (float32 device scalar tensor) and its gradients to
    grads.opacities / grads.log_scales."""
    gr = None
    if grads is not None:
        gr = st.SplatGrads()
        gr.opacities, gr.log_scales = _ptr(grads.opacities), _ptr(grads.log_scales)
    check(load().splat_mcmc_regularizer(C.byref(g.struct()), float(lambda_o), float(lambda_s), _ptr(value),
                                        None if gr is None else C.byref(gr), _stream(stream)),
          "splat_mcmc_regularizer")


# ----------------------------------------------------------------------------------------
# lidar decoder (splat_lidar_decode / splat_lidar_decode_bwd)
# ----------------------------------------------------------------------------------------
MLP_FIELDS = ("w1", "b1", "w2", "b2")


@dataclass
class LidarMLP:
    """Weights of the lidar decoder: w1 [32, C+3], b1 [32], w2 [2, 32], b2 [2] (float32 device)."""
    w1: torch.Tensor
    b1: torch.Tensor
    w2: torch.Tensor
    b2: torch.Tensor

    @property
    def n_feat(self) -> int:
        return int(self.w1.shape[1]) - 3

    def struct(self) -> st.SplatLidarMLP:
        m = st.SplatLidarMLP()
        m.n_feat = self.n_feat
        m.w1, m.b1, m.w2, m.b2 = (_ptr(getattr(self, f)) for f in MLP_FIELDS)
        return m


def lidar_decode(feat: torch.Tensor, az: torch.Tensor, el: torch.Tensor, mlp: LidarMLP, stream=None):
    """(intensity [R], drop probability [R]) of feature rows feat [R, C]."""
    n = int(az.numel())
    if feat.numel() != n * mlp.n_feat:
        raise ValueError("feat must hold n_rays rows of n_feat channels")
    I = torch.empty(n, dtype=torch.float32, device=az.device)
    P = torch.empty(n, dtype=torch.float32, device=az.device)
    check(load().splat_lidar_decode(n, _ptr(feat), _ptr(az), _ptr(el), C.byref(mlp.struct()), _ptr(I), _ptr(P),
                                    _stream(stream)), "splat_lidar_decode")
    return I, P


def lidar_decode_bwd(feat, az, el, mlp: LidarMLP, d_int, d_drop, d_feat=None, d_mlp: Optional[dict] = None,
                     ws: Optional[torch.Tensor] = None, stream=None):
    """Adds dL/dfeat to d_feat and the weight gradients to d_mlp[field] (float32 device tensors)."""
    lib = load()
    n = int(az.numel())
    nb = int(lib.splat_lidar_decode_workspace_bytes(n, mlp.n_feat))
    if ws is None or ws.numel() < nb:
        ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=az.device)
    g = st.SplatLidarMLPGrads()
    d_mlp = d_mlp or {}
    g.w1, g.b1, g.w2, g.b2 = (_ptr(d_mlp.get(f)) for f in MLP_FIELDS)
    check(lib.splat_lidar_decode_bwd(n, _ptr(feat), _ptr(az), _ptr(el), C.byref(mlp.struct()), _ptr(d_int),
                                     _ptr(d_drop), _ptr(d_feat), C.byref(g), C.c_void_p(ws.data_ptr()), ws.numel(),
                                     _stream(stream)), "splat_lidar_decode_bwd")


# ----------------------------------------------------------------------------------------
# camera decoder (splat_camera_decode / splat_camera_decode_bwd)
# ----------------------------------------------------------------------------------------
@dataclass
class CameraCNN:
    """Camera decoder weights (float32 device): embed [E], w_in [32, D_f+3+E, 3, 3], b_in [32],
    w_block / b_block: four [32, 32, 3, 3] / [32], w_out [6, 32], b_out [6]."""
    embed: torch.Tensor
    w_in: torch.Tensor
    b_in: torch.Tensor
    w_block: list
    b_block: list
    w_out: torch.Tensor
    b_out: torch.Tensor

    @property
    def n_embed(self) -> int:
        return int(self.embed.numel())

    @property
    def n_feat(self) -> int:
        return int(self.w_in.shape[1]) - 3 - self.n_embed

    def struct(self) -> st.SplatCameraCNN:
        m = st.SplatCameraCNN()
        m.n_feat, m.n_embed = self.n_feat, self.n_embed
        m.embed, m.w_in, m.b_in = _ptr(self.embed), _ptr(self.w_in), _ptr(self.b_in)
        for k in range(4):
            m.w_block[k], m.b_block[k] = self.w_block[k].data_ptr(), self.b_block[k].data_ptr()
        m.w_out, m.b_out = _ptr(self.w_out), _ptr(self.b_out)
        return m


def camera_decode_workspace(cam, device="cuda") -> torch.Tensor:
    nb = int(load().splat_camera_decode_workspace_bytes(int(cam.width), int(cam.height)))
    if nb == 0:
        raise SplatError("splat_camera_decode_workspace_bytes returned 0")
    return torch.empty(nb, dtype=torch.uint8, device=device)


def camera_decode(cam, feat: torch.Tensor, cnn: CameraCNN, ws: torch.Tensor, stream=None) -> torch.Tensor:
    """Decoded image [H*W, 3] of the camera's feature rows feat [H*W * C]; ws from
    camera_decode_workspace (keeps the activations for camera_decode_bwd)."""
    image = torch.empty(int(cam.width) * int(cam.height) * 3, dtype=torch.float32, device=feat.device)
    check(load().splat_camera_decode(C.byref(st.camera_struct(cam)), _ptr(feat), C.byref(cnn.struct()), _ptr(image),
                                     C.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream)), "splat_camera_decode")
    return image


def camera_decode_bwd(cam, feat, cnn: CameraCNN, d_image, d_feat, d_cnn: dict, ws: torch.Tensor, stream=None):
    """Adds dL/dfeat to d_feat and the weight / embedding gradients to d_cnn (same keys as
    CameraCNN's fields; w_block and b_block lists of four)."""
    g = st.SplatCameraCNNGrads()
    g.embed, g.w_in, g.b_in = _ptr(d_cnn.get("embed")), _ptr(d_cnn.get("w_in")), _ptr(d_cnn.get("b_in"))
    for k in range(4):
        wb, bb = d_cnn.get("w_block"), d_cnn.get("b_block")
        g.w_block[k] = None if wb is None else wb[k].data_ptr()
        g.b_block[k] = None if bb is None else bb[k].data_ptr()
    g.w_out, g.b_out = _ptr(d_cnn.get("w_out")), _ptr(d_cnn.get("b_out"))
    check(load().splat_camera_decode_bwd(C.byref(st.camera_struct(cam)), _ptr(feat), C.byref(cnn.struct()),
                                         _ptr(d_image), _ptr(d_feat), C.byref(g), C.c_void_p(ws.data_ptr()), ws.numel(),
                                         _stream(stream)), "splat_camera_decode_bwd")


# ----------------------------------------------------------------------------------------
# MCMC relocation (splat_mcmc_relocate)
# ----------------------------------------------------------------------------------------
MCMC_DEAD_OPACITY = 0.005
MCMC_N_MAX = 51


def check_relocate_args(g: GaussTensors, u: torch.Tensor):
    """Host-side checks of splat_mcmc_relocate's arrays (the C side sees raw pointers only and
    cannot tell a short or mistyped array): contiguous float32 Gaussian arrays of n rows with
    3 / 3 / 4 / 1 / 3 / C columns on one device, and u a contiguous int32 or uint32 array of at
    least n entries on that device.  Raises SplatError."""
    if g.means is None or g.means.dim() != 2 or g.means.shape[1] != 3:
        raise SplatError("mcmc_relocate: means must be [n, 3]")
    n = int(g.means.shape[0])
    dev = g.means.device
    shapes = {"means": (3,), "log_scales": (3,), "quats": (4,), "opacities": (), "velocities": (3,),
              "features": None}
    for name, cols in shapes.items():
        t = getattr(g, name)
        if t is None:
            if name == "velocities":
                continue
            raise SplatError(f"mcmc_relocate: {name} is required")
        if t.dtype != torch.float32 or not t.is_contiguous() or t.device != dev:
            raise SplatError(f"mcmc_relocate: {name} must be a contiguous float32 tensor on {dev}")
        ok = t.shape[0] == n and (t.dim() == 2 if cols is None else tuple(t.shape[1:]) == cols)
        if not ok:
            raise SplatError(f"mcmc_relocate: {name} has shape {tuple(t.shape)}, expected {n} rows"
                             + ("" if cols is None else f" of shape {cols}"))
    if u is None or u.dtype not in (torch.int32, torch.uint32) or not u.is_contiguous() or u.device != dev:
        raise SplatError(f"mcmc_relocate: u must be a contiguous int32 or uint32 tensor on {dev}")
    if u.numel() < n:
        raise SplatError(f"mcmc_relocate: u holds {u.numel()} randoms for {n} Gaussians")


def mcmc_relocate(g: GaussTensors, u: torch.Tensor, dead_opacity: float = MCMC_DEAD_OPACITY,
                  n_max: int = MCMC_N_MAX, ws: Optional[torch.Tensor] = None, stream=None):
    """Relocates g's dead Gaussians in place.  u: int32 device tensor [n] holding uint32 random
    bits.  Returns (target int32 [n], number relocated as an int64 device tensor)."""
    check_relocate_args(g, u)
    lib = load()
    n = int(g.means.shape[0])
    st_ = st.SplatGaussianState()
    st_.n = n
    st_.means, st_.log_scales, st_.quats = _ptr(g.means), _ptr(g.log_scales), _ptr(g.quats)
    st_.opacities, st_.velocities, st_.features = _ptr(g.opacities), _ptr(g.velocities), _ptr(g.features)
    st_.c_total = int(g.features.shape[1]) if g.features is not None else 0
    nb = int(lib.splat_mcmc_relocate_workspace_bytes(n))
    if ws is None or ws.numel() < nb:
        ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=g.means.device)
    target = torch.empty(max(n, 1), dtype=torch.int32, device=g.means.device)
    moved = torch.zeros(1, dtype=torch.int64, device=g.means.device)
    check(lib.splat_mcmc_relocate(C.byref(st_), _ptr(u), float(dead_opacity), int(n_max), _ptr(target), _ptr(moved),
                                  C.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream)), "splat_mcmc_relocate")
    return target[:n], moved
