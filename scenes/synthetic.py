"""Seeded synthetic scenes and sensor rigs for the SplatAD rasterizer (arXiv 2411.16816).

This module only *generates inputs*: Gaussian parameter arrays, sensor poses, intrinsics,
lidar channel tables and per-ray (azimuth, elevation, time) lists.  It holds none of the
rendering method's arithmetic (no projection, tiling, sorting or compositing), so both the
CPU oracle and the GPU library consume exactly the same FP32 arrays produced here.

Conventions (inputs, shared by every consumer):
  * world frame: x forward, y left, z up (a driving frame);
  * Gaussians: means [N,3], log-scales [N,3] (scale = exp), quaternions [N,4] in (w,x,y,z)
    order, opacities [N] in (0,1), optional world-frame velocities [N,3], features [N,C];
  * camera: x_c = R x_w + t with OpenCV axes (x right, y down, z forward); linear and angular
    velocity are expressed in the camera frame (paper Sec. 3.2, App. D);
  * lidar: x_l = R x_w + t with x forward, y left, z up; velocities in the lidar frame
    (Sec. 3.3); rays are supplied as (azimuth in [0, 2pi), elevation, time relative to the
    middle of the sweep), beam-major: ray index = beam * n_az + azimuth step;
  * lidar elevation tiles: boundaries lie between channels (App. A); we place each interior
    boundary at the midpoint of the two adjacent channels that straddle it, and the outer
    boundaries half a channel gap beyond the extreme channels.

Random draws use NumPy PCG64, are made in float64 and cast once to float32.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Optional

import numpy as np

F32 = np.float32


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# ----------------------------------------------------------------------------------------
# data containers
# ----------------------------------------------------------------------------------------
@dataclass
class Gaussians:
    means: np.ndarray                 # [N,3] f32, world frame
    log_scales: np.ndarray            # [N,3] f32
    quats: np.ndarray                 # [N,4] f32 (w,x,y,z)
    opacities: np.ndarray             # [N] f32 in (0,1)
    velocities: Optional[np.ndarray]  # [N,3] f32 world-frame velocity, or None (all zero)
    features: np.ndarray              # [N,C] f32

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    @property
    def c_total(self) -> int:
        return int(self.features.shape[1])

    def subset(self, idx) -> "Gaussians":
        idx = np.asarray(idx)
        return Gaussians(
            self.means[idx].copy(), self.log_scales[idx].copy(), self.quats[idx].copy(),
            self.opacities[idx].copy(),
            None if self.velocities is None else self.velocities[idx].copy(),
            self.features[idx].copy())


@dataclass
class Camera:
    R: np.ndarray          # [3,3] f32 world -> camera rotation
    t: np.ndarray          # [3] f32
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    lin_vel: np.ndarray = field(default_factory=lambda: np.zeros(3, F32))  # camera frame
    ang_vel: np.ndarray = field(default_factory=lambda: np.zeros(3, F32))  # camera frame
    t_rs: float = 0.0          # rolling-shutter duration, first to last row [s]
    eps2d: float = 0.3         # EWA dilation s in pixels^2 (Sec. 3.2)
    near: float = 0.2
    far: float = 1.0e4
    jac_clamp: float = 1.3     # clamp of x/z, y/z to +-jac_clamp * half-FOV tangent; 0 = off
    feat_offset: int = 0
    n_channels: int = 0
    tile_w: int = 16
    tile_h: int = 16
    time_offset: float = 0.0   # sensor timestamp minus middle of the exposure [s]

    @property
    def n_rays(self) -> int:
        return self.width * self.height


@dataclass
class Lidar:
    R: np.ndarray            # [3,3] f32 world -> lidar rotation
    t: np.ndarray            # [3] f32
    lin_vel: np.ndarray      # [3] f32 lidar frame
    ang_vel: np.ndarray      # [3] f32 lidar frame
    t_rs: float              # sweep duration [s] (0 = global shutter)
    eps2d: float             # dilation in rad^2
    r_min: float
    r_max: float
    az_res: float            # azimuth resolution [rad]
    n_beams: int
    n_az: int
    tile_az: int             # N_phi: azimuth steps per tile
    tile_el: int             # N_omega: channels per tile
    n_az_tiles: int          # M_phi = ceil(n_az / N_phi)
    channel_elev: np.ndarray  # [n_beams] f32, ascending [rad]
    elev_bounds: np.ndarray   # [M_omega+1] f32, ascending [rad]
    ray_az: np.ndarray        # [R] f32 in [0, 2pi)
    ray_el: np.ndarray        # [R] f32
    ray_t: np.ndarray         # [R] f32, seconds relative to the middle of the sweep
    feat_offset: int = 0
    n_channels: int = 0
    ray_range: Optional[np.ndarray] = None   # [R] f32 measured range of each ray, or None
    los_eps: float = 0.8      # line-of-sight margin [m]
    ray_priority: Optional[np.ndarray] = None   # [R] uint16 training-time cap priorities, or None

    @property
    def n_rays(self) -> int:
        return int(self.ray_az.shape[0])

    @property
    def n_el_tiles(self) -> int:
        return int(self.elev_bounds.shape[0]) - 1


@dataclass
class Scene:
    name: str
    gaussians: Gaussians
    cameras: List[Camera]
    lidars: List[Lidar]
    seed: int

    @property
    def n_rays(self) -> int:
        return sum(c.n_rays for c in self.cameras) + sum(l.n_rays for l in self.lidars)


# ----------------------------------------------------------------------------------------
# Gaussians
# ----------------------------------------------------------------------------------------
def random_gaussians(rng: np.random.Generator, means: np.ndarray, n_feat: int,
                     rgb: bool = False, moving_frac: float = 0.2, vel_std: float = 3.0,
                     log_scale_mean: float = -0.5, log_scale_std: float = 0.4) -> Gaussians:
    """Default parameter distributions for a given set of means (float64 [N,3])."""
    n = means.shape[0]
    log_scales = rng.normal(log_scale_mean, log_scale_std, size=(n, 3))
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    opac = 1.0 / (1.0 + np.exp(-rng.normal(size=n)))
    if rgb:
        feats = np.concatenate([rng.uniform(0.0, 1.0, size=(n, 3)),
                                rng.normal(size=(n, n_feat - 3))], axis=1)
    else:
        feats = rng.normal(size=(n, n_feat))
    if moving_frac > 0.0:
        moving = rng.uniform(size=n) < moving_frac
        vel = rng.normal(0.0, vel_std, size=(n, 3)) * moving[:, None]
        vel = vel.astype(F32)
    else:
        vel = None
    return Gaussians(means.astype(F32), log_scales.astype(F32), q.astype(F32),
                     opac.astype(F32), vel, feats.astype(F32))


def uniform_box(rng, n, lo, hi) -> np.ndarray:
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    return lo + (hi - lo) * rng.uniform(size=(n, 3))


def road_slab(rng, n, x_range, y_range, z_max, ground_frac=0.7, ground_std=0.1) -> np.ndarray:
    """Means in a road-like slab: a fraction hugs the ground plane, the rest fill the slab."""
    x = rng.uniform(*x_range, size=n)
    y = rng.uniform(*y_range, size=n)
    ground = rng.uniform(size=n) < ground_frac
    z = np.where(ground, np.abs(rng.normal(0.0, ground_std, size=n)), rng.uniform(0.0, z_max, size=n))
    return np.stack([x, y, z], axis=1)


# ----------------------------------------------------------------------------------------
# sensor rigs (poses are inputs: rotations are built from yaw angles)
# ----------------------------------------------------------------------------------------
def _rot_z(yaw: float) -> np.ndarray:
    c, s = math.cos(yaw), math.sin(yaw)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


# camera axes (x right, y down, z forward) expressed in a yaw-0 vehicle frame (x fwd, y left, z up)
_CAM_AXES_IN_VEHICLE = np.array([[0.0, 0.0, 1.0],
                                 [-1.0, 0.0, 0.0],
                                 [0.0, -1.0, 0.0]])


def make_camera(position, yaw_deg: float, width: int, height: int, fx: float, fy: float = None,
                cx: float = None, cy: float = None, t_rs: float = 0.0,
                ego_vel_world=(0.0, 0.0, 0.0), ego_yaw_rate: float = 0.0,
                feat_offset: int = 0, n_channels: int = 16, tile=(16, 16), **kw) -> Camera:
    fy = fx if fy is None else fy
    cx = width / 2.0 if cx is None else cx
    cy = height / 2.0 if cy is None else cy
    R_cw = _rot_z(math.radians(yaw_deg)) @ _CAM_AXES_IN_VEHICLE   # columns: camera axes in world
    R_wc = R_cw.T
    pos = np.asarray(position, np.float64)
    t = -R_wc @ pos
    lin = R_wc @ np.asarray(ego_vel_world, np.float64)
    ang = R_wc @ np.array([0.0, 0.0, ego_yaw_rate])
    return Camera(R=R_wc.astype(F32), t=t.astype(F32), fx=float(F32(fx)), fy=float(F32(fy)),
                  cx=float(F32(cx)), cy=float(F32(cy)), width=int(width), height=int(height),
                  lin_vel=lin.astype(F32), ang_vel=ang.astype(F32), t_rs=float(F32(t_rs)),
                  feat_offset=feat_offset, n_channels=n_channels, tile_w=tile[0], tile_h=tile[1], **kw)


def channel_elevations(n_beams: int, el_min_deg: float, el_max_deg: float) -> np.ndarray:
    """Channel elevations [rad], denser near 0 deg: quantiles (k+1/2)/n of the density
    rho(w) ~ 1 + 3 exp(-(w / 4deg)^2) on [el_min, el_max]."""
    w = np.linspace(el_min_deg, el_max_deg, 200001)
    dens = 1.0 + 3.0 * np.exp(-(w / 4.0) ** 2)
    cdf = np.concatenate([[0.0], np.cumsum(0.5 * (dens[1:] + dens[:-1]) * np.diff(w))])
    cdf /= cdf[-1]
    q = (np.arange(n_beams) + 0.5) / n_beams
    return np.radians(np.interp(q, cdf, w))


def elevation_tile_bounds(channels: np.ndarray, tile_el: int) -> np.ndarray:
    """Tile boundaries between channel groups of tile_el channels (App. A)."""
    n = channels.shape[0]
    assert n % tile_el == 0, "number of beams must be a multiple of the channels per tile"
    m = n // tile_el
    b = np.empty(m + 1)
    for k in range(1, m):
        b[k] = 0.5 * (channels[k * tile_el - 1] + channels[k * tile_el])
    b[0] = channels[0] - 0.5 * (channels[1] - channels[0])
    b[m] = channels[-1] + 0.5 * (channels[-1] - channels[-2])
    return b


def make_lidar(position, yaw_deg: float, n_beams: int, el_min_deg: float, el_max_deg: float,
               n_az: int, t_sweep: float = 0.1, rolling_shutter: bool = True,
               ego_vel_world=(0.0, 0.0, 0.0), ego_yaw_rate: float = 0.0,
               tile_az: int = 32, tile_el: int = 8, r_min: float = 0.5, r_max: float = 250.0,
               feat_offset: int = 0, n_channels: int = 8, eps2d: Optional[float] = None) -> Lidar:
    R_lw = _rot_z(math.radians(yaw_deg))       # lidar axes in world
    R_wl = R_lw.T
    pos = np.asarray(position, np.float64)
    t = -R_wl @ pos
    lin = R_wl @ np.asarray(ego_vel_world, np.float64)
    ang = R_wl @ np.array([0.0, 0.0, ego_yaw_rate])
    ch = channel_elevations(n_beams, el_min_deg, el_max_deg)
    bounds = elevation_tile_bounds(ch, tile_el)
    az_res = 2.0 * math.pi / n_az
    j = np.arange(n_az)
    az = (j + 0.5) * az_res
    t_ray = ((j + 0.5) / n_az - 0.5) * t_sweep if rolling_shutter else np.zeros(n_az)
    ray_az = np.tile(az, n_beams)
    ray_el = np.repeat(ch, n_az)
    ray_t = np.tile(t_ray, n_beams)
    if eps2d is None:
        # filter std = geometric mean of the horizontal (azimuth step) and vertical (mean
        # channel spacing) divergences, so the dilation variance is their product [rad^2]
        d_el = (ch[-1] - ch[0]) / (n_beams - 1)
        eps2d = az_res * d_el
    return Lidar(R=R_wl.astype(F32), t=t.astype(F32), lin_vel=lin.astype(F32), ang_vel=ang.astype(F32),
                 t_rs=float(F32(t_sweep if rolling_shutter else 0.0)), eps2d=float(F32(eps2d)),
                 r_min=float(F32(r_min)), r_max=float(F32(r_max)), az_res=float(F32(az_res)),
                 n_beams=n_beams, n_az=n_az, tile_az=tile_az, tile_el=tile_el,
                 n_az_tiles=-(-n_az // tile_az), channel_elev=ch.astype(F32),
                 elev_bounds=bounds.astype(F32), ray_az=ray_az.astype(F32),
                 ray_el=ray_el.astype(F32), ray_t=ray_t.astype(F32),
                 feat_offset=feat_offset, n_channels=n_channels)


# ----------------------------------------------------------------------------------------
# the five configurations and the headline workload
# ----------------------------------------------------------------------------------------
SEED_BASE = 16816


def config_1(seed: int = SEED_BASE + 1) -> Scene:
    """Plain lidar forward: 4096 Gaussians in a 40x40x6 m box, static; 32 beams, 1024 az."""
    rng = _rng(seed)
    mu = uniform_box(rng, 4096, (-20, -20, -3), (20, 20, 3))
    g = random_gaussians(rng, mu, n_feat=8, moving_frac=0.0)
    lid = make_lidar((0, 0, 0), 0.0, 32, -25.0, 10.0, 1024, rolling_shutter=False,
                     feat_offset=0, n_channels=8)
    return Scene("C1_lidar_fwd", g, [], [lid], seed)


def config_2(seed: int = SEED_BASE + 2, n: int = 500_000) -> Scene:
    """Camera fwd+bwd: 500k Gaussians in a 100x30x8 m road slab; 1080p rolling-shutter camera."""
    rng = _rng(seed)
    mu = road_slab(rng, n, (0.0, 100.0), (-15.0, 15.0), 8.0)
    g = random_gaussians(rng, mu, n_feat=16, rgb=True)
    cam = make_camera((0, 0, 1.5), 0.0, 1920, 1080, 1500.0, t_rs=0.03, feat_offset=0, n_channels=16)
    return Scene("C2_camera_fwdbwd", g, [cam], [], seed)


def config_3(seed: int = SEED_BASE + 3, n: int = 2_000_000) -> Scene:
    """Lidar fwd+bwd: 2M Gaussians in a 300x300x6 m box; 128 beams x 2048 az, 100 ms sweep,
    15 m/s ego velocity.  Features have 3+13 columns; the lidar blends columns 3..10."""
    rng = _rng(seed)
    mu = uniform_box(rng, n, (-150, -150, -3), (150, 150, 3))
    g = random_gaussians(rng, mu, n_feat=16, rgb=True)
    lid = make_lidar((0, 0, 0), 0.0, 128, -25.0, 15.0, 2048, t_sweep=0.1,
                     ego_vel_world=(15.0, 0.0, 0.0), feat_offset=3, n_channels=8)
    return Scene("C3_lidar_fwdbwd", g, [], [lid], seed)


def config_4(seed: int = SEED_BASE + 4, n: int = 1_500_000) -> Scene:
    """Batched rig: 1.5M Gaussians; 6 rolling-shutter cameras of uneven sizes + 64x1800 lidar."""
    rng = _rng(seed)
    mu = road_slab(rng, n, (-75.0, 75.0), (-75.0, 75.0), 8.0)
    g = random_gaussians(rng, mu, n_feat=16, rgb=True)
    ego = (15.0, 0.0, 0.0)
    cams = []
    for yaw, (w, h) in [(0, (1920, 1080)), (180, (1920, 1080)), (60, (1280, 720)),
                        (-60, (1280, 720)), (120, (960, 640)), (-120, (960, 640))]:
        cams.append(make_camera((0, 0, 1.5), yaw, w, h, 0.78 * w, t_rs=0.03, ego_vel_world=ego,
                                feat_offset=0, n_channels=16))
    lid = make_lidar((0, 0, 2.0), 0.0, 64, -25.0, 15.0, 1800, t_sweep=0.1, ego_vel_world=ego,
                     feat_offset=3, n_channels=8)
    return Scene("C4_batched_rig", g, cams, [lid], seed)


def config_5(seed: int = SEED_BASE + 5, n: int = 3_000_000) -> Scene:
    """Batched simulation sweep: 3M Gaussians along a 500 m road; 48 lidar sweeps of mixed
    beam counts at seeded poses, plus 12 1080p cameras."""
    rng = _rng(seed)
    mu = road_slab(rng, n, (-20.0, 520.0), (-20.0, 20.0), 8.0)
    g = random_gaussians(rng, mu, n_feat=16, rgb=True)
    ego = (15.0, 0.0, 0.0)
    lidars = []
    specs = [(32, -30.0, 10.0)] * 16 + [(64, -25.0, 15.0)] * 16 + [(128, -25.0, 15.0)] * 16
    for beams, lo, hi in specs:
        x = rng.uniform(0.0, 500.0)
        y = rng.normal(0.0, 0.5)
        yaw = rng.normal(0.0, 2.0)
        n_az = int(rng.integers(1024, 2049))
        v = (15.0 * math.cos(math.radians(yaw)), 15.0 * math.sin(math.radians(yaw)), 0.0)
        lidars.append(make_lidar((x, y, 2.0), yaw, beams, lo, hi, n_az, t_sweep=0.1,
                                 ego_vel_world=v, r_max=200.0, feat_offset=3, n_channels=8))
    cams = []
    for k in range(12):
        x = rng.uniform(0.0, 500.0)
        y = rng.normal(0.0, 0.5)
        yaw = (0.0 if k % 2 == 0 else 180.0) + rng.normal(0.0, 2.0)
        cams.append(make_camera((x, y, 1.5), yaw, 1920, 1080, 1500.0, t_rs=0.03, ego_vel_world=ego,
                                feat_offset=0, n_channels=16))
    return Scene("C5_batched_sweep", g, cams, lidars, seed)


def measured_ranges(rng, n_rays: int, lo: float = 2.0, hi: float = 100.0) -> np.ndarray:
    """Stand-in for the ranges a lidar sweep measures: log-uniform in [lo, hi] m (returns are
    denser near the sensor), one per ray, float32."""
    return np.exp(rng.uniform(math.log(lo), math.log(hi), n_rays)).astype(np.float32)


def lidar_points(seed: int, n: int, t_sweep: float = 0.1):
    """Stand-in for a sweep's ego-motion-compensated points: world positions uniform in config 3's
    300 x 300 x 6 m box and capture times uniform over the sweep, relative to its middle
    (float32 [n,3], [n])."""
    rng = _rng(seed)
    pts = uniform_box(rng, n, (-150, -150, -3), (150, 150, 3)).astype(np.float32)
    t = rng.uniform(-0.5 * t_sweep, 0.5 * t_sweep, n).astype(np.float32)
    return pts, t


def headline(seed: int = SEED_BASE + 3, n: int = 2_000_000) -> Scene:
    """Headline workload: the 128-beam x 2048-azimuth lidar of config 3 plus one 1920x1080
    rolling-shutter camera at the lidar origin looking +x, over config 3's 2M Gaussians.
    The camera blends all 16 feature columns, the lidar columns 3..10; the lidar carries
    measured ranges (`measured_ranges`), so a training step includes the line-of-sight sum."""
    sc = config_3(seed, n)
    lid = sc.lidars[0]
    lid = replace(lid, ray_range=measured_ranges(_rng(seed + 100), lid.n_rays))
    cam = make_camera((0, 0, 0), 0.0, 1920, 1080, 1500.0, t_rs=0.03,
                      ego_vel_world=(15.0, 0.0, 0.0), feat_offset=0, n_channels=16)
    return Scene("H_lidar128x2048_cam1080p", sc.gaussians, [cam], [lid], seed)


def make_config(k: int, **kw) -> Scene:
    return {1: config_1, 2: config_2, 3: config_3, 4: config_4, 5: config_5}[k](**kw)


# ----------------------------------------------------------------------------------------
# scene graph: static background + rigid actors (cars on the road)
# ----------------------------------------------------------------------------------------
@dataclass
class ActorScene:
    gaussians: Gaussians        # means / quats in the actor frame for actor Gaussians
    actor_id: np.ndarray        # [N] int32, -1 = static background
    rot: np.ndarray             # [A,4] f32 base rotation (w,x,y,z), actor -> world
    trans: np.ndarray           # [A,3] f32 base translation (box centre), world
    rot_offset: np.ndarray      # [A,4] f32 learnable rotation offset (near identity)
    trans_offset: np.ndarray    # [A,3] f32
    lin_vel: np.ndarray         # [A,3] f32 actor frame
    lin_vel_offset: np.ndarray  # [A,3] f32
    ang_vel: np.ndarray         # [A,3] f32 actor frame


def actor_scene(seed: int, n: int, n_actors: int, actor_frac: float = 0.3, contiguous: bool = True,
                n_feat: int = 16, tumbling: bool = False) -> ActorScene:
    """A road slab (static, world frame) plus n_actors car-sized boxes (4.5 x 2 x 1.6 m) holding
    actor_frac of the Gaussians in their own frame.  Cars sit on the road (x in [5, 100] m,
    y in [-12, 12] m) with uniform yaw and small roll / pitch, drive forward at N(10, 3) m/s along
    their own x axis with yaw rates N(0, 0.2) rad/s; pose and velocity offsets are small (as
    after a few optimisation steps).  Gaussians of one actor are stored together when
    `contiguous`, otherwise the order is shuffled.  `tumbling` draws actor rotations uniformly
    (any roll and pitch) and angular velocities on every axis: a harder case than cars."""
    rng = _rng(seed)
    n_act = int(round(n * actor_frac)) if n_actors > 0 else 0
    n_static = n - n_act
    static_means = road_slab(rng, n_static, (0.5, 100.0), (-15.0, 15.0), 6.0)
    half = np.array([2.25, 1.0, 0.8])
    aid_act = rng.integers(0, max(n_actors, 1), size=n_act)
    aid_act.sort()
    local_means = rng.uniform(-1.0, 1.0, size=(n_act, 3)) * half
    means = np.concatenate([static_means, local_means])
    g = random_gaussians(rng, means, n_feat, rgb=True, moving_frac=0.2)
    aid = np.concatenate([np.full(n_static, -1, np.int64), aid_act]).astype(np.int32)
    if not contiguous:
        perm = rng.permutation(n)
        g = g.subset(perm)
        aid = aid[perm]
    g.velocities[aid >= 0] = 0.0
    A = max(n_actors, 0)
    yaw = rng.uniform(-math.pi, math.pi, size=A)
    tilt = rng.normal(0.0, 0.02, size=(A, 2))
    rot = np.stack([np.cos(yaw / 2), np.sin(tilt[:, 0] / 2), np.sin(tilt[:, 1] / 2), np.sin(yaw / 2)], 1)
    if tumbling:
        rot = rng.normal(size=(A, 4))
    rot /= np.linalg.norm(rot, axis=1, keepdims=True)
    trans = np.stack([rng.uniform(5.0, 100.0, A), rng.uniform(-12.0, 12.0, A), np.full(A, 0.8)], 1)
    rot_off = np.concatenate([np.ones((A, 1)), rng.normal(0.0, 0.01, size=(A, 3))], 1)
    f = lambda x: np.ascontiguousarray(x, dtype=F32)
    return ActorScene(g, aid, f(rot), f(trans), f(rot_off), f(rng.normal(0.0, 0.05, (A, 3))),
                      f(np.stack([rng.normal(10.0, 3.0, A), np.zeros(A), np.zeros(A)], 1)),
                      f(rng.normal(0.0, 0.1, (A, 3))),
                      f(rng.normal(0.0, 0.5, (A, 3)) if tumbling else
                        np.stack([np.zeros(A), np.zeros(A), rng.normal(0.0, 0.2, A)], 1)))


def upstream_grads(seed: int, n_rays: int, n_channels: int):
    """Seeded upstream gradients dL/dF [R,C], dL/dD [R], dL/dA [R] (float32)."""
    rng = _rng(seed)
    dF = rng.normal(size=(n_rays, n_channels)).astype(F32)
    dD = (0.01 * rng.normal(size=n_rays)).astype(F32)
    dA = rng.normal(size=n_rays).astype(F32)
    return dF, dD, dA


def with_tiles(cam: Camera, tile_w: int, tile_h: int) -> Camera:
    return replace(cam, tile_w=tile_w, tile_h=tile_h)
