"""Oracle, step 1-7: covariance, sensor frames, projection, rolling-shutter velocity, boxes.

Plain FP64 torch (CPU).  Test infrastructure only.

Every function is written from the paper (arXiv 2411.16816):
  * covariance from scale and quaternion: Sec. 3.1 (scene representation);
  * camera projection mu^I, Sigma^I = J^I Sigma^C J^I^T, culling, rectangular 3-sigma box
    enlarged by |v^I| t_rs / 2: Sec. 3.2 "Projection, tiling, and sorting" and "Rolling shutter";
  * pixel velocity v^I = J^I(-omega_C x mu^C - v_C + v_dyn): Eq. (pixel_velocity), App. D;
  * lidar spherical projection (phi, omega, r), its Jacobian J^S, Sigma^S, v^S and culling:
    Sec. 3.3 Eq. (spherical_projection) and the printed J^S;
  * EWA dilation s and compensation sqrt(|Sigma|/|Sigma + sI|): Eq. (alpha).

Pins (tests/test_oracle_geometry.py): scipy rotations, closed forms for on-axis Gaussians,
central differences of the pinhole and spherical maps, time derivatives of explicitly moved
sensors (independent of the velocity formula), isotropic EWA factor.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

D = torch.float64
TWO_PI = 2.0 * math.pi


def t64(x) -> torch.Tensor:
    """FP64 tensor of x; a tensor passes through (keeping its autograd graph)."""
    if isinstance(x, torch.Tensor):
        return x.to(D)
    return torch.as_tensor(np.asarray(x, dtype=np.float64), dtype=D)


@dataclass
class Params:
    """Gaussian parameters as FP64 tensors (optionally requiring grad)."""
    means: torch.Tensor       # [N,3]
    log_scales: torch.Tensor  # [N,3]
    quats: torch.Tensor       # [N,4] (w,x,y,z), any norm
    opacities: torch.Tensor   # [N]
    velocities: torch.Tensor  # [N,3] world frame (zeros when the scene has none)
    features: torch.Tensor    # [N,C]

    @staticmethod
    def from_gaussians(g, requires_grad: bool = False) -> "Params":
        vel = np.zeros_like(g.means) if g.velocities is None else g.velocities
        p = Params(t64(g.means), t64(g.log_scales), t64(g.quats), t64(g.opacities), t64(vel),
                   t64(g.features))
        if requires_grad:
            for v in p.tensors():
                v.requires_grad_(True)
        return p

    def tensors(self):
        return [self.means, self.log_scales, self.quats, self.opacities, self.velocities,
                self.features]

    names = ("means", "log_scales", "quats", "opacities", "velocities", "features")


# --------------------------------------------------------------------------------------
# Sec. 3.1: Sigma = R S S^T R^T with S = diag(scale), R from the (normalised) quaternion
# --------------------------------------------------------------------------------------
def quat_to_rotmat(q: torch.Tensor) -> torch.Tensor:
    """Rotation matrix of the unit quaternion q/|q|, q = (w, x, y, z)."""
    q = q / torch.linalg.norm(q, dim=-1, keepdim=True)
    w, x, y, z = q.unbind(-1)
    r00 = 1 - 2 * (y * y + z * z)
    r01 = 2 * (x * y - w * z)
    r02 = 2 * (x * z + w * y)
    r10 = 2 * (x * y + w * z)
    r11 = 1 - 2 * (x * x + z * z)
    r12 = 2 * (y * z - w * x)
    r20 = 2 * (x * z - w * y)
    r21 = 2 * (y * z + w * x)
    r22 = 1 - 2 * (x * x + y * y)
    return torch.stack([torch.stack([r00, r01, r02], -1),
                        torch.stack([r10, r11, r12], -1),
                        torch.stack([r20, r21, r22], -1)], -2)


def covariance(log_scales: torch.Tensor, quats: torch.Tensor) -> torch.Tensor:
    """World covariance Sigma = R diag(exp(2 l)) R^T (scale parameterised as exp(l))."""
    R = quat_to_rotmat(quats)
    M = R * torch.exp(log_scales)[..., None, :]
    return M @ M.transpose(-1, -2)


def to_sensor(p: Params, R, t):
    """Mean and covariance in the sensor frame: mu^s = R mu + t, Sigma^s = R Sigma R^T."""
    R = t64(R)
    t = t64(t)
    mu = p.means @ R.T + t
    Sig = R @ covariance(p.log_scales, p.quats) @ R.T
    return mu, Sig


def relative_velocity(mu_s, p: Params, R, lin_vel, ang_vel):
    """Velocity of each Gaussian relative to the sensor, in the sensor frame (App. D):
    -omega_s x mu^s - v_s + R v_world, where the Gaussian's own world-frame velocity is
    rotated (not translated) into the sensor frame."""
    R = t64(R)
    w = t64(ang_vel).expand_as(mu_s)
    return -torch.linalg.cross(w, mu_s, dim=-1) - t64(lin_vel) + p.velocities @ R.T


# --------------------------------------------------------------------------------------
# common tail: EWA dilation, conic, compensated opacity, rectangular box (Eq. alpha, Sec. 3.2)
# --------------------------------------------------------------------------------------
def _dilate_and_box(mean2d, cov2, vel2, opac, eps2d, t_rs, t_off=0.0):
    """t_off: capture-time offset of the sensor (cameras): the rows are exposed over
    [t_off - t_rs/2, t_off + t_rs/2], so the box is centred on the mean at t_off (a candidacy
    decision, not differentiated)."""
    a = cov2[:, 0, 0] + eps2d
    b = cov2[:, 0, 1]
    c = cov2[:, 1, 1] + eps2d
    det_p = a * c - b * b
    conic = torch.stack([c / det_p, -b / det_p, a / det_p], -1)
    det2 = cov2[:, 0, 0] * cov2[:, 1, 1] - cov2[:, 0, 1] ** 2
    ratio = torch.clamp(det2, min=0.0) / det_p
    o_eff = opac * torch.sqrt(torch.clamp(ratio, min=1e-300))
    o_eff = torch.where(det2 > 0, o_eff, torch.zeros_like(o_eff))
    ext = 3.0 * torch.sqrt(torch.stack([a, c], -1)) + torch.abs(vel2) * (0.5 * t_rs)
    centre = mean2d + vel2.detach() * float(t_off)
    lo = centre - ext
    hi = centre + ext
    return conic, o_eff, ext, lo, hi


@dataclass
class Projection:
    mean2d: torch.Tensor   # [N,2] pixel (u,v) or (phi, omega); phi in [0, 2pi)
    vel2d: torch.Tensor    # [N,2] sensor-space velocity of the 2-D mean
    v_r: torch.Tensor      # [N] range velocity (lidar) or 0 (camera)
    cov2d: torch.Tensor    # [N,2,2] undilated projected covariance
    conic: torch.Tensor    # [N,3] (a,b,c) of (Sigma' )^-1 = [[a,b],[b,c]]
    o_eff: torch.Tensor    # [N] opacity times EWA compensation factor
    depth: torch.Tensor    # [N] sort key: camera z, lidar range r
    blend: torch.Tensor    # [N] value blended into D at t=0: camera z, lidar r
    ext: torch.Tensor      # [N,2] box half extents
    lo: torch.Tensor       # [N,2]
    hi: torch.Tensor       # [N,2]
    valid: torch.Tensor    # [N] bool, survives culling
    kind: str              # "camera" | "lidar"
    near_cull: torch.Tensor  # [N] bool: a culling decision within 1e-5 relative of its threshold


# --------------------------------------------------------------------------------------
# camera (Sec. 3.2)
# --------------------------------------------------------------------------------------
def project_camera(p: Params, cam) -> Projection:
    mu, Sig = to_sensor(p, cam.R, cam.t)
    x, y, z = mu.unbind(-1)
    in_depth = (z > cam.near) & (z < cam.far)
    zs = torch.where(in_depth, z, torch.ones_like(z))
    u = cam.fx * x / zs + cam.cx
    v = cam.fy * y / zs + cam.cy
    # Jacobian of the perspective map (upper two rows); x/z and y/z clamped to
    # +-jac_clamp * tan(half FOV) when jac_clamp > 0 (3DGS convention retained by the paper)
    tx = x / zs
    ty = y / zs
    if cam.jac_clamp > 0:
        limx = cam.jac_clamp * 0.5 * cam.width / cam.fx
        limy = cam.jac_clamp * 0.5 * cam.height / cam.fy
        tx = torch.clamp(tx, -limx, limx)
        ty = torch.clamp(ty, -limy, limy)
    zero = torch.zeros_like(z)
    J = torch.stack([torch.stack([cam.fx / zs, zero, -cam.fx * tx / zs], -1),
                     torch.stack([zero, cam.fy / zs, -cam.fy * ty / zs], -1)], -2)
    cov2 = J @ Sig @ J.transpose(-1, -2)
    vrel = relative_velocity(mu, p, cam.R, cam.lin_vel, cam.ang_vel)
    vel2 = (J @ vrel[..., None])[..., 0]
    mean2d = torch.stack([u, v], -1)
    t_off = getattr(cam, "time_offset", 0.0)
    t_off = float(t_off.detach()) if isinstance(t_off, torch.Tensor) else float(t_off)
    conic, o_eff, ext, lo, hi = _dilate_and_box(mean2d, cov2, vel2, p.opacities, cam.eps2d, cam.t_rs, t_off)
    with torch.no_grad():
        valid = in_depth.clone()
        valid &= (lo[:, 0] < cam.width) & (hi[:, 0] > 0) & (lo[:, 1] < cam.height) & (hi[:, 1] > 0)
        valid &= o_eff >= 1.0 / 255.0
        finite = torch.isfinite(torch.cat([mean2d, conic, lo, hi, vel2], -1)).all(-1) & torch.isfinite(o_eff)
        valid &= finite
        near_cull = (torch.abs(z - cam.near) <= 1e-5 * cam.near) | \
                    (torch.abs(o_eff * 255.0 - 1.0) <= 1e-4)
    return Projection(mean2d, vel2, zero, cov2, conic, o_eff, z, z, ext, lo, hi, valid, "camera",
                      near_cull)


# --------------------------------------------------------------------------------------
# lidar (Sec. 3.3)
# --------------------------------------------------------------------------------------
def spherical_jacobian(mu: torch.Tensor) -> torch.Tensor:
    """The printed 3x3 Jacobian J^S of (atan2(y,x), asin(z/r), r) with respect to (x,y,z)."""
    x, y, z = mu.unbind(-1)
    rho2 = x * x + y * y
    rho = torch.sqrt(rho2)
    r2 = rho2 + z * z
    r = torch.sqrt(r2)
    zero = torch.zeros_like(x)
    row0 = torch.stack([-y / rho2, x / rho2, zero], -1)
    row1 = torch.stack([-x * z / (r2 * rho), -y * z / (r2 * rho), rho / r2], -1)
    row2 = torch.stack([x / r, y / r, z / r], -1)
    return torch.stack([row0, row1, row2], -2)


def project_lidar(p: Params, lid) -> Projection:
    mu, Sig = to_sensor(p, lid.R, lid.t)
    x, y, z = mu.unbind(-1)
    rho = torch.sqrt(x * x + y * y)
    r = torch.sqrt(x * x + y * y + z * z)
    with torch.no_grad():
        in_range = (r >= lid.r_min) & (r <= lid.r_max) & (rho >= 1e-4 * r)
        # the spherical map is singular on the z axis and at the origin: substitute a harmless
        # point there only, so that range-culled entries keep their true (finite) box
        regular = (rho >= 1e-4 * r) & (r > 0)
    safe = regular[:, None]
    mu_s = torch.where(safe, mu, torch.tensor([1.0, 0.0, 0.0], dtype=D).expand_as(mu))
    xs, ys, zs = mu_s.unbind(-1)
    rs = torch.sqrt(xs * xs + ys * ys + zs * zs)
    phi = torch.atan2(ys, xs)
    phi = torch.where(phi < 0, phi + TWO_PI, phi)
    omega = torch.asin(zs / rs)
    J = spherical_jacobian(mu_s)
    J2 = J[:, :2, :]
    cov2 = J2 @ Sig @ J2.transpose(-1, -2)
    vrel = relative_velocity(mu_s, p, lid.R, lid.lin_vel, lid.ang_vel)
    v3 = (J @ vrel[..., None])[..., 0]
    mean2d = torch.stack([phi, omega], -1)
    conic, o_eff, ext, lo, hi = _dilate_and_box(mean2d, cov2, v3[:, :2], p.opacities, lid.eps2d, lid.t_rs)
    b0 = float(lid.elev_bounds[0])
    bM = float(lid.elev_bounds[-1])
    with torch.no_grad():
        valid = in_range.clone()
        valid &= (hi[:, 1] > b0) & (lo[:, 1] < bM)
        valid &= o_eff >= 1.0 / 255.0
        finite = torch.isfinite(torch.cat([mean2d, conic, lo, hi, v3], -1)).all(-1) & torch.isfinite(o_eff)
        valid &= finite
        near_cull = (torch.abs(r - lid.r_min) <= 1e-5 * lid.r_min) | \
                    (torch.abs(r - lid.r_max) <= 1e-5 * lid.r_max) | \
                    (torch.abs(rho - 1e-4 * r) <= 1e-5 * (1e-4 * r)) | \
                    (torch.abs(o_eff * 255.0 - 1.0) <= 1e-4)
    return Projection(mean2d, v3[:, :2], v3[:, 2], cov2, conic, o_eff, rs, rs, ext, lo, hi, valid,
                      "lidar", near_cull)


def project(p: Params, sensor) -> Projection:
    return project_lidar(p, sensor) if hasattr(sensor, "ray_az") else project_camera(p, sensor)
