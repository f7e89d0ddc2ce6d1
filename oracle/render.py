"""Oracle, steps 9-10: brute-force per-ray compositing.

Plain FP64 torch (CPU), differentiable.  Test infrastructure only.

For every ray the oracle evaluates *every* Gaussian (no tiling), keeps the candidates, orders
them by (depth, Gaussian id) and alpha-composites front to back:
  * pixel sample point p = (col + 1/2, row + 1/2) and time t_pix = (p_v / H - 1/2) t_rs
    (Eq. t_pix, Sec. 3.2); lidar rays bring their own (azimuth, elevation, time) (Sec. 3.3);
  * Delta = p - (mu + v t) (Eq. delta); the lidar azimuth difference is wrapped to [-pi, pi);
  * alpha = min(0.99, o_eff exp(-1/2 Delta^T (Sigma + sI)^-1 Delta)) (Eq. alpha; the 0.99
    clamp, the 1/255 skip and the T < 1e-4 stop are the 3DGS rules the paper keeps);
  * F = sum_i f_i alpha_i prod_{j<i}(1 - alpha_j) (Eq. alpha_blend); the depth output blends
    the camera z, or the rolling-shutter corrected lidar range r + v_r t (Sec. 3.3);
  * median range = corrected range of the first Gaussian after which the transmittance is
    below 1/2 (Sec. 3.3), 0 if there is none;
  * line-of-sight sum (the loss term L_los of the training-details appendix): for a lidar ray with a measured range r_p,
    the sum of the alphas of the blended Gaussians whose corrected range is below r_p - eps.

Candidate rule:
  BOX  (default) -- Gaussians whose 3-sigma + rolling-shutter box contains the sample point
                    (lo <= p < hi; the azimuth test is modular: (phi - lo) mod 2pi < hi - lo);
  TILE (literal) -- Gaussians whose tile range contains the ray's tile.
Under either rule a candidacy decided within the float32 band of a box edge (BOX) or of a tile
border (TILE) makes the ray near-decision if that Gaussian would pass the alpha skip rule there.

Pins (tests/test_oracle_render.py): single-Gaussian and two-Gaussian closed forms, empty scene,
monotone transmittance, weights summing to 1 - T, permutation invariance, rolling shutter
collapsing to global shutter at zero velocity, lidar rotation = column shift, scene scaling,
brute-force per-ray loop on tiny scenes.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

from . import geometry as geo
from . import tiles as tl

D = torch.float64
TWO_PI = 2.0 * math.pi
ALPHA_MIN = 1.0 / 255.0
ALPHA_MAX = 0.99
T_STOP = 1e-4
# near-decision windows (relative): a float32 evaluation of the same quantity may fall on the
# other side of a threshold inside these windows; such rays are reported, not compared
NEAR_BOX = 2e-6      # box edges, relative to |mean| + extent
NEAR_ALPHA = 2e-5    # alpha against 1/255 and 0.99
NEAR_T = 1e-4        # transmittance against the stop (1e-4) and the median (1/2) levels
NEAR_DEPTH = 1e-8    # depth ties between two Gaussians that both pass the skip rule (an ordering
                     # key of finite precision may order such a pair either way)


@dataclass
class Rays:
    p: torch.Tensor      # [R,2] sample point (pixel coordinates, or (azimuth, elevation))
    t: torch.Tensor      # [R] time relative to the sensor's mid-exposure
    tile: np.ndarray     # [R] tile id (for the TILE rule), -1 if the ray is outside all tiles
    valid: np.ndarray    # [R] bool
    los_thr: torch.Tensor = None   # [R] lidar: measured range minus the line-of-sight margin


def camera_rays(cam, pixel_idx=None) -> Rays:
    n = cam.width * cam.height
    idx = np.arange(n) if pixel_idx is None else np.asarray(pixel_idx)
    row = idx // cam.width
    col = idx % cam.width
    p = torch.stack([geo.t64(col + 0.5), geo.t64(row + 0.5)], -1)
    # capture time of the row relative to the sensor timestamp (Eq. t_pix), plus the camera's
    # time offset between its timestamp and the middle of the exposure (Sec. 3.2)
    t = geo.t64(((row + 0.5) / cam.height - 0.5) * cam.t_rs) + geo.t64(getattr(cam, "time_offset", 0.0))
    tx = -(-cam.width // cam.tile_w)
    tile = (row // cam.tile_h) * tx + col // cam.tile_w
    return Rays(p, t, tile, np.ones(idx.shape[0], bool))


def lidar_rays(lid, ray_idx=None) -> Rays:
    idx = np.arange(lid.n_rays) if ray_idx is None else np.asarray(ray_idx)
    az = lid.ray_az[idx].astype(np.float64)
    el = lid.ray_el[idx].astype(np.float64)
    p = torch.stack([geo.t64(az), geo.t64(el)], -1)
    a, e, valid = tl.lidar_ray_tiles(az, el, lid)
    tile = np.where(valid, e * lid.n_az_tiles + a, -1)
    rng_ = getattr(lid, "ray_range", None)
    thr = None if rng_ is None else geo.t64(np.asarray(rng_, np.float64)[idx]) - float(lid.los_eps)
    return Rays(p, geo.t64(lid.ray_t[idx]), tile, valid, thr)


def _box_mask(proj, cols, p, lo_pad=0.0):
    """Candidacy of Gaussians `cols` for points p under BOX; `lo_pad` > 0 widens (or < 0
    narrows) every edge by lo_pad * (|mean| + ext) to find near-edge decisions."""
    lo = proj.lo[cols].detach()
    hi = proj.hi[cols].detach()
    pad = lo_pad * (proj.mean2d[cols].detach().abs() + proj.ext[cols].detach())
    lo = lo - pad
    hi = hi + pad
    if proj.kind == "lidar":
        span = hi[:, 0] - lo[:, 0]
        d = torch.remainder(p[:, None, 0] - lo[None, :, 0], TWO_PI)
        m_az = d < span[None, :]
    else:
        m_az = (p[:, None, 0] >= lo[None, :, 0]) & (p[:, None, 0] < hi[None, :, 0])
    m_el = (p[:, None, 1] >= lo[None, :, 1]) & (p[:, None, 1] < hi[None, :, 1])
    return m_az & m_el


def _tile_mask(proj, sensor, cols, rays_tile, lo_pad=0.0):
    """Candidacy of Gaussians `cols` under TILE: the ray's tile lies in the Gaussian's tile
    range.  `lo_pad` widens (> 0) or narrows (< 0) every box edge by lo_pad * (|mean| + ext)
    before the ranges are taken, to find tile decisions within the float32 ambiguity band."""
    lo = proj.lo[cols].detach().numpy()
    hi = proj.hi[cols].detach().numpy()
    if lo_pad != 0.0:
        pad = lo_pad * (np.abs(proj.mean2d[cols].detach().numpy()) + proj.ext[cols].detach().numpy())
        lo = lo - pad
        hi = hi + pad
    if proj.kind == "lidar":
        start, n_az, el0, el1 = tl.lidar_tile_rect(lo, hi, sensor)
        M = sensor.n_az_tiles
        ta = rays_tile % M
        te = rays_tile // M
        m = ((ta[:, None] - start[None, :]) % M < n_az[None, :]) & \
            (te[:, None] >= el0[None, :]) & (te[:, None] < el1[None, :])
    else:
        x0, x1, y0, y1 = tl.camera_tile_rect(lo, hi, sensor)
        tx = -(-sensor.width // sensor.tile_w)
        rx = rays_tile % tx
        ry = rays_tile // tx
        m = (rx[:, None] >= x0[None, :]) & (rx[:, None] < x1[None, :]) & \
            (ry[:, None] >= y0[None, :]) & (ry[:, None] < y1[None, :])
    m &= (rays_tile >= 0)[:, None]
    return torch.from_numpy(m)


def _alpha_at(proj, ids, rays_p, rays_t):
    """alpha of Gaussians `ids` at the rays (as if they were candidates), [r, len(ids)]."""
    mean = proj.mean2d[ids].detach()
    vel = proj.vel2d[ids].detach()
    con = proj.conic[ids].detach()
    o = proj.o_eff[ids].detach()
    delta = rays_p[:, None, :] - (mean[None] + vel[None] * rays_t[:, None, None])
    if proj.kind == "lidar":
        d_az = torch.remainder(delta[..., 0] + math.pi, TWO_PI) - math.pi
        delta = torch.stack([d_az, delta[..., 1]], -1)
    dx, dy = delta[..., 0], delta[..., 1]
    sigma = 0.5 * (con[None, :, 0] * dx * dx + con[None, :, 2] * dy * dy) + con[None, :, 1] * dx * dy
    return torch.clamp(o[None] * torch.exp(-sigma), max=ALPHA_MAX)


def _composite(proj, feats, rays_p, rays_t, idx, cand, amb=None, los_thr=None):
    """Front-to-back compositing of the Gaussians `idx` (already in (depth, id) order) for a
    chunk of rays; `cand` [r,K] marks candidacy.  `amb` [r,K] marks Gaussians whose candidacy
    is a near-edge decision: the ray is near-decision if one of them would pass the alpha skip
    rule at or before the point where the ray stops.  `los_thr` [r] (lidar): the line-of-sight
    sum adds the alpha of every blended Gaussian whose corrected range is below it (the line-of-sight
    loss term of the training-details appendix).  Returns differentiable F, D, A, los and diagnostics."""
    mean = proj.mean2d[idx]
    vel = proj.vel2d[idx]
    con = proj.conic[idx]
    o = proj.o_eff[idx]
    delta = rays_p[:, None, :] - (mean[None] + vel[None] * rays_t[:, None, None])
    if proj.kind == "lidar":
        d_az = torch.remainder(delta[..., 0] + math.pi, TWO_PI) - math.pi
        delta = torch.stack([d_az, delta[..., 1]], -1)
    dx, dy = delta[..., 0], delta[..., 1]
    sigma = 0.5 * (con[None, :, 0] * dx * dx + con[None, :, 2] * dy * dy) + con[None, :, 1] * dx * dy
    alpha_raw = o[None] * torch.exp(-sigma)
    alpha = torch.clamp(alpha_raw, max=ALPHA_MAX)
    with torch.no_grad():
        keep1 = cand & (alpha >= ALPHA_MIN)
        t_try = torch.cumprod(1.0 - torch.where(keep1, alpha, torch.zeros_like(alpha)), dim=1)
        stop = t_try < T_STOP
        K = alpha.shape[1]
        first = torch.where(stop.any(1), stop.to(torch.int64).argmax(1), torch.full_like(stop[:, 0], K, dtype=torch.int64))
        keep = keep1 & (torch.arange(K)[None, :] < first[:, None])
    a = torch.where(keep, alpha, torch.zeros_like(alpha))
    t_after = torch.cumprod(1.0 - a, dim=1)
    ones = torch.ones_like(t_after[:, :1])
    t_before = torch.cat([ones, t_after[:, :-1]], 1)
    w = a * t_before
    if proj.kind == "lidar":
        g = proj.blend[idx][None] + proj.v_r[idx][None] * rays_t[:, None]
    else:
        g = proj.blend[idx][None].expand_as(w)
    F = w @ feats[idx]
    Dv = (w * g).sum(1)
    if los_thr is not None:
        front = keep & (g.detach() < los_thr[:, None])
        los = torch.where(front, alpha, torch.zeros_like(alpha)).sum(1)
    else:
        los = torch.zeros_like(Dv)
    T_final = t_after[:, -1]
    A = 1.0 - T_final
    with torch.no_grad():
        ta = t_after.detach()
        med_hit = keep & (ta < 0.5)
        has_med = med_hit.any(1)
        mi = med_hit.to(torch.int64).argmax(1)
        median = torch.where(has_med, g.detach().gather(1, mi[:, None])[:, 0], torch.zeros_like(A))
        has_last = keep.any(1)
        li = K - 1 - keep.flip(1).to(torch.int64).argmax(1)
        last_id = torch.where(has_last, torch.as_tensor(idx)[li], torch.full_like(li, -1))
        n_kept = keep.sum(1)
        ids1 = torch.as_tensor(idx, dtype=D)[None, :] + 1.0
        clamped = cand & (alpha_raw > ALPHA_MAX)
        sig = torch.stack([(keep * ids1).sum(1), (keep * ids1 * ids1).sum(1),
                           (clamped * ids1).sum(1)], -1)
        # near-decision diagnostics: decisions at or before the point where the ray stops
        reached = cand & (torch.arange(K)[None, :] <= first[:, None])
        near = (reached & (torch.abs(alpha * 255.0 - 1.0) <= NEAR_ALPHA)).any(1)
        near |= (reached & (torch.abs(alpha_raw / ALPHA_MAX - 1.0) <= NEAR_ALPHA)).any(1)
        upto = keep1 & (torch.arange(K)[None, :] <= first[:, None])
        near |= (upto & (torch.abs(t_try / T_STOP - 1.0) <= NEAR_T)).any(1)
        near |= (keep & (torch.abs(ta / 0.5 - 1.0) <= NEAR_T)).any(1)
        if amb is not None:
            matters = amb & (alpha >= ALPHA_MIN * (1.0 - NEAR_ALPHA)) & (torch.arange(K)[None, :] <= first[:, None])
            near |= matters.any(1)
        if los_thr is not None:   # a corrected range within float32 reach of the threshold
            gd = g.detach()
            near |= (keep & (torch.abs(gd - los_thr[:, None]) <= NEAR_BOX * (torch.abs(gd) + 1.0))).any(1)
        # depth near-ties among Gaussians that pass the skip rule up to the stop: distinct depths
        # closer than the ordering key resolves may be ordered differently; exactly equal depths
        # are ordered by id on both sides
        dep = proj.depth[idx].detach()
        if K > 1:
            gap = torch.abs(dep[1:] - dep[:-1])
            close = (gap <= NEAR_DEPTH * dep[1:]) & (gap > 0)
            both = upto[:, 1:] & upto[:, :-1]
            near |= (both & close[None, :]).any(1)
    return F, Dv, A, T_final, median, last_id, n_kept, near, sig, los


def render(proj, sensor, feats_all, rays: Rays, mode: str = "box", chunk: int = None):
    """Render every ray in `rays` against every Gaussian of `proj`.

    feats_all: [N, C_total] tensor; the sensor blends columns
    [feat_offset, feat_offset + n_channels).  Returns a dict of tensors."""
    off, C = sensor.feat_offset, sensor.n_channels
    feats = feats_all[:, off:off + C]
    valid = proj.valid.numpy()
    vid = np.nonzero(valid)[0]
    dep = proj.depth.detach().numpy()[vid]
    order = vid[np.lexsort((vid, dep))]
    n_rays = rays.p.shape[0]
    if chunk is None:
        chunk = int(max(1, min(256, 4_000_000 // max(1, order.shape[0]))))
    outF, outD, outA, outT, outM, outL, outN, outNear, outS, outLos = [], [], [], [], [], [], [], [], [], []
    near_cull = proj.near_cull.numpy()
    for s in range(0, n_rays, chunk):
        e = min(n_rays, s + chunk)
        p = rays.p[s:e]
        t = rays.t[s:e]
        rv = torch.from_numpy(rays.valid[s:e])
        if mode == "box":
            cand_all = _box_mask(proj, order, p) & rv[:, None]
            wide = _box_mask(proj, order, p, NEAR_BOX) & rv[:, None]
            narrow = _box_mask(proj, order, p, -NEAR_BOX) & rv[:, None]
            amb_all = wide != narrow   # candidacy decided within the float32 ambiguity band
            near_box = torch.zeros(e - s, dtype=torch.bool)
        else:
            cand_all = _tile_mask(proj, sensor, order, rays.tile[s:e])
            # a box edge within the float32 band of a tile border: the tile decision may differ
            wide = _tile_mask(proj, sensor, order, rays.tile[s:e], NEAR_BOX)
            narrow = _tile_mask(proj, sensor, order, rays.tile[s:e], -NEAR_BOX)
            amb_all = wide != narrow
            near_box = torch.zeros(e - s, dtype=torch.bool)
        # Gaussians whose culling is a near-threshold decision make the ray near if their box
        # reaches it and they would pass the alpha skip rule there
        nc_ids = np.nonzero(near_cull)[0]
        if nc_ids.shape[0] > 0:
            reach = _box_mask(proj, nc_ids, p, NEAR_BOX) & rv[:, None]
            blends = _alpha_at(proj, nc_ids, p, t) >= ALPHA_MIN * (1.0 - NEAR_ALPHA)
            near_box |= (reach & blends).any(1)
        cols = (cand_all | (amb_all if amb_all is not None else cand_all)).any(0).numpy()
        idx = order[cols]
        if idx.shape[0] == 0:
            r = e - s
            z = torch.zeros(r, dtype=D)
            outF.append(torch.zeros(r, C, dtype=D) + 0.0 * feats.sum())
            outD.append(z + 0.0 * proj.blend.sum())
            outA.append(z + 0.0 * proj.o_eff.sum())
            outT.append(torch.ones(r, dtype=D))
            outM.append(z)
            outL.append(torch.full((r,), -1, dtype=torch.int64))
            outN.append(torch.zeros(r, dtype=torch.int64))
            outNear.append(near_box)
            outS.append(torch.zeros(r, 3, dtype=D))
            outLos.append(z + 0.0 * proj.o_eff.sum())
            continue
        thr = None if rays.los_thr is None else rays.los_thr[s:e]
        F, Dv, A, T, M, L, N, near, S, LOS = _composite(proj, feats, p, t, idx, cand_all[:, cols],
                                                        None if amb_all is None else amb_all[:, cols], thr)
        outLos.append(LOS)
        outS.append(S)
        outF.append(F)
        outD.append(Dv)
        outA.append(A)
        outT.append(T)
        outM.append(M)
        outL.append(L)
        outN.append(N)
        outNear.append(near | near_box)
    return dict(F=torch.cat(outF), D=torch.cat(outD), A=torch.cat(outA), T=torch.cat(outT),
                median=torch.cat(outM), last_id=torch.cat(outL), n_kept=torch.cat(outN), los=torch.cat(outLos),
                near=torch.cat(outNear).numpy(), sig=torch.cat(outS))


def render_sensor(g_or_params, sensor, ray_idx=None, mode: str = "box", requires_grad=False,
                  chunk=None):
    """Project + render a sensor.  `g_or_params` is a scenes.Gaussians or a geometry.Params."""
    p = g_or_params if isinstance(g_or_params, geo.Params) else \
        geo.Params.from_gaussians(g_or_params, requires_grad)
    proj = geo.project(p, sensor)
    rays = lidar_rays(sensor, ray_idx) if hasattr(sensor, "ray_az") else camera_rays(sensor, ray_idx)
    out = render(proj, sensor, p.features, rays, mode, chunk)
    out["proj"] = proj
    out["params"] = p
    return out
