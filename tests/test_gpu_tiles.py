"""Tile ranges end to end and the lidar azimuth seam (Sec. 3.2 "Projection, tiling, and sorting";
App. A, lidar tiling, the Phi_low / Phi_high cases and the wrap to [0, M_phi)).

* The library's tile rectangles against the oracle's FP64 App. A formulas evaluated on the
  oracle's own FP64 boxes (not on the library's float32 boxes): equal for every Gaussian both
  sides keep, except those whose box edge lies within 1e-5 relative (of |mean| + extent) of a
  tile border or of the 0 / 2 pi branch points, which are excluded and counted.
* Lidars whose last azimuth tile is partial (1800 steps in tiles of 32: M_phi = 57, tiles reach
  364.8 deg; 300 steps in tiles of 16: M_phi = 19), with Gaussians placed across 0 deg, inside the
  360 - 364.8 deg overlap and spanning every column: rectangles bit-exact under the documented
  float32 arithmetic and end to end against FP64, and every ray of the first two and last two
  azimuth tile columns rendered against the oracle in BOX and TILE modes."""
import math

import numpy as np
import pytest
import torch

from oracle import geometry as geo
from oracle import render as rd
from oracle import tiles as tl
from scenes import synthetic as S
from tests.gpu_helpers import gpu_outputs, last_ids_gpu, rtol_check

pytestmark = pytest.mark.gpu

TWO_PI = 2.0 * math.pi
NEAR_REL = 1e-5


def _binding():
    from paper_2411_16816_amd import binding
    binding.load()
    return binding


def _frac_near(a, tol):
    """|a - round(a)| <= tol (a, tol arrays in units of one tile)."""
    return np.abs(a - np.round(a)) <= tol


def near_tile_border(pr, sensor):
    """Gaussians whose FP64 box edge lies within NEAR_REL (|mean| + extent) of a tile border or
    of a branch point of the lidar formulas (lo = 0, hi = 2 pi), per App. A's cases."""
    lo = pr.lo.detach().numpy()
    hi = pr.hi.detach().numpy()
    tol = NEAR_REL * (np.abs(pr.mean2d.detach().numpy()) + pr.ext.detach().numpy())
    if hasattr(sensor, "ray_az"):
        w = sensor.tile_az * float(sensor.az_res)
        phi_max = sensor.n_az_tiles * w
        a_lo = np.where(lo[:, 0] >= 0, lo[:, 0] / w, (lo[:, 0] + TWO_PI - phi_max) / w)
        a_hi = np.where(hi[:, 0] <= TWO_PI, hi[:, 0] / w, np.mod(hi[:, 0], TWO_PI) / w)
        near = _frac_near(a_lo, tol[:, 0] / w) | _frac_near(a_hi, tol[:, 0] / w)
        near |= (np.abs(lo[:, 0]) <= tol[:, 0]) | (np.abs(hi[:, 0] - TWO_PI) <= tol[:, 0])
        b = np.asarray(sensor.elev_bounds, np.float64)
        for e, t in ((lo[:, 1], tol[:, 1]), (hi[:, 1], tol[:, 1])):
            near |= (np.abs(e[:, None] - b[None, :]) <= t[:, None]).any(1)
    else:
        near = np.zeros(lo.shape[0], bool)
        for k, T in ((0, sensor.tile_w), (1, sensor.tile_h)):
            near |= _frac_near(lo[:, k] / T, tol[:, k] / T) | _frac_near(hi[:, k] / T, tol[:, k] / T)
    return near


def check_rect_end_to_end(sp, g, sensor, k=0, first_record=0):
    """GPU rectangles of sensor k of a pass against the FP64 formulas on FP64 boxes.  Returns
    (compared, excluded near a border)."""
    n = g.n
    sl = slice(first_record + k * n, first_record + (k + 1) * n)
    nt = sp.ntiles.cpu().numpy()[sl]
    rect = sp.rect.cpu().numpy()[sl]
    pr = geo.project(geo.Params.from_gaussians(g), sensor)
    valid = pr.valid.numpy() & ~pr.near_cull.numpy()
    keep = nt > 0
    both = valid & keep
    lo, hi = pr.lo.detach().numpy(), pr.hi.detach().numpy()
    near = near_tile_border(pr, sensor)
    cmp_ = both & ~near
    if hasattr(sensor, "ray_az"):
        st, naz, e0, e1 = tl.lidar_tile_rect(lo, hi, sensor)
        want = np.stack([st, e0, naz, e1 - e0], 1)
    else:
        x0, x1, y0, y1 = tl.camera_tile_rect(lo, hi, sensor)
        want = np.stack([x0, y0, x1 - x0, y1 - y0], 1)
    bad = cmp_ & (rect != want).any(1)
    if bad.any():
        i = np.nonzero(bad)[0][:6]
        raise AssertionError(f"{int(bad.sum())} of {int(cmp_.sum())} rectangles differ from FP64; "
                             f"first ids {i.tolist()}: gpu {rect[i].tolist()} fp64 {want[i].tolist()}")
    # a record the library keeps with a non-empty FP64 rectangle is one the oracle keeps, and
    # vice versa, away from culling and border decisions
    np.testing.assert_array_equal(nt[cmp_], want[cmp_, 2] * want[cmp_, 3])
    n_near = int((both & near).sum())
    print(f"[tiles] {type(sensor).__name__}: {int(cmp_.sum())} rectangles equal to FP64, "
          f"{n_near} excluded near a tile border", flush=True)
    assert cmp_.sum() > 0.9 * both.sum()
    return int(cmp_.sum()), n_near


def _pass(b, cams, lids, g, k=0, count=1, batched=False):
    rig = b.Rig(cams, lids)
    G = b.GaussTensors.from_numpy(g)
    sp = b.SensorPass(rig, k, count, g.n, 1, batched=batched)
    sp.fit_capacity(G)
    return rig, G, sp


@pytest.mark.parametrize("tile", [(16, 16), (8, 32), (13, 7)])
def test_camera_rect_end_to_end(tile):
    b = _binding()
    rng = np.random.default_rng(31 + tile[0])
    mu = S.road_slab(rng, 40000, (0.5, 80.0), (-25.0, 25.0), 6.0)
    g = S.random_gaussians(rng, mu, 16, rgb=True, moving_frac=0.3)
    cam = S.make_camera((0, 0, 1.5), 4.0, 517, 301, 400.0, t_rs=0.03, ego_vel_world=(12.0, 0.5, 0.0),
                        ego_yaw_rate=0.2, n_channels=16, tile=tile)
    rig, G, sp = _pass(b, [cam], [], g)
    sp.project(G)
    torch.cuda.synchronize()
    check_rect_end_to_end(sp, g, cam)


def test_headline_rect_end_to_end():
    """The headline scene (2M Gaussians) in its batched form: both sensors' rectangles."""
    b = _binding()
    sc = S.headline()
    rig, G, sp = _pass(b, sc.cameras, sc.lidars, sc.gaussians, 0, 2, batched=True)
    sp.project(G)
    torch.cuda.synchronize()
    for k, sensor in enumerate(rig.sensors):
        check_rect_end_to_end(sp, sc.gaussians, sensor, k)


# ------------------------------------------------------------------------------------------
# the lidar seam
# ------------------------------------------------------------------------------------------
def seam_scene(seed, n_az, tile_az, beams=64, n=12000):
    """Gaussians across azimuth 0 (inside [-15, 15] deg, so the 360 - 364.8 deg overlap of a
    partial last tile is covered), a quarter uniform in azimuth, some near the sensor (boxes
    spanning many or all columns), 30 % moving; a rolling-shutter lidar moving at 12 m/s."""
    rng = np.random.default_rng(seed)
    m = n // 4
    az = np.concatenate([rng.uniform(-math.radians(15), math.radians(15), n - m), rng.uniform(0, TWO_PI, m)])
    r = np.concatenate([rng.uniform(2.0, 40.0, n - m), rng.uniform(0.6, 4.0, m)])
    el = rng.uniform(math.radians(-22), math.radians(12), n)
    mu = np.stack([r * np.cos(el) * np.cos(az), r * np.cos(el) * np.sin(az), r * np.sin(el)], 1)
    g = S.random_gaussians(rng, mu, 16, rgb=True, moving_frac=0.3, log_scale_mean=-1.2)
    lid = S.make_lidar((0, 0, 0), 0.0, beams, -25.0, 15.0, n_az, t_sweep=0.1, ego_vel_world=(12.0, 0, 0),
                       ego_yaw_rate=0.2, tile_az=tile_az, tile_el=8, feat_offset=3, n_channels=8, r_min=0.5)
    return g, lid


def seam_rays(lid):
    """Every ray of the first two and the last two azimuth tile columns."""
    cols = [0, 1, lid.n_az_tiles - 2, lid.n_az_tiles - 1]
    steps = np.concatenate([np.arange(c * lid.tile_az, min((c + 1) * lid.tile_az, lid.n_az)) for c in cols])
    beams = np.arange(lid.n_beams)
    return np.sort((beams[:, None] * lid.n_az + steps[None, :]).reshape(-1))


@pytest.mark.parametrize("n_az,tile_az", [(1800, 32), (300, 16)])
def test_lidar_seam_rects_and_render(n_az, tile_az):
    b = _binding()
    g, lid = seam_scene(700 + tile_az, n_az, tile_az)
    M = lid.n_az_tiles
    assert M * tile_az > n_az                         # the last tile is partial
    phi_max = M * tile_az * lid.az_res
    print(f"[seam] n_az {n_az}, N_phi {tile_az}: M_phi {M}, phi_max {math.degrees(phi_max):.2f} deg", flush=True)
    rig, G, sp = _pass(b, [], [lid], g)
    sp.project(G)
    torch.cuda.synchronize()
    # Gaussians inside the overlap and across 0 exist and are kept
    pr = geo.project(geo.Params.from_gaussians(g), lid)
    lo = pr.lo.detach().numpy()[:, 0]
    hi = pr.hi.detach().numpy()[:, 0]
    v = pr.valid.numpy()
    assert (v & (lo < 0)).sum() > 50 and (v & (hi > TWO_PI)).sum() > 20
    assert (v & (hi - lo >= TWO_PI)).sum() > 0 or (v & (hi - lo > 0.5 * TWO_PI)).sum() > 0
    # stage check (float32 formulas on the library's boxes) and end to end (FP64)
    keep = sp.ntiles.cpu().numpy() > 0
    rect = sp.rect.cpu().numpy()[keep]
    box = sp.box.cpu().numpy()[keep]
    st, naz, e0, e1 = tl.lidar_tile_rect_f32(box[:, :2], box[:, 2:], lid)
    np.testing.assert_array_equal(rect, np.stack([st, e0, naz, e1 - e0], 1))
    wraps = (rect[:, 0] + rect[:, 2] > M).sum()
    last_col = ((rect[:, 0] <= M - 1) & (rect[:, 0] + rect[:, 2] > M - 1)).sum()
    print(f"[seam] {int(keep.sum())} kept, {int(wraps)} rectangles wrap past the last column, "
          f"{int(last_col)} reach the last (partial) column", flush=True)
    assert wraps > 0 and last_col > 0
    check_rect_end_to_end(sp, g, lid)
    # every ray of the first two and last two columns, BOX and TILE
    idx = seam_rays(lid)
    for support, mode in ((0, "box"), (1, "tile")):
        sp.bin_sort()
        sp.raster_fwd(G, support)
        torch.cuda.synchronize()
        out = gpu_outputs(sp, 0)
        ref = rd.render_sensor(g, lid, idx, mode=mode)
        ok = ~ref["near"]
        print(f"[seam] {mode}: {len(idx)} rays, {int((~ok).sum())} near-decision rays excluded", flush=True)
        assert ok.mean() > 0.9
        for key in ("F", "D", "A", "median"):
            bad = rtol_check(out[key][idx], ref[key].detach().numpy(), 1e-4, 1e-5, ok)
            assert not bad.any(), (mode, key, int(bad.sum()))
        np.testing.assert_allclose(out["T"][idx][ok], ref["T"].numpy()[ok], rtol=1e-4, atol=1e-5)
        lid_ids = last_ids_gpu(sp, 0, lid, idx, out["last"][idx])
        assert np.array_equal(lid_ids[ok], ref["last_id"].numpy()[ok]), mode
        assert float(np.abs(ref["A"].numpy()).max()) > 0.5      # the columns are not empty
