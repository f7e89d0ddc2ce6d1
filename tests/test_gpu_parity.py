"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Bars: culling and tile assignment bit-exact under the library's documented float32 arithmetic
(stage check) and within near-threshold exclusions end to end; sorted per-tile lists
bit-exact; rendered features / depth / opacity / median within 1e-5 + 1e-4 |ref| per element on
rays with no near-threshold decision; gradients within 1e-3 relative (per tensor, and per
element with atol = 1e-5 max |ref|)."""
import math

import numpy as np
import pytest
import torch

from oracle import geometry as geo
from oracle import grad as ogr
from oracle import render as rd
from oracle import tiles as tl
from scenes import synthetic as S
from tests.gpu_helpers import grad_mismatch, assert_grad_close, gpu_outputs, last_ids_gpu, rtol_check, tile_lists_gpu

pytestmark = pytest.mark.gpu


def _binding():
    from paper_2411_16816_amd import binding
    binding.load()
    return binding


# ------------------------------------------------------------------------------------------
# scenes (seeded)
# ------------------------------------------------------------------------------------------
def cam_scene(seed=101, n=20000, W=333, H=245, tile=(16, 16), t_rs=0.03):
    rng = np.random.default_rng(seed)
    mu = S.road_slab(rng, n, (0.5, 60.0), (-20.0, 20.0), 6.0)
    g = S.random_gaussians(rng, mu, 16, rgb=True, moving_frac=0.3)
    cam = S.make_camera((0, 0, 1.5), 3.0, W, H, 250.0, t_rs=t_rs, ego_vel_world=(12.0, 0.5, 0.0),
                        ego_yaw_rate=0.2, n_channels=16, tile=tile)
    return g, cam


def lidar_rs_scene(seed=102, n=3000):
    rng = np.random.default_rng(seed)
    mu = S.uniform_box(rng, n, (-30, -30, -3), (30, 30, 3))
    g = S.random_gaussians(rng, mu, 16, rgb=True, moving_frac=0.3)
    lid = S.make_lidar((0, 0, 0), 7.0, 32, -25.0, 15.0, 512, t_sweep=0.1, ego_vel_world=(15.0, 0, 0),
                       ego_yaw_rate=0.3, feat_offset=3, n_channels=8)
    return g, lid


def _pass(cams, lids, g, k=0, count=1, margin=1.2):
    b = _binding()
    rig = b.Rig(cams, lids)
    G = b.GaussTensors.from_numpy(g)
    sp = b.SensorPass(rig, k, count, g.n, k_cap=1)
    sp.fit_capacity(G, margin)
    return rig, G, sp


# ------------------------------------------------------------------------------------------
# a1 / a2: projection
# ------------------------------------------------------------------------------------------
def _check_projection(sp, g, sensor):
    torch.cuda.synchronize()
    nt = sp.ntiles.cpu().numpy()
    keep = nt > 0
    pr = geo.project(geo.Params.from_gaussians(g), sensor)
    valid = pr.valid.numpy()
    lo, hi = pr.lo.detach().numpy(), pr.hi.detach().numpy()
    # box edge within 1e-5 relative of the domain edge: culling may legitimately differ
    if hasattr(sensor, "ray_az"):
        b = sensor.elev_bounds.astype(np.float64)
        edge = np.minimum(np.abs(hi[:, 1] - b[0]), np.abs(lo[:, 1] - b[-1]))
        near = pr.near_cull.numpy() | (edge <= 1e-5)
    else:
        edge = np.minimum.reduce([np.abs(hi[:, 0]), np.abs(lo[:, 0] - sensor.width),
                                  np.abs(hi[:, 1]), np.abs(lo[:, 1] - sensor.height)])
        near = pr.near_cull.numpy() | (edge <= 1e-2)
    mism = (keep != valid) & ~near
    assert mism.sum() == 0, f"{mism.sum()} culling mismatches"
    both = keep & valid
    assert both.sum() > 0.5 * valid.sum()
    mv = sp.mv.cpu().numpy()[both]
    cn = sp.cn.cpu().numpy()[both]
    bx = sp.box.cpu().numpy()[both]
    dv = sp.dv.cpu().numpy()[both]
    ref = dict(mean=pr.mean2d.detach().numpy()[both], vel=pr.vel2d.detach().numpy()[both],
               conic=pr.conic.detach().numpy()[both], o=pr.o_eff.detach().numpy()[both],
               lo=lo[both], hi=hi[both], depth=pr.depth.detach().numpy()[both], vr=pr.v_r.detach().numpy()[both])
    got = dict(mean=mv[:, :2], vel=mv[:, 2:], conic=cn[:, :3], o=cn[:, 3], lo=bx[:, :2], hi=bx[:, 2:],
               depth=dv[:, 0], vr=dv[:, 1])
    for k in ref:
        scale = max(1e-12, float(np.abs(ref[k]).max()))
        bad = rtol_check(got[k], ref[k], rtol=2e-5, atol=2e-6 * scale)
        if bad.any():
            i = np.argwhere(bad)[:6]
            rows = [(tuple(int(v) for v in ix), float(got[k][tuple(ix)]), float(ref[k][tuple(ix)])) for ix in i]
            raise AssertionError(f"projection {k}: {int(bad.sum())} of {bad.size} elements beyond 2e-5 relative "
                                 f"/ 2e-6 of the largest; first: {rows}")
    # stage check: tile rectangles bit-exact with the documented float32 arithmetic
    rect = sp.rect.cpu().numpy()[keep]
    gb = sp.box.cpu().numpy()[keep]
    if hasattr(sensor, "ray_az"):
        st, naz, e0, e1 = tl.lidar_tile_rect_f32(gb[:, :2], gb[:, 2:], sensor)
        np.testing.assert_array_equal(rect[:, 0], st)
        np.testing.assert_array_equal(rect[:, 1], e0)
        np.testing.assert_array_equal(rect[:, 2], naz)
        np.testing.assert_array_equal(rect[:, 3], e1 - e0)
    else:
        x0, x1, y0, y1 = tl.camera_tile_rect_f32(gb[:, :2], gb[:, 2:], sensor)
        np.testing.assert_array_equal(rect, np.stack([x0, y0, x1 - x0, y1 - y0], 1))
    np.testing.assert_array_equal(nt[keep], rect[:, 2] * rect[:, 3])
    return keep


def test_project_camera():
    g, cam = cam_scene()
    rig, G, sp = _pass([cam], [], g)
    _check_projection(sp, g, cam)


def test_project_lidar():
    g, lid = lidar_rs_scene()
    rig, G, sp = _pass([], [lid], g)
    _check_projection(sp, g, lid)


# ------------------------------------------------------------------------------------------
# a3 / a4: binning and sorting, bit-exact against the stage check
# ------------------------------------------------------------------------------------------
def depth_sort_key(bits):
    """The library's documented 32-bit ordering key of float64 depth bits (splat.h, dkey)."""
    bits = np.asarray(bits, np.uint64)
    e = ((bits >> np.uint64(52)) & np.uint64(0x7FF)).astype(np.int64) - (1023 - 16)
    key = (np.clip(e, 0, 31).astype(np.uint64) << np.uint64(27)) | ((bits & np.uint64(0xFFFFFFFFFFFFF)) >> np.uint64(25))
    key = np.where(e < 0, np.uint64(0), key)
    return np.where(e > 31, np.uint64((1 << 32) - 1), key)


def ray_cell_codes_f32(lid, n_bins):
    """The library's documented order of rays inside a lidar tile (splat_common.hpp,
    ray_cell_code; binsort.hip, ray_cell_bits): the rest of the bin's last 8-bit radix digit holds
    a Z-order cell code of the ray inside its tile, computed in float32."""
    F = np.float32
    bin_bits = max(1, int(np.ceil(np.log2(n_bins))))
    c = (8 - bin_bits % 8) % 8
    ab, eb = (c + 1) // 2, c // 2
    az = np.asarray(lid.ray_az, F)
    el = np.asarray(lid.ray_el, F)
    u = (az / tl.lidar_tile_width_f32(lid)).astype(F)
    fa = (u - np.floor(u)).astype(F)
    b = np.asarray(lid.elev_bounds, F)
    e = np.clip(np.searchsorted(b, el, side="right") - 1, 0, b.shape[0] - 2)
    fe = ((el - b[e]).astype(F) / (b[e + 1] - b[e]).astype(F)).astype(F)
    qa = np.clip(np.trunc((fa * F(1 << ab)).astype(F)).astype(np.int64), 0, (1 << ab) - 1)
    qe = np.clip(np.trunc((fe * F(1 << eb)).astype(F)).astype(np.int64), 0, (1 << eb) - 1)
    z = np.zeros_like(qa)
    for i in range(ab):
        z |= ((qa >> i) & 1) << (2 * i)
    for i in range(eb):
        z |= ((qe >> i) & 1) << (2 * i + 1)
    return z


def _expected_lists(sp, sensor, g_n):
    nt = sp.ntiles.cpu().numpy()[:g_n]
    keep = nt > 0
    box = sp.box.cpu().numpy()[:g_n]
    depth = depth_sort_key(sp.dkey.cpu().numpy()[:g_n].view(np.uint64))
    if hasattr(sensor, "ray_az"):
        rect = tl.lidar_tile_rect_f32(box[:, :2], box[:, 2:], sensor)
        per = tl.lidar_tiles_of(rect, sensor)
        n_t = sensor.n_az_tiles * sensor.n_el_tiles
    else:
        rect = tl.camera_tile_rect_f32(box[:, :2], box[:, 2:], sensor)
        per = tl.camera_tiles_of(rect, sensor)
        n_t = (-(-sensor.width // sensor.tile_w)) * (-(-sensor.height // sensor.tile_h))
    per = [p if k else [] for p, k in zip(per, keep)]
    return tl.tile_lists(per, depth, keep, n_t)


@pytest.mark.parametrize("kind", ["camera", "camera_256_supertiles", "camera_many_supertiles", "lidar"])
def test_bin_sort_bit_exact(kind):
    if kind == "camera":
        g, sensor = cam_scene(n=8000)
        rig, G, sp = _pass([sensor], [], g)
    elif kind == "camera_256_supertiles":
        # 128 x 128 tiles of 4 x 4 pixels: 16 x 16 = 256 supertiles, every digit of the one-pass
        # supertile sort in use
        g, sensor = cam_scene(n=8000, W=512, H=512, tile=(4, 4))
        rig, G, sp = _pass([sensor], [], g)
    elif kind == "camera_many_supertiles":
        # 200 x 150 tiles of 8 x 8 pixels: 25 x 19 = 475 supertiles, more than one radix digit, so
        # the supertile sort takes two passes and a separate ranges pass (6 supertiles above: one
        # pass whose scatter writes the ranges)
        g, sensor = cam_scene(n=8000, W=1600, H=1200, tile=(8, 8))
        rig, G, sp = _pass([sensor], [], g)
    else:
        g, sensor = lidar_rs_scene()
        rig, G, sp = _pass([], [sensor], g)
    sp.render(G)
    torch.cuda.synchronize()
    st = _binding().read_status(sp.status)
    assert st.overflow == 0 and st.n_isect > 0
    want = _expected_lists(sp, sensor, g.n)
    got = tile_lists_gpu(sp)
    assert sum(len(x) for x in want) == st.n_isect
    assert got == want
    if kind == "lidar":
        a, e, v = tl.lidar_ray_tiles_f32(sensor.ray_az, sensor.ray_el, sensor)
        tiles = np.where(v, e * sensor.n_az_tiles + a, sensor.n_az_tiles * sensor.n_el_tiles)
        order = sp.ray_order.cpu().numpy()[:sensor.n_rays]
        rr = sp.ray_range.cpu().numpy()
        code = ray_cell_codes_f32(sensor, sensor.n_az_tiles * sensor.n_el_tiles + 1)
        for t in range(rr.shape[0]):
            ids = order[rr[t, 0]:rr[t, 1]]
            want_ids = np.nonzero(tiles == t)[0]
            c = np.where(t < sensor.n_az_tiles * sensor.n_el_tiles, code[want_ids], 0)
            np.testing.assert_array_equal(ids, want_ids[np.lexsort((want_ids, c))])
        nw = int(sp.n_work.cpu()[0])
        work = sp.work.cpu().numpy()[:nw]
        counts = rr[:, 1] - rr[:, 0]
        assert nw == int(np.sum((counts + 255) // 256))


def test_overflow_is_reported_and_safe():
    g, cam = cam_scene(n=4000)
    b = _binding()
    rig = b.Rig([cam], [])
    G = b.GaussTensors.from_numpy(g)
    sp = b.SensorPass(rig, 0, 1, g.n, k_cap=1000)
    sp.status.zero_()
    sp.render(G)
    torch.cuda.synchronize()
    st = b.read_status(sp.status)
    assert st.overflow == 1 and st.n_isect > 1000 and st.k_cap == 1000
    assert int(sp.tile_range.max()) <= 1000


# ------------------------------------------------------------------------------------------
# a5 / a6: forward rendering
# ------------------------------------------------------------------------------------------
def _compare_render(sp, k, sensor, g, ray_idx, support=0, out=None):
    gout = gpu_outputs(sp, k)
    ref = rd.render_sensor(g, sensor, ray_idx, mode="box" if support == 0 else "tile")
    near = ref["near"]
    ok = ~near
    assert near.mean() < 0.05, near.mean()
    for key in ("F", "D", "A"):
        a = gout[key][ray_idx]
        r = ref[key].detach().numpy()
        bad = rtol_check(a, r, 1e-4, 1e-5, ok)
        assert not bad.any(), (key, int(bad.sum()))
    np.testing.assert_allclose(gout["T"][ray_idx][ok], ref["T"].numpy()[ok], rtol=1e-4, atol=1e-5)
    if "median" in gout:
        bad = rtol_check(gout["median"][ray_idx], ref["median"].numpy(), 1e-4, 1e-5, ok)
        assert not bad.any()
    lid = last_ids_gpu(sp, k, sensor, ray_idx, gout["last"][ray_idx])
    assert np.array_equal(lid[ok], ref["last_id"].numpy()[ok])
    return ref


def test_forward_lidar_config1_all_rays():
    sc = S.config_1()
    lid = sc.lidars[0]
    rig, G, sp = _pass([], [lid], sc.gaussians)
    sp.render(G)
    torch.cuda.synchronize()
    _compare_render(sp, 0, lid, sc.gaussians, np.arange(lid.n_rays))


def test_forward_lidar_rolling_shutter():
    g, lid = lidar_rs_scene()
    rig, G, sp = _pass([], [lid], g)
    sp.render(G)
    torch.cuda.synchronize()
    _compare_render(sp, 0, lid, g, np.arange(0, lid.n_rays, 3))


def test_forward_lidar_near_sensor_fast_motion():
    """Gaussians 0.35-3 m from a lidar moving at 60 m/s: their azimuth velocities reach hundreds
    of rad/s, so the rolling-shutter shift v t spans several turns and the azimuth difference
    must be reduced modulo 2 pi."""
    rng = np.random.default_rng(103)
    n = 600
    r = rng.uniform(0.35, 3.0, n)
    az = rng.uniform(0, 2 * np.pi, n)
    mu = np.stack([r * np.cos(az), r * np.sin(az), rng.uniform(-0.8, 0.8, n)], 1)
    g = S.random_gaussians(rng, mu, 16, rgb=True, moving_frac=0.3, log_scale_mean=-1.5)
    lid = S.make_lidar((0, 0, 0), 0.0, 32, -25.0, 15.0, 512, t_sweep=0.1, ego_vel_world=(60.0, 0, 0),
                       ego_yaw_rate=0.5, feat_offset=3, n_channels=8, r_min=0.3)
    pr = geo.project(geo.Params.from_gaussians(g), lid)
    assert float((pr.vel2d[:, 0].abs() * 0.05).max()) > 2 * math.pi   # shifts beyond a full turn exist
    rig, G, sp = _pass([], [lid], g)
    sp.render(G)
    torch.cuda.synchronize()
    _compare_render(sp, 0, lid, g, np.arange(0, lid.n_rays, 2))


@pytest.mark.parametrize("tile", [(16, 16), (32, 8), (8, 8)])
def test_forward_camera_ragged(tile):
    g, cam = cam_scene(n=12000, tile=tile)
    rig, G, sp = _pass([cam], [], g)
    sp.render(G)
    torch.cuda.synchronize()
    idx = np.arange(0, cam.n_rays, 7)
    _compare_render(sp, 0, cam, g, idx)


def test_forward_tile_mode():
    g, cam = cam_scene(n=3000, W=96, H=80)
    rig, G, sp = _pass([cam], [], g)
    sp.render(G, support=1)
    torch.cuda.synchronize()
    _compare_render(sp, 0, cam, g, np.arange(cam.n_rays), support=1)


def test_box_result_independent_of_tile_shape():
    outs = []
    for tile in [(16, 16), (32, 8), (8, 32), (8, 8)]:
        g, cam = cam_scene(n=6000, tile=tile)
        rig, G, sp = _pass([cam], [], g)
        sp.render(G)
        torch.cuda.synchronize()
        o = gpu_outputs(sp, 0)
        outs.append(o)
    for o in outs[1:]:
        for k in ("F", "D", "A", "T"):
            np.testing.assert_array_equal(o[k], outs[0][k])


def test_empty_scene_and_invalid_rays():
    g, cam = cam_scene(n=500)
    g.means[:, 0] = -np.abs(g.means[:, 0]) - 1.0          # everything behind the camera
    rig, G, sp = _pass([cam], [], g)
    sp.render(G)
    torch.cuda.synchronize()
    o = gpu_outputs(sp, 0)
    assert np.all(o["F"] == 0) and np.all(o["A"] == 0) and np.all(o["T"] == 1)
    g2, lid = lidar_rs_scene(n=500)
    lid.ray_el = lid.ray_el.copy()
    lid.ray_el[:100] = np.float32(1.2)                     # far above the top boundary
    lid.ray_az = lid.ray_az.copy()
    lid.ray_az[100:150] = np.float32(7.0)                  # outside [0, 2pi)
    rig, G, sp = _pass([], [lid], g2)
    sp.status.zero_()
    sp.render(G)
    torch.cuda.synchronize()
    st = _binding().read_status(sp.status)
    assert st.n_rays_invalid == 150
    o = gpu_outputs(sp, 0)
    assert np.all(o["F"][:150] == 0) and np.all(o["A"][:150] == 0) and np.all(o["D"][:150] == 0)


def test_batched_equals_plain():
    g, cam = cam_scene(n=6000)
    cam2 = S.make_camera((0, 0, 1.5), -25.0, 200, 130, 180.0, t_rs=0.02, ego_vel_world=(10.0, 0, 0), n_channels=16)
    b = _binding()
    rig = b.Rig([cam, cam2], [])
    G = b.GaussTensors.from_numpy(g)
    both = b.SensorPass(rig, 0, 2, g.n, 1)
    both.fit_capacity(G)
    both.render(G)
    plain = []
    for k in range(2):
        sp = b.SensorPass(rig, k, 1, g.n, 1)
        sp.fit_capacity(G)
        sp.render(G)
        plain.append(sp)
    torch.cuda.synchronize()
    for k in range(2):
        a = gpu_outputs(both, k)
        p = gpu_outputs(plain[k], 0)
        for key in ("F", "D", "A", "T", "last"):
            np.testing.assert_array_equal(a[key], p[key])
    g2, lid = lidar_rs_scene()
    lid2 = S.make_lidar((1.0, 2.0, 0), -40.0, 16, -20.0, 10.0, 300, t_sweep=0.1, ego_vel_world=(8.0, 0, 0),
                        tile_az=16, feat_offset=3, n_channels=8)
    rig = b.Rig([], [lid, lid2])
    G = b.GaussTensors.from_numpy(g2)
    both = b.SensorPass(rig, 0, 2, g2.n, 1)
    both.fit_capacity(G)
    both.render(G)
    for k in range(2):
        sp = b.SensorPass(rig, k, 1, g2.n, 1)
        sp.fit_capacity(G)
        sp.render(G)
        torch.cuda.synchronize()
        a = gpu_outputs(both, k)
        p = gpu_outputs(sp, 0)
        for key in ("F", "D", "A", "T", "last", "median"):
            np.testing.assert_array_equal(a[key], p[key])


def test_batched_few_gaussians_many_work_items():
    """A batched call whose work items outnumber its records and its list capacity (40
    Gaussians, a 1920x1080 camera of 8160 tiles and a small one): the queue's sort still fits
    the workspace, every camera tile is queued once, and the forward equals the per-sensor
    calls.  A batched call over the big camera alone runs the per-sensor kernels: same result."""
    b = _binding()
    g, _ = cam_scene(n=40)
    cam = S.make_camera((0, 0, 1.5), 3.0, 1920, 1080, 1400.0, t_rs=0.03, ego_vel_world=(12.0, 0.5, 0.0),
                        n_channels=16)
    cam2 = S.make_camera((0, 0, 1.5), -25.0, 200, 130, 180.0, t_rs=0.02, ego_vel_world=(10.0, 0, 0), n_channels=16)
    rig = b.Rig([cam, cam2], [])
    G = b.GaussTensors.from_numpy(g)
    bat = b.SensorPass(rig, 0, 2, g.n, 1, batched=True)
    bat.fit_capacity(G)
    assert bat.k_cap < bat.n_tiles and 2 * g.n < bat.n_tiles
    bat.render(G)
    one = b.SensorPass(rig, 0, 1, g.n, 1, batched=True)
    one.fit_capacity(G)
    one.render(G)
    torch.cuda.synchronize()
    assert b.read_status(bat.status).overflow == 0
    nw = int(bat.n_work.cpu()[0])
    work = bat.work.cpu().numpy()[:nw]
    assert sorted(work[:, 0].tolist()) == list(range(bat.n_tiles))
    for k in range(2):
        sp = b.SensorPass(rig, k, 1, g.n, 1)
        sp.fit_capacity(G)
        sp.render(G)
        torch.cuda.synchronize()
        p_ = gpu_outputs(sp, 0)
        if k == 0:
            assert np.any(p_["A"] > 0)
        for got in ([bat, k], [one, 0]) if k == 0 else ([bat, k],):
            a_ = gpu_outputs(*got)
            for key in ("F", "D", "A", "T", "last"):
                np.testing.assert_array_equal(a_[key], p_[key])


def queue_length_code(lens):
    """The library's documented queue bucket of a list length (binsort.hip, length_code):
    4 bits of binary exponent and 4 bits of mantissa of min(len, 2^20 - 1) + 1."""
    x = np.minimum(np.asarray(lens, np.int64), 0xFFFFF) + 1
    e = np.floor(np.log2(x)).astype(np.int64)
    m = np.where(e >= 4, (x >> np.maximum(e - 4, 0)) & 15, (x << np.maximum(4 - e, 0)) & 15)
    return np.minimum((e << 4) | m, 255)


def test_batched_queue_equals_plain():
    """Batched form (cameras and lidars in one call, persistent queue) against per-sensor calls:
    forward bit-identical, adjoint equal up to float atomic order."""
    b = _binding()
    g, cam = cam_scene(n=8000)
    cam2 = S.make_camera((0, 0, 1.5), -25.0, 200, 130, 180.0, t_rs=0.02, ego_vel_world=(10.0, 0, 0), n_channels=16)
    _, lid = lidar_rs_scene()
    lid2 = S.make_lidar((1.0, 2.0, 0), -40.0, 16, -20.0, 10.0, 300, t_sweep=0.1, ego_vel_world=(8.0, 0, 0),
                        tile_az=16, feat_offset=3, n_channels=8)
    rig = b.Rig([cam, cam2], [lid, lid2])
    G = b.GaussTensors.from_numpy(g)
    bat = b.SensorPass(rig, 0, 4, g.n, 1, batched=True)
    bat.fit_capacity(G)
    bat.render(G)
    torch.cuda.synchronize()
    assert b.read_status(bat.status).overflow == 0
    # queue: every camera tile once, every lidar ray in exactly one item, longest lists first
    nw = int(bat.n_work.cpu()[0])
    work = bat.work.cpu().numpy()[:nw]
    tr = bat.tile_range.cpu().numpy()
    lens = np.array([tr[t, 1] - tr[t, 0] if t < bat.n_tiles else 0 for t in work[:, 0]])
    n_cam_tiles = int(rig.tile_base[2])
    is_cam = work[:, 0] < n_cam_tiles
    assert np.all(is_cam[:-1] <= is_cam[1:])   # the lidar items, then the camera items
    for part in (~is_cam, is_cam):   # grouped form (the adjoint keeps rows): by cost inside each kind
        assert np.all(np.diff(queue_length_code(lens[part]) >> 1) <= 0)
    assert sorted(work[work[:, 0] < n_cam_tiles, 0].tolist()) == list(range(n_cam_tiles))
    R = bat.n_rays
    up = np.random.default_rng(3)
    dF = torch.from_numpy(up.normal(size=bat.n_feat).astype(np.float32)).cuda()
    dD = torch.from_numpy((0.1 * up.normal(size=R)).astype(np.float32)).cuda()
    dA = torch.from_numpy(up.normal(size=R).astype(np.float32)).cuda()
    gb = b.zeros_like_grads(G)
    bat.raster_bwd(G, dF, dD, dA, gb)
    gp = b.zeros_like_grads(G)
    for k in range(4):
        sp = b.SensorPass(rig, k, 1, g.n, 1)
        sp.fit_capacity(G)
        sp.render(G)
        rs, fs, C = bat.sensor_slices(k)
        sp.raster_bwd(G, dF[fs].contiguous(), dD[rs].contiguous(), dA[rs].contiguous(), gp)
        torch.cuda.synchronize()
        a_ = gpu_outputs(bat, k)
        p_ = gpu_outputs(sp, 0)
        for key in ("F", "D", "A", "T", "last"):
            np.testing.assert_array_equal(a_[key], p_[key])
        if "median" in p_:
            np.testing.assert_array_equal(a_["median"], p_["median"])
    for name in ("means", "log_scales", "quats", "opacities", "velocities", "features"):
        x = getattr(gb, name).cpu().numpy().astype(np.float64)
        y = getattr(gp, name).cpu().numpy().astype(np.float64)
        assert np.linalg.norm(x - y) <= 1e-5 * np.linalg.norm(y), name


@pytest.mark.parametrize("kind", ["camera", "lidar"])
def test_batched_single_kind_queue_equals_plain(kind):
    """A batched call over two sensors of one kind runs the queue kernels compiled for that kind
    alone (camera-only adjoint at 4 waves per SIMD; lidar-only): forward bit-identical to the
    per-sensor calls, gradients equal up to float atomic order."""
    b = _binding()
    if kind == "camera":
        g, s1 = cam_scene(n=6000)
        s2 = S.make_camera((0, 0, 1.5), -25.0, 200, 130, 180.0, t_rs=0.02, ego_vel_world=(10.0, 0, 0), n_channels=16)
        rig = b.Rig([s1, s2], [])
    else:
        g, s1 = lidar_rs_scene()
        s2 = S.make_lidar((1.0, 2.0, 0), -40.0, 16, -20.0, 10.0, 300, t_sweep=0.1, ego_vel_world=(8.0, 0, 0),
                          tile_az=16, feat_offset=3, n_channels=8)
        rig = b.Rig([], [s1, s2])
    G = b.GaussTensors.from_numpy(g)
    bat = b.SensorPass(rig, 0, 2, g.n, 1, batched=True)
    bat.fit_capacity(G)
    bat.render(G)
    up = np.random.default_rng(5)
    dF = torch.from_numpy(up.normal(size=bat.n_feat).astype(np.float32)).cuda()
    dD = torch.from_numpy((0.1 * up.normal(size=bat.n_rays)).astype(np.float32)).cuda()
    dA = torch.from_numpy(up.normal(size=bat.n_rays).astype(np.float32)).cuda()
    gb = b.zeros_like_grads(G)
    bat.raster_bwd(G, dF, dD, dA, gb)
    gp = b.zeros_like_grads(G)
    for k in range(2):
        sp = b.SensorPass(rig, k, 1, g.n, 1)
        sp.fit_capacity(G)
        sp.render(G)
        rs, fs, C = bat.sensor_slices(k)
        sp.raster_bwd(G, dF[fs].contiguous(), dD[rs].contiguous(), dA[rs].contiguous(), gp)
        torch.cuda.synchronize()
        a_ = gpu_outputs(bat, k)
        p_ = gpu_outputs(sp, 0)
        for key in ("F", "D", "A", "T", "last"):
            np.testing.assert_array_equal(a_[key], p_[key])
    for name in ("means", "log_scales", "quats", "opacities", "velocities", "features"):
        x = getattr(gb, name).cpu().numpy().astype(np.float64)
        y = getattr(gp, name).cpu().numpy().astype(np.float64)
        assert np.linalg.norm(y) > 0, name
        assert np.linalg.norm(x - y) <= 1e-5 * np.linalg.norm(y), name


# ------------------------------------------------------------------------------------------
# a7: adjoint
# ------------------------------------------------------------------------------------------
def _grad_check(kind, seed, lidar_tile_az=16):
    b = _binding()
    rng = np.random.default_rng(seed)
    if kind == "camera":
        sensor = S.make_camera((0, 0, 0), 0.0, 64, 48, 60.0, t_rs=0.04, ego_vel_world=(6.0, 0.5, 0),
                               ego_yaw_rate=0.3, n_channels=16)
        n = 250
        mu = np.stack([rng.uniform(2, 12, n), rng.uniform(-5, 5, n), rng.uniform(-3.5, 3.5, n)], 1)
        rig = b.Rig([sensor], [])
    else:
        sensor = S.make_lidar((0, 0, 0), 0.0, 16, -15.0, 15.0, 256, tile_az=lidar_tile_az, tile_el=8, t_sweep=0.1,
                              ego_vel_world=(10.0, 1.0, 0), feat_offset=3, n_channels=8)
        n = 300
        mu = np.stack([rng.uniform(-10, 10, n), rng.uniform(-10, 10, n), rng.uniform(-1.5, 1.5, n)], 1)
        rig = b.Rig([], [sensor])
    g = S.random_gaussians(rng, mu, 16, rgb=True, moving_frac=0.5, log_scale_mean=-0.6)
    G = b.GaussTensors.from_numpy(g)
    sp = b.SensorPass(rig, 0, 1, g.n, 1)
    sp.fit_capacity(G)
    sp.render(G)
    if kind != "camera":
        # bin_sort's split flag (n_work[2]): set exactly when a tile holds more than 256 rays; the
        # adjoint clears the lidar records' atomic accumulators only then
        torch.cuda.synchronize()
        rr = sp.ray_range.cpu().numpy().reshape(-1, 2)[:-1]
        split = int(np.any(rr[:, 1] - rr[:, 0] > 256))
        assert split == (1 if lidar_tile_az * 8 > 256 else 0)
        assert int(sp.n_work.cpu()[2]) == split
    R = sensor.n_rays
    C = sensor.n_channels
    up = np.random.default_rng(seed + 1)
    dF = up.normal(size=(R, C)).astype(np.float32)
    dD = (0.1 * up.normal(size=R)).astype(np.float32)
    dA = up.normal(size=R).astype(np.float32)
    grads = b.zeros_like_grads(G)
    t = lambda a: torch.from_numpy(a.reshape(-1)).cuda()
    sp.raster_bwd(G, t(dF), t(dD), t(dA), grads)
    torch.cuda.synchronize()
    ref, out = ogr.reference_grads(g, sensor, np.arange(R), dF, dD, dA)
    near = out["near"]
    assert near.mean() < 0.05
    # the reference gradient counts every ray; re-run excluding near-decision rays on both sides
    if near.any():
        keep = ~near
        dF2, dD2, dA2 = dF * keep[:, None], dD * keep, dA * keep
        ref, _ = ogr.reference_grads(g, sensor, np.arange(R), dF2, dD2, dA2)
        grads = b.zeros_like_grads(G)
        sp.raster_bwd(G, t(dF2.astype(np.float32)), t(dD2.astype(np.float32)), t(dA2.astype(np.float32)), grads)
        torch.cuda.synchronize()
    got = dict(means=grads.means, log_scales=grads.log_scales, quats=grads.quats, opacities=grads.opacities,
               velocities=grads.velocities, features=grads.features)
    for name in geo.Params.names:
        assert_grad_close(got[name].cpu().numpy(), ref[name], f"{kind} {name}")


def test_backward_camera():
    _grad_check("camera", 7)


def test_backward_lidar():
    _grad_check("lidar", 8)


def test_backward_lidar_split_tiles():
    """64 x 8 = 512 rays per tile: every tile is two work items, whose gradients add atomically."""
    _grad_check("lidar", 9, lidar_tile_az=64)


def test_split_tile_atomics_match_fixed_order():
    """The adjoint's atomic path (lidar tiles of 512 rays, two work items each, adding their
    per-Gaussian rows with global atomics) against its fixed-order path (tiles of 128 rays, one
    item each, rows summed in a fixed order) on the same rays and Gaussians: the rendered
    outputs are identical (the tile layout only changes the candidate search) and the gradients
    agree to rounding.  Two runs of the atomic path agree to rounding as well."""
    b = _binding()
    rng = np.random.default_rng(23)
    n = 2000
    mu = np.stack([rng.uniform(-12, 12, n), rng.uniform(-12, 12, n), rng.uniform(-1.5, 1.5, n)], 1)
    g = S.random_gaussians(rng, mu, 16, rgb=True, moving_frac=0.5, log_scale_mean=-0.6)
    G = b.GaussTensors.from_numpy(g)
    up = np.random.default_rng(24)
    runs = []
    for tile_az in (16, 64, 64):
        lid = S.make_lidar((0, 0, 0), 0.0, 16, -15.0, 15.0, 256, tile_az=tile_az, tile_el=8, t_sweep=0.1,
                           ego_vel_world=(10.0, 1.0, 0), feat_offset=3, n_channels=8)
        rays_per_tile = tile_az * 8
        print(f"[split] tile_az {tile_az}: {rays_per_tile} rays per tile", flush=True)
        rig = b.Rig([], [lid])
        sp = b.SensorPass(rig, 0, 1, g.n, 1)
        sp.fit_capacity(G)
        sp.render(G)
        if not runs:
            R, C = lid.n_rays, lid.n_channels
            ups = [torch.from_numpy(a).cuda() for a in (up.normal(size=R * C).astype(np.float32),
                                                        (0.1 * up.normal(size=R)).astype(np.float32),
                                                        up.normal(size=R).astype(np.float32))]
        grads = b.zeros_like_grads(G)
        sp.raster_bwd(G, *ups, grads)
        torch.cuda.synchronize()
        runs.append((gpu_outputs(sp, 0), {name: getattr(grads, name).cpu().numpy() for name in geo.Params.names}))
    (o_ref, g_ref), (o_split, g_split), (o_again, g_again) = runs
    for key in ("F", "D", "A", "T"):
        np.testing.assert_array_equal(o_split[key], o_ref[key], err_msg=key)
        np.testing.assert_array_equal(o_again[key], o_ref[key], err_msg=key)
    for name in geo.Params.names:
        assert np.abs(g_ref[name]).max() > 0, name
        for other in (g_split, g_again):
            bad = grad_mismatch(other[name], g_ref[name], rtol=1e-4, afloor=1e-5)
            assert not bad.any(), (name, int(bad.sum()))


def test_adjoint_after_row_limit_change_between_calls():
    """bin/sort orders the persistent queue by the adjoint row limit of its own call (grouped by
    kind with rows, one mixed cost order without).  An adjoint run after the limit changed,
    on lists binned under the other limit, must still render every work item: the rig remembers
    each lists' queue order and the adjoint picks its kernel by it.  Gradients match a run that
    kept the default limit throughout."""
    b = _binding()
    rng = np.random.default_rng(33)
    n = 3000
    mu = np.stack([rng.uniform(2, 30, n), rng.uniform(-12, 12, n), rng.uniform(-2, 2, n)], 1)
    g = S.random_gaussians(rng, mu, 19, rgb=True, moving_frac=0.5, log_scale_mean=-0.6)
    G = b.GaussTensors.from_numpy(g)
    cam = S.make_camera((0, 0, 0), 0.0, 200, 120, 150.0, t_rs=0.03, ego_vel_world=(3.0, 0, 0), n_channels=16)
    lid = S.make_lidar((0, 0, 0), 0.0, 16, -15.0, 15.0, 256, tile_az=16, tile_el=8, t_sweep=0.1,
                       ego_vel_world=(10.0, 1.0, 0), feat_offset=3, n_channels=8)
    rig = b.Rig([cam], [lid])
    up = np.random.default_rng(34)
    grads, outs = [], []
    try:
        for binned_without_rows in (False, True):
            b.set_adjoint_row_limit(b.ADJOINT_ROW_LIMIT)
            sp = b.SensorPass(rig, 0, 2, g.n, 1, batched=True)
            sp.fit_capacity(G)   # workspace sized with rows
            if binned_without_rows:
                b.set_adjoint_row_limit(0)   # this bin/sort builds the mixed queue order
            sp.render(G)
            b.set_adjoint_row_limit(b.ADJOINT_ROW_LIMIT)   # the adjoint keeps rows
            if not grads:
                ups = [torch.from_numpy(a).cuda() for a in (
                    up.normal(size=sp.n_feat).astype(np.float32),
                    (0.1 * up.normal(size=sp.n_rays)).astype(np.float32),
                    up.normal(size=sp.n_rays).astype(np.float32))]
            gr = b.zeros_like_grads(G)
            sp.raster_bwd(G, *ups, gr)
            torch.cuda.synchronize()
            grads.append({name: getattr(gr, name).cpu().numpy().astype(np.float64) for name in geo.Params.names})
            outs.append(sp.outputs()["feat"].cpu().numpy())
    finally:
        b.set_adjoint_row_limit(b.ADJOINT_ROW_LIMIT)
    np.testing.assert_array_equal(outs[0], outs[1])
    for name in geo.Params.names:
        x, y = grads[1][name], grads[0][name]
        assert np.linalg.norm(y) > 0, name
        assert np.linalg.norm(x - y) <= 1e-5 * np.linalg.norm(y), name


def test_adjoint_without_rows_matches_rows():
    """Beyond the adjoint row limit a call keeps no per-entry gradient rows: every work item adds
    its per-Gaussian sums to the record's gradient atomically.  The same camera + lidar step, in
    the batched form and in the plain per-sensor form, with the limit at 0 (no rows) matches the
    default (rows summed in a fixed order) to rounding, with identical forward outputs; the
    workspace without rows is smaller."""
    b = _binding()
    rng = np.random.default_rng(31)
    n = 3000
    mu = np.stack([rng.uniform(2, 30, n), rng.uniform(-12, 12, n), rng.uniform(-2, 2, n)], 1)
    g = S.random_gaussians(rng, mu, 19, rgb=True, moving_frac=0.5, log_scale_mean=-0.6)
    G = b.GaussTensors.from_numpy(g)
    cam = S.make_camera((0, 0, 0), 0.0, 200, 120, 150.0, t_rs=0.03, ego_vel_world=(3.0, 0, 0), n_channels=16)
    lid = S.make_lidar((0, 0, 0), 0.0, 16, -15.0, 15.0, 256, tile_az=64, tile_el=8, t_sweep=0.1,
                       ego_vel_world=(10.0, 1.0, 0), feat_offset=3, n_channels=8)
    up = np.random.default_rng(32)
    runs = {}
    try:
        for limit in (b.ADJOINT_ROW_LIMIT, 0):
            b.set_adjoint_row_limit(limit)
            rig = b.Rig([cam], [lid])
            for batched in (True, False):
                print(f"[rows] limit {limit}, batched {batched}", flush=True)
                passes = [b.SensorPass(rig, 0, 2, g.n, 1, batched=True)] if batched else \
                    [b.SensorPass(rig, k, 1, g.n, 1) for k in range(2)]
                grads = b.zeros_like_grads(G)
                outs = []
                for sp in passes:
                    sp.fit_capacity(G)
                    sp.render(G)
                    if "ups" not in runs:
                        runs["ups"] = {}
                    key = (sp.first, sp.count)
                    if key not in runs["ups"]:
                        runs["ups"][key] = [torch.from_numpy(a).cuda() for a in (
                            up.normal(size=sp.n_feat).astype(np.float32),
                            (0.1 * up.normal(size=sp.n_rays)).astype(np.float32),
                            up.normal(size=sp.n_rays).astype(np.float32))]
                    sp.raster_bwd(G, *runs["ups"][key], grads)
                    outs.append(sp.outputs())
                torch.cuda.synchronize()
                if batched and limit == 0:   # mixed queue: one cost order, lidar lists counted 4x longer
                    sp = passes[0]
                    work = sp.work.cpu().numpy()[:int(sp.n_work.cpu()[0])]
                    tr = sp.tile_range.cpu().numpy()
                    lens = np.array([tr[t, 1] - tr[t, 0] if t < sp.n_tiles else 0 for t in work[:, 0]])
                    lid_item = work[:, 0] >= int(rig.tile_base[1])
                    cost = np.minimum(queue_length_code(lens) + np.where(lid_item, 32, 0), 255)
                    assert np.all(np.diff(cost) <= 0) and lid_item.any() and (~lid_item).any()
                ws = [int(rig.lib.splat_workspace_bytes(rig.handle, sp.first, sp.count, g.n, sp.k_cap)) for sp in passes]
                runs[(limit, batched)] = ([{k: o[k].cpu().numpy() for k in ("feat", "depth", "alpha", "t_final")}
                                           for o in outs],
                                          {name: getattr(grads, name).cpu().numpy() for name in geo.Params.names}, ws)
    finally:
        b.set_adjoint_row_limit(b.ADJOINT_ROW_LIMIT)
    for batched in (True, False):
        o_r, g_r, ws_r = runs[(b.ADJOINT_ROW_LIMIT, batched)]
        o_a, g_a, ws_a = runs[(0, batched)]
        assert all(x <= y for x, y in zip(ws_a, ws_r)) and sum(ws_a) < sum(ws_r), (ws_a, ws_r)
        for x, y in zip(o_a, o_r):
            for key in x:
                np.testing.assert_array_equal(x[key], y[key], err_msg=key)
        for name in geo.Params.names:
            assert np.abs(g_r[name]).max() > 0, name
            bad = grad_mismatch(g_a[name], g_r[name], rtol=1e-4, afloor=1e-5)
            assert not bad.any(), (batched, name, int(bad.sum()))


def test_autograd_function_camera():
    b = _binding()
    g, cam = cam_scene(n=2000, W=96, H=64)
    rig = b.Rig([cam], [])
    G = b.GaussTensors.from_numpy(g)
    sp = b.SensorPass(rig, 0, 1, g.n, 16)      # too small: the Function grows it
    ps = [t.clone().requires_grad_(True) for t in (G.means, G.log_scales, G.quats, G.opacities, G.velocities, G.features)]
    F, D, A = b.SplatRenderFn.apply(sp, 0, *ps)
    loss = (F ** 2).sum() + D.sum() * 0.01 + A.sum()
    loss.backward()
    for p in ps:
        assert p.grad is not None and torch.isfinite(p.grad).all()
    assert float(ps[0].grad.abs().sum()) > 0
