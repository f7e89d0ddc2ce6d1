"""Pins of the oracle's compositing: closed forms (one and two Gaussians, the stop rule, the
median), an empty scene, sum of weights = 1 - T, permutation invariance, rolling shutter ->
global shutter at zero velocity, lidar rotation = column shift, scene scaling, TILE vs BOX
relations, and an independent per-ray Python loop on tiny scenes."""
import math

import numpy as np
import pytest
import torch

from oracle import geometry as geo
from oracle import render as rd
from oracle import tiles as tl
from scenes import synthetic as S


def _gauss(means, log_scales, opac, feats, quats=None, vel=None):
    means = np.asarray(means, np.float32).reshape(-1, 3)
    n = means.shape[0]
    q = np.tile(np.array([1, 0, 0, 0], np.float32), (n, 1)) if quats is None else np.asarray(quats, np.float32)
    return S.Gaussians(means, np.asarray(log_scales, np.float32).reshape(n, 3), q,
                       np.asarray(opac, np.float32).reshape(n), None if vel is None else np.asarray(vel, np.float32),
                       np.asarray(feats, np.float32).reshape(n, -1))


def _cam(W=33, H=25, t_rs=0.0, **kw):
    # principal point on a pixel centre so an on-axis Gaussian sits exactly on pixel (W//2, H//2)
    return S.make_camera((0, 0, 0), 0.0, W, H, 40.0, cx=W // 2 + 0.5, cy=H // 2 + 0.5, t_rs=t_rs,
                         n_channels=3, tile=(8, 8), **kw)


def _centre(cam):
    return (cam.height // 2) * cam.width + cam.width // 2


def test_single_gaussian_on_the_ray():
    cam = _cam()
    for o in (0.3, 0.95, 0.999):
        g = _gauss([[6.0, 0, 0]], [[math.log(0.2)] * 3], [o], [[0.2, -1.0, 3.0]])
        out = rd.render_sensor(g, cam, [_centre(cam)])
        pr = out["proj"]
        a = min(0.99, float(pr.o_eff[0]))
        np.testing.assert_allclose(out["F"][0].numpy(), a * np.array([0.2, -1.0, 3.0], np.float32).astype(np.float64), rtol=1e-12)
        assert float(out["A"][0]) == pytest.approx(a, rel=1e-12)
        assert float(out["D"][0]) == pytest.approx(6.0 * a, rel=1e-12)
        assert float(out["T"][0]) == pytest.approx(1 - a, rel=1e-12)


def test_two_gaussians_over_operator_and_median():
    cam = _cam()
    # near Gaussian (depth 4) alpha a1, far (depth 9) alpha a2, both centred on the ray
    g = _gauss([[9.0, 0, 0], [4.0, 0, 0]], [[math.log(0.3)] * 3, [math.log(0.15)] * 3], [0.6, 0.4],
               [[1.0, 0, 0], [0, 1.0, 0]])
    out = rd.render_sensor(g, cam, [_centre(cam)])
    o = out["proj"].o_eff.numpy()
    a_far, a_near = o[0], o[1]
    F = out["F"][0].numpy()
    np.testing.assert_allclose(F, [a_far * (1 - a_near), a_near, 0.0], rtol=1e-12, atol=1e-15)
    assert float(out["A"][0]) == pytest.approx(1 - (1 - a_near) * (1 - a_far), rel=1e-12)
    assert float(out["D"][0]) == pytest.approx(4.0 * a_near + 9.0 * a_far * (1 - a_near), rel=1e-12)
    # median: first Gaussian after which T < 1/2
    med = 4.0 if (1 - a_near) < 0.5 else (9.0 if (1 - a_near) * (1 - a_far) < 0.5 else 0.0)
    assert float(out["median"][0]) == pytest.approx(med)
    assert int(out["last_id"][0]) == 0


def test_stop_rule_closed_form():
    cam = _cam()
    # five Gaussians with alpha clamped to 0.99 would stop after two; use o_eff ~ 0.95 instead:
    # T after k = 0.05^k; k = 3 gives 1.25e-4 (kept), k = 4 gives 6.25e-6 < 1e-4 (stop)
    n = 5
    z = np.arange(n) + 3.0
    sig = 2.0
    g = _gauss(np.stack([z, 0 * z, 0 * z], 1), [[math.log(sig)] * 3] * n, [0.95] * n, np.ones((n, 3)))
    out = rd.render_sensor(g, cam, [_centre(cam)])
    a = out["proj"].o_eff.numpy()
    assert np.all(a > 0.94) and np.all(a < 0.95)
    Tk = np.cumprod(1 - a)
    assert Tk[2] >= 1e-4 and Tk[3] < 1e-4
    assert int(out["n_kept"][0]) == 3
    assert float(out["T"][0]) == pytest.approx(Tk[2], rel=1e-12)
    assert float(out["F"][0, 0]) == pytest.approx(1 - Tk[2], rel=1e-12)


def test_empty_scene():
    cam = _cam()
    g = _gauss([[-5.0, 0, 0]], [[0.0] * 3], [0.5], [[1.0, 1.0, 1.0]])   # behind the camera
    out = rd.render_sensor(g, cam)
    assert float(out["F"].abs().max()) == 0.0 and float(out["D"].abs().max()) == 0.0
    assert float(out["A"].abs().max()) == 0.0 and float(out["T"].min()) == 1.0


def _random_scene(seed, n=60):
    rng = np.random.default_rng(seed)
    means = np.stack([rng.uniform(2, 12, n), rng.uniform(-3, 3, n), rng.uniform(-2, 2, n)], 1)
    return S.random_gaussians(rng, means, 3, moving_frac=0.5)


def test_weights_sum_and_permutation_invariance():
    cam = _cam(t_rs=0.03)
    g = _random_scene(0)
    g1 = S.Gaussians(g.means, g.log_scales, g.quats, g.opacities, g.velocities, np.ones_like(g.features))
    out = rd.render_sensor(g1, cam)
    np.testing.assert_allclose(out["F"][:, 0].numpy(), out["A"].numpy(), rtol=1e-12, atol=1e-14)
    assert float(out["A"].min()) >= 0.0 and float(out["A"].max()) < 1.0
    perm = np.random.default_rng(1).permutation(g.n)
    a = rd.render_sensor(g, cam)
    b = rd.render_sensor(g.subset(perm), cam)
    for k in ("F", "D", "A"):
        np.testing.assert_allclose(a[k].numpy(), b[k].numpy(), rtol=1e-12, atol=1e-14)


def test_rolling_shutter_collapses_to_global_shutter():
    g = _random_scene(2)
    static = S.Gaussians(g.means, g.log_scales, g.quats, g.opacities, None, g.features)
    rs = rd.render_sensor(static, _cam(t_rs=0.05))
    gs = rd.render_sensor(static, _cam(t_rs=0.0))
    for k in ("F", "D", "A"):
        np.testing.assert_array_equal(rs[k].numpy(), gs[k].numpy())
    # and with motion the shutter matters
    moving = rd.render_sensor(g, _cam(t_rs=0.05))
    assert float((moving["F"] - gs["F"]).abs().max()) > 1e-3


def _small_lidar(yaw=0.0, **kw):
    return S.make_lidar((0, 0, 0), yaw, 16, -15.0, 15.0, 256, tile_az=16, tile_el=4,
                        rolling_shutter=False, n_channels=3, **kw)


def test_lidar_rotation_shifts_columns():
    rng = np.random.default_rng(3)
    n = 80
    means = np.stack([rng.uniform(-15, 15, n), rng.uniform(-15, 15, n), rng.uniform(-2, 2, n)], 1)
    g = S.random_gaussians(rng, means, 3, moving_frac=0.0)
    k = 5
    base = _small_lidar(0.0)
    rot = _small_lidar(math.degrees(k * 2 * math.pi / 256))
    a = rd.render_sensor(g, base)
    b = rd.render_sensor(g, rot)
    # rotating the sensor by k azimuth steps: ray j of the rotated sensor sees what ray j + k saw
    # (the float32 rotation matrices differ by rounding, so compare to 1e-5 and skip rays
    # with a near-threshold decision in either render)
    near = np.roll(a["near"].reshape(16, 256), -k, axis=1) | b["near"].reshape(16, 256)
    for key in ("F", "D", "A"):
        A = np.roll(a[key].numpy().reshape(16, 256, -1), -k, axis=1)
        B = b[key].numpy().reshape(16, 256, -1)
        np.testing.assert_allclose(B[~near], A[~near], rtol=1e-4, atol=1e-5)
    assert near.mean() < 0.05


def test_lidar_scene_scaling():
    rng = np.random.default_rng(4)
    n = 60
    means = np.stack([rng.uniform(-10, 10, n), rng.uniform(-10, 10, n), rng.uniform(-1.5, 1.5, n)], 1)
    g = S.random_gaussians(rng, means, 3, moving_frac=0.0)
    lam = 2.5
    g2 = S.Gaussians(g.means * np.float32(lam), g.log_scales + np.float32(math.log(lam)), g.quats,
                     g.opacities, None, g.features)
    a = rd.render_sensor(g, _small_lidar(r_min=0.5, r_max=100.0))
    b = rd.render_sensor(g2, _small_lidar(r_min=0.5 * lam, r_max=100.0 * lam))
    ok = ~(a["near"] | b["near"])
    np.testing.assert_allclose(b["F"].numpy()[ok], a["F"].numpy()[ok], rtol=1e-5, atol=1e-7)
    np.testing.assert_allclose(b["A"].numpy()[ok], a["A"].numpy()[ok], rtol=1e-5, atol=1e-7)
    np.testing.assert_allclose(b["D"].numpy()[ok], lam * a["D"].numpy()[ok], rtol=1e-5, atol=1e-6)


def _loop_render(g, sensor, ray_ids):
    """Independent sequential implementation of the per-ray rules, one Gaussian at a time."""
    p = geo.Params.from_gaussians(g)
    pr = geo.project(p, sensor)
    lid = hasattr(sensor, "ray_az")
    rays = rd.lidar_rays(sensor, ray_ids) if lid else rd.camera_rays(sensor, ray_ids)
    off, C = sensor.feat_offset, sensor.n_channels
    res = []
    for r in range(len(ray_ids)):
        px, py = rays.p[r].tolist()
        t = float(rays.t[r])
        items = []
        for i in range(g.n):
            if not bool(pr.valid[i]):
                continue
            lo = pr.lo[i].tolist()
            hi = pr.hi[i].tolist()
            if lid:
                inside_az = any(lo[0] <= px + k * 2 * math.pi < hi[0] for k in range(-3, 4))
            else:
                inside_az = lo[0] <= px < hi[0]
            if inside_az and lo[1] <= py < hi[1]:
                items.append((float(pr.depth[i]), i))
        items.sort()
        T, F, Dv = 1.0, np.zeros(C), 0.0
        for _, i in items:
            mx, my = pr.mean2d[i].tolist()
            vx, vy = pr.vel2d[i].tolist()
            dx, dy = px - (mx + vx * t), py - (my + vy * t)
            if lid:
                while dx >= math.pi:
                    dx -= 2 * math.pi
                while dx < -math.pi:
                    dx += 2 * math.pi
            a_, b_, c_ = pr.conic[i].tolist()
            alpha = min(0.99, float(pr.o_eff[i]) * math.exp(-(0.5 * (a_ * dx * dx + c_ * dy * dy) + b_ * dx * dy)))
            if alpha < 1 / 255:
                continue
            Tn = T * (1 - alpha)
            if Tn < 1e-4:
                break
            gval = float(pr.blend[i]) + (float(pr.v_r[i]) * t if lid else 0.0)
            F += alpha * T * g.features[i, off:off + C].astype(np.float64)
            Dv += alpha * T * gval
            T = Tn
        res.append((F, Dv, 1 - T))
    return res


@pytest.mark.parametrize("kind", ["camera", "lidar"])
def test_vectorised_equals_sequential_loop(kind):
    rng = np.random.default_rng(5)
    if kind == "camera":
        sensor = _cam(W=20, H=16, t_rs=0.04, ego_vel_world=(8.0, 0, 0))
        g = _random_scene(6, n=40)
        ids = np.arange(sensor.width * sensor.height)[::3]
    else:
        sensor = S.make_lidar((0, 0, 0), 0.0, 8, -15.0, 15.0, 64, tile_az=8, tile_el=4, t_sweep=0.1,
                              ego_vel_world=(10.0, 0, 0), n_channels=3)
        n = 50
        means = np.stack([rng.uniform(-8, 8, n), rng.uniform(-8, 8, n), rng.uniform(-1, 1, n)], 1)
        g = S.random_gaussians(rng, means, 3, moving_frac=0.5)
        ids = np.arange(sensor.n_rays)[::2]
    out = rd.render_sensor(g, sensor, ids)
    ref = _loop_render(g, sensor, ids)
    for r, (F, Dv, A) in enumerate(ref):
        np.testing.assert_allclose(out["F"][r].numpy(), F, rtol=1e-10, atol=1e-12)
        assert float(out["D"][r]) == pytest.approx(Dv, rel=1e-10, abs=1e-12)
        assert float(out["A"][r]) == pytest.approx(A, rel=1e-10, abs=1e-12)


def test_tile_rule_is_superset_of_box_candidates():
    cam = _cam(W=40, H=32)
    g = _random_scene(7, n=50)
    p = geo.Params.from_gaussians(g)
    pr = geo.project(p, cam)
    rays = rd.camera_rays(cam)
    order = np.nonzero(pr.valid.numpy())[0]
    box = rd._box_mask(pr, order, rays.p).numpy()
    tile = rd._tile_mask(pr, cam, order, rays.tile).numpy()
    assert np.all(tile[box])
    assert tile.sum() > box.sum()


def test_tile_rule_hand_worked():
    """TILE mode (the paper's rule: every Gaussian listed for the pixel's tile, Sec. 3.2, and
    App. A's lidar tile ranges) on boxes chosen by hand: the candidate set is the union of
    whole tiles, worked out on paper below, including pixels outside the box."""
    from types import SimpleNamespace
    cam = _cam(W=64, H=48)              # 8 x 8 tiles: 8 tiles across, 6 down
    # box x in [17.5, 40.2) -> tiles x 2..5 (17.5/8 = 2.19, 40.2/8 = 5.03); y in [3, 20) -> 0..2
    lo = torch.tensor([[17.5, 3.0], [-5.0, 40.1]], dtype=torch.float64)
    hi = torch.tensor([[40.2, 20.0], [7.9, 47.0]], dtype=torch.float64)
    # second box: x in [-5, 7.9) -> tile 0 only; y in [40.1, 47) -> tile 5
    proj = SimpleNamespace(lo=lo, hi=hi, kind="camera")
    pix = np.array([[16, 0], [17, 3], [40, 23], [47, 23], [48, 0], [20, 24], [0, 40], [7, 47],
                    [8, 47], [0, 39]])
    tiles = (pix[:, 1] // 8) * 8 + pix[:, 0] // 8
    m = rd._tile_mask(proj, cam, np.array([0, 1]), tiles).numpy()
    want0 = [True, True, True, True, False, False, False, False, False, False]
    want1 = [False, False, False, False, False, False, True, True, False, False]
    assert m[:, 0].tolist() == want0
    assert m[:, 1].tolist() == want1
    # lidar: 5 azimuth tiles of 2 pi / 5 rad, elevation boundaries (-0.2, 0, 0.2)
    lid = SimpleNamespace(n_az_tiles=5, tile_az=4, az_res=2 * math.pi / 20,
                          elev_bounds=np.array([-0.2, 0.0, 0.2]))
    w = 2 * math.pi / 5
    # box A: azimuth [-0.3, 0.5) wraps: floor(-0.3 / w) = -1 -> tile 4, floor(0.5 / w) + 1 = 1
    #   -> tiles {4, 0}; elevation [-0.05, 0.05) -> both rows.  Tiles {4, 0, 9, 5}.
    # box B: azimuth [2w + 0.1, 2w + 0.2), elevation [0.01, 0.02) -> tile 2 + 5 * 1 = 7.
    # box C: azimuth [1.0, 1.0 + 2 pi) spans every column; elevation [-0.3, -0.1) -> row 0.
    lo = torch.tensor([[-0.3, -0.05], [2 * w + 0.1, 0.01], [1.0, -0.3]], dtype=torch.float64)
    hi = torch.tensor([[0.5, 0.05], [2 * w + 0.2, 0.02], [1.0 + 2 * math.pi, -0.1]], dtype=torch.float64)
    proj = SimpleNamespace(lo=lo, hi=hi, kind="lidar")
    tiles = np.arange(10)
    m = rd._tile_mask(proj, lid, np.array([0, 1, 2]), tiles).numpy()
    assert np.nonzero(m[:, 0])[0].tolist() == [0, 4, 5, 9]
    assert np.nonzero(m[:, 1])[0].tolist() == [7]
    assert np.nonzero(m[:, 2])[0].tolist() == [0, 1, 2, 3, 4]
    # a ray outside every tile (tile -1) is never a candidate
    assert not rd._tile_mask(proj, lid, np.array([0, 1, 2]), np.array([-1])).numpy().any()
