"""Pins of the oracle's geometry (covariance, projections, rolling-shutter velocities) against
facts that do not come from the oracle itself: scipy rotations, closed forms, central
differences of the projection maps and time derivatives of explicitly moved sensors."""
import math

import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

from oracle import geometry as geo
from scenes import synthetic as S

D = torch.float64


def _gauss(means, log_scales=None, quats=None, opac=None, vel=None, feats=None):
    means = np.atleast_2d(np.asarray(means, np.float32))
    n = means.shape[0]
    ls = np.zeros((n, 3), np.float32) if log_scales is None else np.atleast_2d(np.asarray(log_scales, np.float32))
    q = np.tile(np.array([1, 0, 0, 0], np.float32), (n, 1)) if quats is None else np.atleast_2d(np.asarray(quats, np.float32))
    o = np.full(n, 0.5, np.float32) if opac is None else np.asarray(opac, np.float32).reshape(n)
    f = np.ones((n, 4), np.float32) if feats is None else np.asarray(feats, np.float32)
    v = None if vel is None else np.atleast_2d(np.asarray(vel, np.float32))
    return S.Gaussians(means, ls, q, o, v, f)


def test_rotation_matches_scipy():
    rng = np.random.default_rng(0)
    q = rng.normal(size=(64, 4)) * rng.uniform(0.2, 3.0, size=(64, 1))
    R = geo.quat_to_rotmat(geo.t64(q)).numpy()
    ref = Rotation.from_quat(q[:, [1, 2, 3, 0]]).as_matrix()   # scipy is scalar-last
    np.testing.assert_allclose(R, ref, atol=1e-12)


def test_covariance_identity_quat_and_invariances():
    rng = np.random.default_rng(1)
    ls = rng.normal(size=(16, 3))
    q1 = np.tile([1.0, 0, 0, 0], (16, 1))
    Sig = geo.covariance(geo.t64(ls), geo.t64(q1)).numpy()
    for i in range(16):
        np.testing.assert_allclose(Sig[i], np.diag(np.exp(2 * ls[i])), rtol=1e-12)
    q = rng.normal(size=(16, 4))
    a = geo.covariance(geo.t64(ls), geo.t64(q)).numpy()
    b = geo.covariance(geo.t64(ls), geo.t64(-q)).numpy()
    c = geo.covariance(geo.t64(ls), geo.t64(3.7 * q)).numpy()
    np.testing.assert_allclose(a, b, rtol=1e-12)
    np.testing.assert_allclose(a, c, rtol=1e-12)
    # eigenvalues of the covariance are the squared scales
    ev = np.sort(np.linalg.eigvalsh(a), axis=1)
    np.testing.assert_allclose(ev, np.sort(np.exp(2 * ls), axis=1), rtol=1e-10)


def _front_camera(**kw):
    kw.setdefault("t_rs", 0.0)
    return S.make_camera((0, 0, 0), 0.0, 64, 48, 100.0, cx=32.0, cy=24.0, **kw)


def test_camera_axes_and_pinhole_value():
    cam = _front_camera()
    # world point (10, -2, 1): camera x = -Y = 2, y = -Z = -1, z = X = 10
    g = _gauss([[10.0, -2.0, 1.0]])
    pr = geo.project_camera(geo.Params.from_gaussians(g), cam)
    np.testing.assert_allclose(pr.mean2d[0].numpy(), [100 * 0.2 + 32, 100 * -0.1 + 24], atol=1e-12)
    assert float(pr.depth[0]) == pytest.approx(10.0)


def test_camera_on_axis_isotropic_closed_form():
    sig = 0.3
    cam = _front_camera()
    for z in (2.0, 5.0, 17.0):
        g = _gauss([[z, 0, 0]], log_scales=[[math.log(sig)] * 3], opac=[0.8])
        pr = geo.project_camera(geo.Params.from_gaussians(g), cam)
        s2 = (100.0 * sig / z) ** 2
        # float32 inputs: sigma and z are rounded once
        np.testing.assert_allclose(pr.cov2d[0].numpy(), s2 * np.eye(2), rtol=1e-6)
        # EWA compensation for an isotropic 2-D Gaussian: o * s2 / (s2 + eps)
        assert float(pr.o_eff[0]) == pytest.approx(0.8 * s2 / (s2 + 0.3), rel=1e-6)
        # box: 3 sqrt(s2 + eps)
        np.testing.assert_allclose(pr.ext[0].numpy(), 3 * math.sqrt(s2 + 0.3), rtol=1e-6)
        np.testing.assert_allclose(pr.conic[0].numpy(), [1 / (s2 + 0.3), 0, 1 / (s2 + 0.3)], rtol=1e-6, atol=1e-12)


def _num_jac(f, x, h=1e-6):
    x = np.asarray(x, np.float64)
    cols = []
    for k in range(x.shape[0]):
        e = np.zeros_like(x)
        e[k] = h
        cols.append((f(x + e) - f(x - e)) / (2 * h))
    return np.stack(cols, -1)


def test_camera_cov2d_equals_numeric_jacobian():
    rng = np.random.default_rng(2)
    cam = _front_camera(jac_clamp=0.0)
    n = 20
    means = np.stack([rng.uniform(3, 20, n), rng.uniform(-3, 3, n), rng.uniform(-2, 2, n)], 1)
    g = S.random_gaussians(rng, means, 4)
    pr = geo.project_camera(geo.Params.from_gaussians(g), cam)
    Rwc = cam.R.astype(np.float64)
    for i in range(n):
        mu_c = Rwc @ g.means[i].astype(np.float64) + cam.t.astype(np.float64)
        pin = lambda m: np.array([cam.fx * m[0] / m[2] + cam.cx, cam.fy * m[1] / m[2] + cam.cy])
        J = _num_jac(pin, mu_c)
        Rq = Rotation.from_quat(g.quats[i, [1, 2, 3, 0]].astype(np.float64)).as_matrix()
        Sig = Rq @ np.diag(np.exp(2 * g.log_scales[i].astype(np.float64))) @ Rq.T
        ref = J @ (Rwc @ Sig @ Rwc.T) @ J.T
        np.testing.assert_allclose(pr.cov2d[i].numpy(), ref, rtol=1e-6, atol=1e-9)


def _moved_point_in_sensor(R_ws, t_ws, lin, ang, X_world_fn, t):
    """Sensor moving with body-frame linear velocity `lin` and angular velocity `ang`; returns
    the coordinates of world point X(t) in the sensor frame at time t (explicit motion)."""
    R_sw0 = R_ws.T
    c0 = -R_sw0 @ t_ws
    R_sw = R_sw0 @ Rotation.from_rotvec(np.asarray(ang) * t).as_matrix()
    c = c0 + R_sw0 @ (np.asarray(lin) * t)
    return R_sw.T @ (X_world_fn(t) - c)


def test_camera_pixel_velocity_is_time_derivative():
    rng = np.random.default_rng(3)
    cam = _front_camera(jac_clamp=0.0, ego_vel_world=(12.0, 1.0, -0.5), ego_yaw_rate=0.4)
    cam.ang_vel = np.array([0.05, -0.1, 0.2], np.float32)   # any body rates
    n = 12
    means = np.stack([rng.uniform(4, 30, n), rng.uniform(-4, 4, n), rng.uniform(-2, 2, n)], 1)
    vel = rng.normal(0, 3, size=(n, 3))
    g = _gauss(means, vel=vel)
    pr = geo.project_camera(geo.Params.from_gaussians(g), cam)
    R = cam.R.astype(np.float64)
    t = cam.t.astype(np.float64)
    for i in range(n):
        X0 = g.means[i].astype(np.float64)
        V = g.velocities[i].astype(np.float64)
        def uv(tt):
            m = _moved_point_in_sensor(R, t, cam.lin_vel.astype(np.float64), cam.ang_vel.astype(np.float64),
                                       lambda s: X0 + V * s, tt)
            return np.array([cam.fx * m[0] / m[2] + cam.cx, cam.fy * m[1] / m[2] + cam.cy])
        h = 1e-5
        ref = (uv(h) - uv(-h)) / (2 * h)
        np.testing.assert_allclose(pr.vel2d[i].numpy(), ref, rtol=1e-6, atol=1e-6)


def test_camera_uniform_shift_cases():
    # pure yaw rate about the camera y axis: on-axis points move by -fx * w_y for every depth
    cam = _front_camera(jac_clamp=0.0)
    cam.ang_vel = np.array([0.0, 0.25, 0.0], np.float32)
    for z in (3.0, 11.0, 40.0):
        pr = geo.project_camera(geo.Params.from_gaussians(_gauss([[z, 0, 0]])), cam)
        np.testing.assert_allclose(pr.vel2d[0].numpy(), [-100.0 * 0.25, 0.0], atol=1e-9)
    # sideways camera motion v_C = (v, 0, 0): on-axis points move by -fx v / z
    cam = _front_camera(jac_clamp=0.0)
    cam.lin_vel = np.array([2.0, 0.0, 0.0], np.float32)
    for z in (3.0, 11.0):
        pr = geo.project_camera(geo.Params.from_gaussians(_gauss([[z, 0, 0]])), cam)
        np.testing.assert_allclose(pr.vel2d[0].numpy(), [-100.0 * 2.0 / z, 0.0], atol=1e-9)


def test_camera_culling():
    cam = _front_camera()
    g = _gauss([[0.1, 0, 0], [5.0, 0, 0], [-5.0, 0, 0], [5.0, 50.0, 0]], log_scales=[[-3.0] * 3] * 4)
    pr = geo.project_camera(geo.Params.from_gaussians(g), cam)
    # too near, visible, behind the camera, far outside the image
    assert pr.valid.tolist() == [False, True, False, False]


def _lidar(**kw):
    kw.setdefault("rolling_shutter", False)
    return S.make_lidar((0, 0, 0), 0.0, 16, -15.0, 15.0, 360, tile_az=8, tile_el=4, **kw)


def test_spherical_mean_and_jacobian_numeric():
    rng = np.random.default_rng(4)
    n = 20
    mu = rng.uniform(-20, 20, size=(n, 3))
    J = geo.spherical_jacobian(geo.t64(mu)).numpy()
    sph = lambda m: np.array([math.atan2(m[1], m[0]), math.asin(m[2] / np.linalg.norm(m)), np.linalg.norm(m)])
    for i in range(n):
        np.testing.assert_allclose(J[i], _num_jac(sph, mu[i]), rtol=1e-7, atol=1e-9)


def test_lidar_closed_forms():
    lid = _lidar()
    R = 10.0
    sy, sz = 0.2, 0.35
    g = _gauss([[R, 0, 0]], log_scales=[[math.log(0.5), math.log(sy), math.log(sz)]])
    pr = geo.project_lidar(geo.Params.from_gaussians(g), lid)
    np.testing.assert_allclose(pr.mean2d[0].numpy(), [0.0, 0.0], atol=1e-12)
    np.testing.assert_allclose(pr.cov2d[0].numpy(), np.diag([sy ** 2, sz ** 2]) / R ** 2, rtol=1e-6)
    assert float(pr.depth[0]) == pytest.approx(R)
    # ego motion (v, 0, 0): the range shrinks at v, angles stay
    lid2 = _lidar(ego_vel_world=(7.0, 0, 0))
    pr = geo.project_lidar(geo.Params.from_gaussians(g), lid2)
    np.testing.assert_allclose([*pr.vel2d[0].numpy(), float(pr.v_r[0])], [0.0, 0.0, -7.0], atol=1e-12)


def test_lidar_azimuth_range_and_culling():
    lid = _lidar(r_min=1.0, r_max=50.0)
    g = _gauss([[-3.0, -0.1, 0.0], [0.5, 0, 0], [60.0, 0, 0], [0.0, 0.0, 5.0], [3.0, 0.2, 0.1]],
               log_scales=[[-4.0] * 3] * 5)
    pr = geo.project_lidar(geo.Params.from_gaussians(g), lid)
    phi = pr.mean2d[:, 0].numpy()
    assert 0.0 <= phi[0] < 2 * math.pi and phi[0] > math.pi       # atan2 mapped to [0, 2pi)
    # behind (360 deg field of view); too near; too far; on the pole (rho < 1e-4 r); visible
    assert pr.valid.tolist() == [True, False, False, False, True]
    # above the top elevation boundary (15 deg) by more than the box: culled
    g2 = _gauss([[3.0, 0.0, 3.0]], log_scales=[[-4.0] * 3])
    assert not bool(geo.project_lidar(geo.Params.from_gaussians(g2), lid).valid[0])


def test_lidar_velocity_is_time_derivative():
    rng = np.random.default_rng(5)
    lid = _lidar(ego_vel_world=(15.0, -2.0, 0.3), ego_yaw_rate=0.3)
    lid.ang_vel = np.array([0.02, -0.05, 0.3], np.float32)
    n = 12
    means = np.stack([rng.uniform(5, 40, n), rng.uniform(-30, 30, n), rng.uniform(-3, 3, n)], 1)
    vel = rng.normal(0, 3, size=(n, 3))
    g = _gauss(means, vel=vel)
    pr = geo.project_lidar(geo.Params.from_gaussians(g), lid)
    R = lid.R.astype(np.float64)
    t = lid.t.astype(np.float64)
    for i in range(n):
        X0 = g.means[i].astype(np.float64)
        V = g.velocities[i].astype(np.float64)
        def sph(tt):
            m = _moved_point_in_sensor(R, t, lid.lin_vel.astype(np.float64), lid.ang_vel.astype(np.float64),
                                       lambda s: X0 + V * s, tt)
            return np.array([math.atan2(m[1], m[0]), math.asin(m[2] / np.linalg.norm(m)), np.linalg.norm(m)])
        h = 1e-5
        ref = (sph(h) - sph(-h)) / (2 * h)
        got = np.array([*pr.vel2d[i].numpy(), float(pr.v_r[i])])
        np.testing.assert_allclose(got, ref, rtol=1e-6, atol=1e-8)


def test_rolling_shutter_box_extension():
    cam = _front_camera(t_rs=0.04, jac_clamp=0.0)
    cam.lin_vel = np.array([2.0, 0.0, 0.0], np.float32)
    g = _gauss([[5.0, 0, 0]], log_scales=[[math.log(0.1)] * 3])
    pr = geo.project_camera(geo.Params.from_gaussians(g), cam)
    s2 = (100.0 * 0.1 / 5.0) ** 2
    v = 100.0 * 2.0 / 5.0
    np.testing.assert_allclose(pr.ext[0].numpy(), [3 * math.sqrt(s2 + 0.3) + v * 0.02, 3 * math.sqrt(s2 + 0.3)], rtol=1e-6)


# ------------------------------------------------------------------------------------------
# Jacobian clamp off the frustum (the 3DGS projection the paper keeps, Sec. 3.2): J^I is
# evaluated at x/z and y/z clamped to +-jac_clamp * (size / 2) / f, while the mean is not
# ------------------------------------------------------------------------------------------
def _clamp_camera(jac_clamp):
    # fx != fy and width != height, so a swapped focal length or half-size changes the limits
    return S.make_camera((0, 0, 0), 0.0, 64, 48, 100.0, fy=80.0, cx=32.0, cy=24.0, t_rs=0.0,
                         jac_clamp=jac_clamp)


def _clamp_closed_form(fx, fy, z, tx, ty, sig, vrel):
    """Hand-expanded J Sigma J^T for an isotropic Sigma = sig^2 I and J v, with J evaluated at
    (tx, ty) = (x/z, y/z) after the clamp: J = [[fx/z, 0, -fx tx/z], [0, fy/z, -fy ty/z]]."""
    s = (sig / z) ** 2
    cov = s * np.array([[fx * fx * (1 + tx * tx), fx * fy * tx * ty],
                        [fx * fy * tx * ty, fy * fy * (1 + ty * ty)]])
    vx, vy, vz = vrel
    vel = np.array([fx * (vx - tx * vz) / z, fy * (vy - ty * vz) / z])
    return cov, vel


def _clamp_cases(geo_mod):
    """Yields (got cov, got vel, got mean, expected cov, expected vel, expected mean) for points
    beyond the clamp on both axes (one of them negative), inside it, and with the clamp off."""
    sig = 0.25
    lin = np.array([-1.5, 0.7, -2.0])              # camera frame; the Gaussian is static
    vrel = -lin                                    # relative velocity of a static point
    cases = []
    # (x/z, y/z, z, jac_clamp) -> clamped (tx, ty) by hand
    for rx, ry, z, jc, tx, ty in [
        (0.8, -0.6, 10.0, 1.3, 1.3 * 32 / 100, -1.3 * 24 / 80),    # both clamped
        (-0.5, 0.45, 7.0, 1.3, -1.3 * 32 / 100, 1.3 * 24 / 80),    # both clamped, signs flipped
        (0.2, 0.1, 12.0, 1.3, 0.2, 0.1),                           # inside: untouched
        (0.8, -0.6, 10.0, 2.0, 2.0 * 32 / 100, -2.0 * 24 / 80),    # another clamp value
        (0.8, -0.6, 10.0, 0.0, 0.8, -0.6),                         # clamp off
    ]:
        cam = _clamp_camera(jc)
        cam.lin_vel = lin.astype(np.float32)
        # camera axes: x_c = -Y_w, y_c = -Z_w, z_c = X_w for this camera at the origin
        xc, yc = rx * z, ry * z
        g = _gauss([[z, -xc, -yc]], log_scales=[[math.log(sig)] * 3])
        pr = geo_mod.project_camera(geo_mod.Params.from_gaussians(g), cam)
        m = g.means[0].astype(np.float64)
        zf, xf, yf = m[0], -m[1], -m[2]             # the float32 point actually used
        t_x = tx if jc > 0 and abs(xf / zf) > jc * 32 / 100 else xf / zf
        t_y = ty if jc > 0 and abs(yf / zf) > jc * 24 / 80 else yf / zf
        s_f = float(np.float32(sig))
        cov, vel = _clamp_closed_form(100.0, 80.0, zf, t_x, t_y, math.exp(math.log(s_f)), vrel.astype(np.float32).astype(np.float64))
        mean = np.array([100.0 * xf / zf + 32.0, 80.0 * yf / zf + 24.0])   # never clamped
        cases.append((pr.cov2d[0].detach().numpy(), pr.vel2d[0].detach().numpy(),
                      pr.mean2d[0].detach().numpy(), cov, vel, mean, (rx, ry, jc)))
    return cases


def _check_clamp(geo_mod):
    for got_c, got_v, got_m, cov, vel, mean, tag in _clamp_cases(geo_mod):
        np.testing.assert_allclose(got_c, cov, rtol=1e-6, atol=1e-9, err_msg=str(tag))
        np.testing.assert_allclose(got_v, vel, rtol=1e-6, atol=1e-9, err_msg=str(tag))
        np.testing.assert_allclose(got_m, mean, rtol=1e-9, atol=1e-9, err_msg=str(tag))


def test_jacobian_clamp_closed_form():
    _check_clamp(geo)


def test_jacobian_clamp_changes_the_projection():
    """With the clamp on, an off-frustum Gaussian's covariance and velocity differ from the
    unclamped ones by far more than the pin's tolerance (the pin can tell them apart)."""
    cases = _clamp_cases(geo)
    on, off = cases[0], cases[4]
    assert np.abs(on[0] - off[0]).max() > 0.05 * np.abs(off[0]).max()
    assert np.abs(on[1] - off[1]).max() > 0.05 * np.abs(off[1]).max()
    np.testing.assert_allclose(on[2], off[2], rtol=1e-12)          # the mean is the same


def _mutant_geometry(old, new):
    """The oracle's geometry module with one planted mistake (source replaced once), on the CPU."""
    import inspect
    import types
    src = inspect.getsource(geo)
    assert src.count(old) == 1, old
    import sys
    name = "oracle._geometry_mutant"
    mod = types.ModuleType(name)
    sys.modules[name] = mod          # dataclasses look their module up while being created
    try:
        exec(compile(src.replace(old, new), name, "exec"), mod.__dict__)
    finally:
        del sys.modules[name]
    return mod


@pytest.mark.parametrize("old,new", [
    # full size instead of half size
    ("limx = cam.jac_clamp * 0.5 * cam.width / cam.fx", "limx = cam.jac_clamp * cam.width / cam.fx"),
    # x clamped instead of x/z
    ("tx = torch.clamp(tx, -limx, limx)", "tx = torch.clamp(x, -limx, limx) / zs"),
    # width and height swapped
    ("limy = cam.jac_clamp * 0.5 * cam.height / cam.fy", "limy = cam.jac_clamp * 0.5 * cam.width / cam.fy"),
    # the clamp dropped on y
    ("ty = torch.clamp(ty, -limy, limy)", "ty = ty"),
    # the clamped ratio leaking into the mean
    ("u = cam.fx * x / zs + cam.cx", "u = cam.fx * torch.clamp(x / zs, -1.3 * 0.5 * cam.width / cam.fx, 1.3 * 0.5 * cam.width / cam.fx) + cam.cx"),
])
def test_jacobian_clamp_pin_catches_planted_mistakes(old, new):
    with pytest.raises(AssertionError):
        _check_clamp(_mutant_geometry(old, new))
