"""Pins of the oracle's lidar points-to-rays map (oracle/points.py; App. A "Lidar points to
rasterization points"): textbook spherical coordinates, a round trip through the spherical
parametrisation, the world pose of a sensor that moves (exactly for linear motion, to second
order when it also turns), and the rolling-shutter mean the projection gives a Gaussian placed
at the point."""
import numpy as np
import torch
from scipy.spatial.transform import Rotation

from oracle import geometry as geo
from oracle import points as op
from scenes import synthetic as S

I3 = np.eye(3)
Z3 = np.zeros(3)


def test_axis_points():
    pts = np.array([[1, 0, 0], [0, 2, 0], [-3, 0, 0], [0, -1, 0], [1, 0, 1], [2, 2, 0], [0, 0, 5], [0, 0, 0]], float)
    phi, om, r = op.points_to_rays(pts, np.zeros(len(pts)), I3, Z3, Z3, Z3)
    np.testing.assert_allclose(phi, [0, np.pi / 2, np.pi, 1.5 * np.pi, 0, np.pi / 4, 0, 0], atol=1e-15)
    np.testing.assert_allclose(om, [0, 0, 0, 0, np.pi / 4, 0, np.pi / 2, 0], atol=1e-15)
    np.testing.assert_allclose(r, [1, 2, 3, 1, np.sqrt(2), np.sqrt(8), 5, 0], atol=1e-15)


def test_round_trip_through_spherical_parametrisation():
    rng = np.random.default_rng(1)
    phi = rng.uniform(0, 2 * np.pi, 1000)
    om = rng.uniform(-0.6, 0.5, 1000)
    r = rng.uniform(1, 120, 1000)
    x = np.stack([r * np.cos(om) * np.cos(phi), r * np.cos(om) * np.sin(phi), r * np.sin(om)], 1)
    p2, o2, r2 = op.points_to_rays(x, np.zeros(1000), I3, Z3, Z3, Z3)
    d = np.abs(((p2 - phi + np.pi) % (2 * np.pi)) - np.pi)
    assert d.max() < 1e-12 and np.all((p2 >= 0) & (p2 < 2 * np.pi))
    np.testing.assert_allclose(o2, om, atol=1e-12)
    np.testing.assert_allclose(r2, r, rtol=1e-13)


def _pose(rng):
    R = Rotation.from_euler("zyx", rng.uniform(-0.5, 0.5, 3)).as_matrix()
    return R, rng.uniform(-5, 5, 3)


def test_linear_motion_matches_the_moving_sensor_pose():
    """w = 0: the sensor origin moves to c0 + R^T v t in the world; the point relative to it is
    R (x_w - c(t)), exactly."""
    rng = np.random.default_rng(2)
    R, ts = _pose(rng)
    v = np.array([14.0, -1.0, 0.3])
    xw = rng.uniform(-60, 60, (500, 3))
    t = rng.uniform(-0.05, 0.05, 500)
    c0 = -R.T @ ts
    exact = np.stack([R @ (xw[i] - (c0 + R.T @ v * t[i])) for i in range(500)])
    want = op.spherical(exact)
    got = op.points_to_rays(xw, t, R, ts, v, Z3)
    for a, b in zip(got, want):
        np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-12)


def test_turning_sensor_agrees_to_second_order():
    """With an angular velocity the map is the first-order form of an exactly rotating frame:
    halving the time quarters the difference."""
    rng = np.random.default_rng(3)
    R, ts = _pose(rng)
    v, w = np.array([10.0, 0.5, 0.0]), np.array([0.05, -0.02, 0.6])
    xw = rng.uniform(-40, 40, (200, 3))
    xl = op.to_sensor_frame(xw, R, ts)

    def err(tt):
        t = np.full(200, tt)
        exact = np.stack([Rotation.from_rotvec(-w * tt).as_matrix() @ (xl[i] - v * tt) for i in range(200)])
        return np.abs(op.undo_compensation(xl, t, v, w) - exact).max()

    e1, e2 = err(0.04), err(0.02)
    assert e1 > 1e-6 and 3.6 < e1 / e2 < 4.4, (e1, e2)


def test_gaussian_at_the_point_meets_its_ray():
    """A static Gaussian centred on a world point: the projection's rolling-shutter mean at time t
    (phi + dphi/dt t, omega + domega/dt t, r + v_r t) and the point's ray agree to first order in
    t (the difference shrinks four-fold when t halves)."""
    rng = np.random.default_rng(4)
    lid = S.make_lidar((1.0, -2.0, 1.8), 20.0, 32, -25.0, 15.0, 512, t_sweep=0.1, ego_vel_world=(12.0, 3.0, 0.0),
                       ego_yaw_rate=0.4)
    n = 300
    xw = np.stack([rng.uniform(-50, 50, n), rng.uniform(-50, 50, n), rng.uniform(-1.0, 3.0, n)], 1)
    g = S.Gaussians(xw.astype(np.float32), np.full((n, 3), -1.0, np.float32), np.tile(np.float32([1, 0, 0, 0]), (n, 1)),
                    np.full(n, 0.5, np.float32), np.zeros((n, 3), np.float32), np.ones((n, 3), np.float32))
    pr = geo.project(geo.Params.from_gaussians(g), lid)
    xw64 = g.means.astype(np.float64)   # the Gaussian means the projection saw
    m = pr.mean2d.detach().numpy()
    vel = pr.vel2d.detach().numpy()
    r0 = pr.blend.detach().numpy()
    vr = pr.v_r.detach().numpy()

    def err(tt):
        t = np.full(n, tt)
        phi, om, r = op.points_to_rays(xw64, t, lid.R, lid.t, lid.lin_vel, lid.ang_vel)
        dphi = np.abs(((phi - (m[:, 0] + vel[:, 0] * tt) + np.pi) % (2 * np.pi)) - np.pi)
        return max(dphi.max(), np.abs(om - (m[:, 1] + vel[:, 1] * tt)).max(), np.abs(r - (r0 + vr * tt)).max() / 50)

    e0 = err(0.0)
    assert e0 < 1e-12
    e1, e2 = err(0.05), err(0.025)
    assert e1 > 1e-8 and 3.5 < e1 / e2 < 4.5, (e1, e2)
