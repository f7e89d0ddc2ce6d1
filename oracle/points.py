"""Oracle, lidar points to rasterisation rays (App. A "Lidar points to rasterization points").

Plain FP64 numpy (CPU).  Test infrastructure only.

A lidar sweep is delivered as points with the ego motion compensated: every point is expressed
as if the whole sweep had been captured at one reference time (the middle of the sweep), in
world coordinates here.  To render the sweep, each point is first put back where the sensor saw
it at its own capture time t (relative to the reference time), assuming the sensor moves with
constant velocity during the sweep, and then converted to spherical coordinates; the azimuth and
elevation become the ray the rasteriser renders at time t, and the range is the measured range
r_p of the line-of-sight term.

    x_l   = R x_w + t_s                        (sensor frame at the reference time;
                                                x_l = R x_w + t, as for the projection)
    x_cap = x_l + t (-w x x_l - v)             (the point relative to the sensor at time t)
    phi   = atan2(y, x) in [0, 2 pi),  omega = asin(z / r),  r = |x_cap|

v and w are the sensor's linear and angular velocities in its own frame.  Readings (not fixed
by the paper; listed in the design notes): the paper assumes linear motion; the motion used here
is the rigid motion the rolling-shutter model applies to a static Gaussian (App. D: relative
velocity -w x mu - v), to first order in t, so that a Gaussian at a measured point renders on
that point's ray; with w = 0 it is exact linear motion.  A point at the sensor origin (r = 0)
gets phi = omega = 0; z / r is clamped to [-1, 1] before the arcsine.

Pins (tests/test_oracle_points.py): textbook spherical values of axis points, a round trip
through the spherical parametrisation, exact agreement with the moving sensor's world pose for
w = 0 and second-order agreement with an exactly rotating sensor, and the rasteriser's own
rolling-shutter mean of a Gaussian placed at the point, which the ray meets to first order.
"""
import numpy as np

TWO_PI = 2.0 * np.pi


def to_sensor_frame(points_w, R, t_s):
    """x_l = R x_w + t_s for [P,3] world points."""
    R = np.asarray(R, np.float64).reshape(3, 3)
    return np.asarray(points_w, np.float64) @ R.T + np.asarray(t_s, np.float64).reshape(3)


def undo_compensation(x_l, t, lin_vel, ang_vel):
    """The point relative to the sensor at its capture time: x_l + t (-w x x_l - v)."""
    x_l = np.asarray(x_l, np.float64)
    t = np.asarray(t, np.float64).reshape(-1, 1)
    w = np.asarray(ang_vel, np.float64).reshape(1, 3)
    v = np.asarray(lin_vel, np.float64).reshape(1, 3)
    return x_l + t * (-np.cross(w, x_l) - v)


def spherical(x):
    """(phi in [0, 2 pi), omega = asin(z / r), r) of [P,3] points (App. A)."""
    x = np.asarray(x, np.float64)
    r = np.sqrt((x * x).sum(-1))
    phi = np.arctan2(x[:, 1], x[:, 0])
    phi = np.where(phi < 0.0, phi + TWO_PI, phi)
    with np.errstate(invalid="ignore", divide="ignore"):
        s = np.where(r > 0.0, x[:, 2] / np.where(r > 0.0, r, 1.0), 0.0)
    omega = np.arcsin(np.clip(s, -1.0, 1.0))
    return phi, omega, r


def points_to_rays(points_w, t, R, t_s, lin_vel, ang_vel):
    """World points [P,3] captured at times t [P] -> (azimuth, elevation, range), each [P] float64."""
    return spherical(undo_compensation(to_sensor_frame(points_w, R, t_s), t, lin_vel, ang_vel))
