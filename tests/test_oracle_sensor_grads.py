"""Pins of the sensor-parameter part of the oracle: the camera time offset (Sec. 3.2, the offset
between a camera's timestamp and the middle of its exposure) and the gradients with respect to
the sensors' linear and angular velocities and the time offset (oracle/grad.py)."""
import dataclasses

import numpy as np

from oracle import grad as ogr
from oracle import render as rd
from scenes import synthetic as S


def _scene(seed=3, n=300, moving=True):
    rng = np.random.default_rng(seed)
    mu = S.road_slab(rng, n, (2.0, 30.0), (-8.0, 8.0), 3.0)
    g = S.random_gaussians(rng, mu, 16, rgb=True, moving_frac=0.5 if moving else 0.0)
    cam = S.make_camera((0, 0, 1.5), 0.0, 48, 32, 30.0, t_rs=0.03, ego_vel_world=(9.0, 0.5, 0.0),
                        ego_yaw_rate=0.3, n_channels=16)
    lid = S.make_lidar((0, 0, 1.8), 0.0, 8, -20.0, 10.0, 64, t_sweep=0.1, ego_vel_world=(9.0, 0.5, 0.0),
                       ego_yaw_rate=0.3, tile_az=8, feat_offset=3, n_channels=8)
    return g, cam, lid


def test_time_offset_has_no_effect_without_motion():
    """With no Gaussian velocity and a still camera every pixel mean is time independent."""
    g, cam, _ = _scene(moving=False)
    still = dataclasses.replace(cam, lin_vel=np.zeros(3, np.float32), ang_vel=np.zeros(3, np.float32))
    a = rd.render_sensor(g, still)
    b = rd.render_sensor(g, dataclasses.replace(still, time_offset=0.02))
    for k in ("F", "D", "A", "T"):
        np.testing.assert_array_equal(a[k].numpy(), b[k].numpy(), err_msg=k)


def test_time_offset_moves_the_image():
    """With motion the offset changes the image (it is not dropped somewhere)."""
    g, cam, _ = _scene()
    a = rd.render_sensor(g, cam)
    b = rd.render_sensor(g, dataclasses.replace(cam, time_offset=0.02))
    assert float((a["A"] - b["A"]).abs().max()) > 1e-3


def _check_sensor(g, sensor, idx):
    rng = np.random.default_rng(5)
    n = len(idx)
    C = sensor.n_channels
    dF, dD, dA = rng.normal(size=(n, C)), 0.1 * rng.normal(size=n), rng.normal(size=n)
    gr, _ = ogr.reference_sensor_grads(g, sensor, idx, dF, dD, dA)
    for name, val in gr.items():
        if val.ndim == 0:
            fd = ogr.sensor_finite_diff(g, sensor, idx, dF, dD, dA, name, h=1e-7)
            np.testing.assert_allclose(val, fd, rtol=2e-4, atol=1e-6, err_msg=name)
        else:
            for k in range(3):
                fd = ogr.sensor_finite_diff(g, sensor, idx, dF, dD, dA, name, index=k, h=1e-6)
                np.testing.assert_allclose(val[k], fd, rtol=2e-4, atol=1e-6, err_msg=f"{name}[{k}]")
    return gr


def test_camera_sensor_gradients_against_central_differences():
    g, cam, _ = _scene()
    cam = dataclasses.replace(cam, time_offset=0.004)
    gr = _check_sensor(g, cam, np.arange(0, cam.n_rays, 3))
    assert abs(float(gr["time_offset"])) > 0 and np.abs(gr["lin_vel"]).max() > 0


def test_lidar_sensor_gradients_against_central_differences():
    g, _, lid = _scene()
    gr = _check_sensor(g, lid, np.arange(0, lid.n_rays, 2))
    assert "time_offset" not in gr and np.abs(gr["ang_vel"]).max() > 0
