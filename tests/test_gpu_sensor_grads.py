"""Sensor parameters through the C ABI against the FP64 oracle: a camera with a time offset
(Sec. 3.2: timestamp minus mid-exposure) renders within 1e-4 relative / 1e-5 absolute, and the
gradients with respect to the sensors' linear and angular velocities and the camera time offset
(SplatGrads.sensor_*) match the oracle's autograd within 1e-3 relative, alone and batched."""
import numpy as np
import pytest
import torch

from oracle import grad as ogr
from oracle import render as rd
from scenes import synthetic as S
from tests.gpu_helpers import assert_grad_close

pytestmark = pytest.mark.gpu


def _binding():
    from paper_2411_16816_amd import binding
    binding.load()
    return binding


def _sensors(time_offset=0.006):
    cam = S.make_camera((0, 0, 0), 0.0, 64, 48, 60.0, t_rs=0.04, ego_vel_world=(6.0, 0.5, 0), ego_yaw_rate=0.3,
                        n_channels=16)
    cam.time_offset = time_offset
    lid = S.make_lidar((0, 0, 0), 0.0, 16, -15.0, 15.0, 256, tile_az=16, tile_el=8, t_sweep=0.1,
                       ego_vel_world=(10.0, 1.0, 0), ego_yaw_rate=0.2, feat_offset=3, n_channels=8)
    return cam, lid


def _scene(seed):
    rng = np.random.default_rng(seed)
    n = 300
    mu = np.concatenate([np.stack([rng.uniform(2, 12, n), rng.uniform(-5, 5, n), rng.uniform(-3.5, 3.5, n)], 1),
                         np.stack([rng.uniform(-10, 10, n), rng.uniform(-10, 10, n), rng.uniform(-1.5, 1.5, n)], 1)])
    return S.random_gaussians(rng, mu, 16, rgb=True, moving_frac=0.5, log_scale_mean=-0.6)


def _upstream(sensor, seed, keep=None):
    up = np.random.default_rng(seed)
    R, C = sensor.n_rays, sensor.n_channels
    dF = up.normal(size=(R, C)).astype(np.float32)
    dD = (0.1 * up.normal(size=R)).astype(np.float32)
    dA = up.normal(size=R).astype(np.float32)
    if keep is not None:
        dF, dD, dA = dF * keep[:, None], dD * keep, dA * keep
    return dF, dD, dA


def test_camera_time_offset_forward():
    b = _binding()
    g = _scene(11)
    cam, _ = _sensors()
    rig = b.Rig([cam], [])
    G = b.GaussTensors.from_numpy(g)
    sp = b.SensorPass(rig, 0, 1, g.n, 1)
    sp.fit_capacity(G)
    sp.render(G)
    torch.cuda.synchronize()
    ref = rd.render_sensor(g, cam)
    ok = ~ref["near"]
    assert ok.mean() > 0.9
    o = sp.outputs()
    for key, r in (("feat", ref["F"].numpy().reshape(-1, 16)), ("depth", ref["D"].numpy()), ("alpha", ref["A"].numpy())):
        a = o[key].cpu().numpy().astype(np.float64).reshape(r.shape)
        err = np.abs(a[ok] - r[ok]) / (1e-5 + 1e-4 * np.abs(r[ok]))
        assert err.max() <= 1.0, (key, float(err.max()))
    # the offset matters: without it the image differs
    cam0, _ = _sensors(0.0)
    ref0 = rd.render_sensor(g, cam0)
    assert float((ref0["A"] - ref["A"]).abs().max()) > 1e-3


@pytest.mark.parametrize("batched", [False, True])
def test_sensor_velocity_and_time_offset_gradients(batched):
    b = _binding()
    g = _scene(12)
    cam, lid = _sensors()
    G = b.GaussTensors.from_numpy(g)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a).reshape(-1)).cuda()
    refs, ups = [], []
    for k, sensor in enumerate((cam, lid)):
        dF, dD, dA = _upstream(sensor, 40 + k)
        _, out = ogr.reference_sensor_grads(g, sensor, np.arange(sensor.n_rays), dF, dD, dA)
        keep = ~out["near"]
        assert keep.mean() > 0.9
        dF, dD, dA = _upstream(sensor, 40 + k, keep)   # near-decision rays carry no gradient
        ref, _ = ogr.reference_sensor_grads(g, sensor, np.arange(sensor.n_rays), dF, dD, dA)
        refs.append(ref)
        ups.append((dF, dD, dA))
    rig = b.Rig([cam], [lid])
    if batched:
        passes = [(b.SensorPass(rig, 0, 2, g.n, 1, batched=True), [0, 1])]
    else:
        passes = [(b.SensorPass(rig, 0, 1, g.n, 1), [0]), (b.SensorPass(rig, 1, 1, g.n, 1), [1])]
    got = {0: {}, 1: {}}
    for sp, ks in passes:
        sp.fit_capacity(G)
        sp.render(G)
        n = len(ks)
        sg = {"sensor_lin_vel": torch.zeros(n, 3, device="cuda"), "sensor_ang_vel": torch.zeros(n, 3, device="cuda"),
              "sensor_time_offset": torch.zeros(n, device="cuda")}
        dF = np.concatenate([ups[k][0].reshape(-1) for k in ks])
        dD = np.concatenate([ups[k][1] for k in ks])
        dA = np.concatenate([ups[k][2] for k in ks])
        sp.raster_bwd(G, t(dF), t(dD), t(dA), b.zeros_like_grads(G), sensor_grads=sg)
        torch.cuda.synchronize()
        for j, k in enumerate(ks):
            got[k] = {"lin_vel": sg["sensor_lin_vel"][j].cpu().numpy(), "ang_vel": sg["sensor_ang_vel"][j].cpu().numpy(),
                      "time_offset": sg["sensor_time_offset"][j].cpu().numpy()}
    for k in (0, 1):
        for name, r in refs[k].items():
            assert_grad_close(got[k][name], r, f"sensor {k} {name}")
    assert float(got[1]["time_offset"]) == 0.0   # the lidar entry is untouched
