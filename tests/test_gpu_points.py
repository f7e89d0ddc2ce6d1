"""Lidar points to rasterisation rays (splat_lidar_points_to_rays; App. A "Lidar points to
rasterization points") through the C ABI against the FP64 oracle (oracle/points.py) on the same
float32 inputs: azimuth (compared on the circle), elevation and range within 1e-4 relative /
1e-5 absolute.  Sizes with a ragged tail, the 16-byte and the unaligned path, a full 128 x 2048
sweep, edge cases, and the rays fed to the lidar rasteriser."""
import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

from oracle import points as op
from oracle import render as rd
from scenes import synthetic as S

pytestmark = pytest.mark.gpu


def _binding():
    from paper_2411_16816_amd import binding
    binding.load()
    return binding


def _sweep(seed, n):
    """Points of a sweep around a sensor at (3, -1, 1.8) yawed 25 deg: ranges 1-120 m, elevations
    -25..15 deg, some right on the azimuth seam; times over a 100 ms sweep."""
    rng = np.random.default_rng(seed)
    R = Rotation.from_euler("z", 25, degrees=True).as_matrix().T   # world -> sensor
    c = np.array([3.0, -1.0, 1.8])
    az = rng.uniform(0, 2 * np.pi, n)
    az[::97] = rng.choice([0.0, 1e-7, 2 * np.pi - 1e-7], len(az[::97]))
    el = np.radians(rng.uniform(-25, 15, n))
    r = rng.uniform(1.0, 120.0, n)
    xs = np.stack([r * np.cos(el) * np.cos(az), r * np.cos(el) * np.sin(az), r * np.sin(el)], 1)
    pts = xs @ R + c                      # sensor frame -> world
    t = rng.uniform(-0.05, 0.05, n)
    lin, ang = np.array([15.0, 0.4, 0.0]), np.array([0.0, 0.0, 0.3])
    return (pts.astype(np.float32), t.astype(np.float32), R.astype(np.float32),
            (-(R @ c)).astype(np.float32), lin.astype(np.float32), ang.astype(np.float32))


def _close(a, r, what, circular=False):
    a = a.astype(np.float64)
    d = np.abs(((a - r + np.pi) % (2 * np.pi)) - np.pi) if circular else np.abs(a - r)
    err = d / (1e-5 + 1e-4 * np.abs(r))
    assert float(err.max(initial=0.0)) <= 1.0, (what, float(err.max()))


def _check(b, pts, t, R, ts, lin, ang, offset=0):
    n = pts.shape[0]
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    if offset:   # views starting `offset` floats into larger buffers: not 16-byte aligned
        P = torch.zeros(n * 3 + offset, device="cuda")
        P[offset:] = dev(pts.reshape(-1))
        T = torch.zeros(n + offset, device="cuda")
        T[offset:] = dev(t)
        Pv, Tv = P[offset:].view(n, 3), T[offset:]
    else:
        Pv, Tv = dev(pts), dev(t)
    az, el, rg = b.points_to_rays(Pv, Tv, R, ts, lin, ang)
    torch.cuda.synchronize()
    ra, re, rr = op.points_to_rays(pts.astype(np.float64), t.astype(np.float64), R.astype(np.float64),
                                   ts.astype(np.float64), lin.astype(np.float64), ang.astype(np.float64))
    a = az.cpu().numpy()
    assert np.all((a >= 0) & (a < np.float32(2 * np.pi)))
    _close(a, ra, "azimuth", circular=True)
    _close(el.cpu().numpy(), re, "elevation")
    _close(rg.cpu().numpy(), rr, "range")
    return az, el, rg


@pytest.mark.parametrize("n,offset", [(100003, 0), (100003, 1), (4, 0), (7, 0), (262144, 0)])
def test_points_to_rays_matches_oracle(n, offset):
    b = _binding()
    print(f"[points] n={n} offset={offset}", flush=True)
    _check(b, *_sweep(n + offset, n), offset=offset)


def test_points_to_rays_edge_cases():
    b = _binding()
    I = np.eye(3, dtype=np.float32)
    z = np.zeros(3, np.float32)
    # no points: a no-op
    e = torch.empty(0, device="cuda")
    b.points_to_rays(torch.empty(0, 3, device="cuda"), e, I, z)
    # a point at the origin, one on each axis, one non-finite; no velocities; no range output
    pts = np.array([[0, 0, 0], [2, 0, 0], [0, 0, -3], [np.nan, 1, 1], [-1, -0.0, 0]], np.float32)
    P, T = torch.from_numpy(pts).cuda(), torch.zeros(5, device="cuda")
    az, el, rg = b.points_to_rays(P, T, I, z, with_range=False)
    assert rg is None
    a, e = az.cpu().numpy(), el.cpu().numpy()
    assert a[0] == 0.0 and e[0] == 0.0
    assert a[1] == 0.0 and e[1] == 0.0
    assert abs(e[2] + np.pi / 2) < 1e-6
    assert np.isnan(a[3]) and np.isnan(e[3])
    assert abs(a[4] - np.pi) < 1e-6 and a[4] < 2 * np.pi
    # a missing pose is an argument error
    from paper_2411_16816_amd.binding import SplatError
    with pytest.raises(SplatError):
        b.points_to_rays(P, T, None, z)


def test_rays_from_points_render_like_the_oracle():
    """Rays made on the GPU from a sweep's points (times, azimuths, elevations, ranges) feed the
    lidar rasteriser; its outputs, line-of-sight sum included, match the oracle rendering the
    same float32 rays."""
    b = _binding()
    rng = np.random.default_rng(9)
    n_g = 600
    mu = np.stack([rng.uniform(-25, 25, n_g), rng.uniform(-25, 25, n_g), rng.uniform(-1.5, 2.5, n_g)], 1)
    g = S.random_gaussians(rng, mu, 8, moving_frac=0.3, log_scale_mean=-0.5)
    lid = S.make_lidar((3.0, -1.0, 1.8), 25.0, 32, -25.0, 15.0, 512, tile_az=16, tile_el=8, t_sweep=0.1,
                       ego_vel_world=(15.0, 0.4, 0.0), ego_yaw_rate=0.3, n_channels=8)
    # the sweep's points: a Gaussian mean or a far return along every ray of the sensor
    n = lid.n_rays
    k = rng.integers(0, n_g, n)
    pts = (mu[k] + rng.normal(0, 0.2, (n, 3))).astype(np.float32)
    t = rng.uniform(-0.05, 0.05, n).astype(np.float32)
    P, T = torch.from_numpy(pts).cuda(), torch.from_numpy(t).cuda()
    az, el, rg = b.points_to_rays(P, T, lid.R, lid.t, lid.lin_vel, lid.ang_vel)
    torch.cuda.synchronize()
    import dataclasses
    lid2 = dataclasses.replace(lid, ray_az=az.cpu().numpy(), ray_el=el.cpu().numpy(), ray_t=t,
                               ray_range=rg.cpu().numpy())
    rig = b.Rig([], [lid2])
    G = b.GaussTensors.from_numpy(g)
    sp = b.SensorPass(rig, 0, 1, g.n, 1)
    sp.fit_capacity(G)
    sp.render(G)
    torch.cuda.synchronize()
    ref = rd.render_sensor(g, lid2)
    ok = ~ref["near"]
    assert ok.mean() > 0.9
    o = sp.outputs()
    A = ref["A"].numpy()
    assert (A[ok] > 0.1).mean() > 0.5   # the rays meet the Gaussians their points came from
    for key, r in (("alpha", A), ("depth", ref["D"].numpy()), ("los", ref["los"].numpy())):
        a = o[key].cpu().numpy().astype(np.float64)
        err = np.abs(a[ok] - r[ok]) / (1e-5 + 1e-4 * np.abs(r[ok]))
        assert err.max() <= 1.0, (key, float(err.max()))
