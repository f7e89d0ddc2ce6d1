"""The batched step captured as a hipGraph (splat_pipeline_*), against eager calls of the same
batched step on separate buffers.  The rig is moved between replays (eager work and host
synchronisation in between), and every replay must reproduce the eager result for the rig's
current state: forward outputs and list statistics bit-identical, gradients equal up to the
order in which a workgroup's wavefronts add their partial sums."""
import numpy as np
import pytest
import torch

from scenes import synthetic as S

pytestmark = pytest.mark.gpu


def _binding():
    from paper_2411_16816_amd import binding
    binding.load()
    return binding


def _sensors(k, width=160):
    cam = S.make_camera((0.4 * k, 0.1 * k, 1.5), 2.0 + 3.0 * k, width, 96, 150.0, t_rs=0.03,
                        ego_vel_world=(12.0, 0.0, 0.0), ego_yaw_rate=0.1 * k, n_channels=16)
    lid = S.make_lidar((0.3 * k, 0.0, 1.8), 5.0 + 4.0 * k, 16, -20.0, 10.0, 256, t_sweep=0.1,
                       ego_vel_world=(12.0, 0.0, 0.0), tile_az=16, feat_offset=3, n_channels=8)
    return cam, lid


def _scene():
    rng = np.random.default_rng(211)
    mu = S.road_slab(rng, 6000, (0.5, 50.0), (-20.0, 20.0), 6.0)
    return S.random_gaussians(rng, mu, 16, rgb=True, moving_frac=0.3)


def test_pipeline_replays_match_eager():
    b = _binding()
    g = _scene()
    cam, lid = _sensors(0)
    rig = b.Rig([cam], [lid])
    G = b.GaussTensors.from_numpy(g)
    sp = b.SensorPass(rig, 0, 2, g.n, 1, batched=True)
    sp.fit_capacity(G, margin=2.0)
    ref = b.SensorPass(rig, 0, 2, g.n, sp.k_cap, batched=True)
    up = np.random.default_rng(5)
    dF = torch.from_numpy(up.normal(size=sp.n_feat).astype(np.float32)).cuda()
    dD = torch.from_numpy((0.1 * up.normal(size=sp.n_rays)).astype(np.float32)).cuda()
    dA = torch.from_numpy(up.normal(size=sp.n_rays).astype(np.float32)).cuda()
    gpipe = b.zeros_like_grads(G)
    pipe = b.Pipeline(sp, G, b.BOX, gpipe, dF, dD, dA)
    prev = None
    for k in range(3):
        print(f"[pipeline] replay {k}", flush=True)
        rig.update(*[[s] for s in _sensors(k)])
        ref.status.zero_()
        ref.render(G)
        gref = b.zeros_like_grads(G)
        ref.raster_bwd(G, dF, dD, dA, gref)
        torch.cuda.synchronize()
        pipe.run()
        torch.cuda.synchronize()
        s_p, s_r = b.read_status(sp.status), b.read_status(ref.status)
        assert s_p.overflow == 0 and s_r.overflow == 0
        assert s_p.n_isect == s_r.n_isect
        o_p, o_r = sp.outputs(), ref.outputs()
        for key in ("feat", "depth", "alpha", "t_final", "last"):
            np.testing.assert_array_equal(o_p[key].cpu().numpy(), o_r[key].cpu().numpy(), err_msg=key)
        lid_rays = sp.sensor_slices(1)[0]          # the median is written for lidar rays only
        np.testing.assert_array_equal(o_p["median"][lid_rays].cpu().numpy(), o_r["median"][lid_rays].cpu().numpy())
        for name in ("means", "log_scales", "quats", "opacities", "velocities", "features"):
            x = getattr(gpipe, name).cpu().numpy().astype(np.float64)
            y = getattr(gref, name).cpu().numpy().astype(np.float64)
            assert np.linalg.norm(y) > 0, name
            assert np.linalg.norm(x - y) <= 1e-5 * np.linalg.norm(y), (k, name)
        # the replay saw the moved sensors
        cur = o_p["depth"].cpu().numpy().copy()
        if prev is not None:
            assert not np.array_equal(cur, prev)
        prev = cur
        # the forward counts pairs only when the step asks for it
        assert s_p.n_pairs == 0 and s_p.n_stopped == 0
    # a counting pipeline (forward only) reports the eager counting forward's pairs
    pipe_c = b.Pipeline(sp, G, b.BOX, count_pairs=True)
    pipe_c.run()
    ref.status.zero_()
    ref.raster_fwd(G, count_pairs=True)
    torch.cuda.synchronize()
    s_c, s_r = b.read_status(sp.status), b.read_status(ref.status)
    assert s_c.n_pairs > 0 and s_c.n_pairs == s_r.n_pairs and s_c.n_stopped == s_r.n_stopped
    pipe_c.close()
    # a sensor with another tile count invalidates the pipeline: nothing is launched
    cam_w, lid_w = _sensors(0, width=192)
    rig.update([cam_w], [lid_w])
    with pytest.raises(b.SplatError):
        pipe.run()
    pipe.close()
    torch.cuda.synchronize()


def test_pipeline_with_line_of_sight_and_cap():
    """A lidar with measured ranges (line-of-sight sum, its upstream gradient d_los) and the
    training-time cap (priorities redrawn between replays, copied into the same device arrays):
    every replay reproduces the eager batched calls, the sums and dropped flags included."""
    b = _binding()
    g = _scene()
    cam, lid = _sensors(0)
    lid = S.make_lidar((0.0, 0.0, 1.8), 5.0, 16, -20.0, 10.0, 512, t_sweep=0.1, ego_vel_world=(12.0, 0.0, 0.0),
                       tile_az=64, feat_offset=3, n_channels=8)   # 64 x 8 = 512 rays per tile: half dropped
    rng = np.random.default_rng(17)
    lid.ray_range = rng.uniform(1.0, 40.0, lid.n_rays).astype(np.float32)
    lid.ray_priority = rng.integers(0, 1 << 16, lid.n_rays).astype(np.uint16)
    rig = b.Rig([cam], [lid])
    G = b.GaussTensors.from_numpy(g)
    sp = b.SensorPass(rig, 0, 2, g.n, 1, batched=True)
    sp.fit_capacity(G, margin=2.0)
    ref = b.SensorPass(rig, 0, 2, g.n, sp.k_cap, batched=True)
    up = np.random.default_rng(6)
    dF = torch.from_numpy(up.normal(size=sp.n_feat).astype(np.float32)).cuda()
    dD = torch.from_numpy((0.1 * up.normal(size=sp.n_rays)).astype(np.float32)).cuda()
    dA = torch.from_numpy(up.normal(size=sp.n_rays).astype(np.float32)).cuda()
    dl = torch.from_numpy(up.normal(size=sp.n_rays).astype(np.float32)).cuda()
    gpipe = b.zeros_like_grads(G)
    pipe = b.Pipeline(sp, G, b.BOX, gpipe, dF, dD, dA, d_los=dl)
    lid_rays = sp.sensor_slices(1)[0]
    prev = None
    for k in range(3):
        print(f"[pipeline] los + cap replay {k}", flush=True)
        lid.ray_priority = rng.integers(0, 1 << 16, lid.n_rays).astype(np.uint16)
        rig.update(lidars=[lid])
        ref.render(G)
        gref = b.zeros_like_grads(G)
        ref.raster_bwd(G, dF, dD, dA, gref, d_los=dl)
        torch.cuda.synchronize()
        pipe.run()
        torch.cuda.synchronize()
        o_p, o_r = sp.outputs(), ref.outputs()
        for key in ("feat", "depth", "alpha", "t_final", "last"):
            np.testing.assert_array_equal(o_p[key].cpu().numpy(), o_r[key].cpu().numpy(), err_msg=key)
        for key in ("median", "los", "dropped"):
            np.testing.assert_array_equal(o_p[key][lid_rays].cpu().numpy(), o_r[key][lid_rays].cpu().numpy(),
                                          err_msg=key)
        dropped = o_p["dropped"][lid_rays].cpu().numpy()
        assert 0.3 < dropped.mean() < 0.6 and float(o_p["los"][lid_rays].abs().max()) > 0
        for name in ("means", "log_scales", "quats", "opacities", "velocities", "features"):
            x = getattr(gpipe, name).cpu().numpy().astype(np.float64)
            y = getattr(gref, name).cpu().numpy().astype(np.float64)
            assert np.linalg.norm(y) > 0, name
            assert np.linalg.norm(x - y) <= 1e-5 * np.linalg.norm(y), (k, name)
        if prev is not None:   # a new shuffle drops another set of rays
            assert (dropped != prev).any()
        prev = dropped
