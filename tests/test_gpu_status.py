"""Asynchronous status conditions (SplatStatus) and the inputs that raise them: non-finite
Gaussian parameters (counted, culled, and without effect on the other Gaussians' outputs and
gradients), and lidar rays outside the sweep's +-t_rs/2 window (counted, still rendered as the
oracle renders them).  Through the C ABI, against the FP64 oracle."""
import numpy as np
import pytest
import torch

from oracle import render as rd
from scenes import synthetic as S
from tests.gpu_helpers import gpu_outputs, grad_mismatch, rtol_check

pytestmark = pytest.mark.gpu


def _binding():
    from paper_2411_16816_amd import binding
    binding.load()
    return binding


def _poison(g, rng, k):
    """Copies of k Gaussians placed in view, each with one non-finite parameter kind."""
    kinds = ["mean_nan", "mean_inf", "scale_inf", "scale_nan", "quat_nan", "opac_nan", "vel_nan", "vel_inf"]
    pick = rng.choice(g.n, size=k, replace=False)
    bad = g.subset(pick)
    tags = []
    for i in range(k):
        kind = kinds[i % len(kinds)]
        tags.append(kind)
        if kind == "mean_nan":
            bad.means[i, 1] = np.nan
        elif kind == "mean_inf":
            bad.means[i, 2] = np.inf
        elif kind == "scale_inf":
            bad.log_scales[i, 0] = np.inf
        elif kind == "scale_nan":
            bad.log_scales[i, 2] = np.nan
        elif kind == "quat_nan":
            bad.quats[i, 0] = np.nan
        elif kind == "opac_nan":
            bad.opacities[i] = np.nan
        elif kind == "vel_nan":
            bad.velocities[i, 0] = np.nan
        else:
            bad.velocities[i, 1] = -np.inf
    return bad, tags


def _cat(a, b):
    v = None if a.velocities is None else np.concatenate([a.velocities, b.velocities])
    return S.Gaussians(np.concatenate([a.means, b.means]), np.concatenate([a.log_scales, b.log_scales]),
                       np.concatenate([a.quats, b.quats]), np.concatenate([a.opacities, b.opacities]), v,
                       np.concatenate([a.features, b.features]))


@pytest.mark.parametrize("kind", ["camera", "lidar"])
def test_nonfinite_gaussians_counted_and_harmless(kind):
    b = _binding()
    rng = np.random.default_rng(61)
    if kind == "camera":
        mu = S.road_slab(rng, 6000, (2.0, 40.0), (-10.0, 10.0), 4.0)
        sensor = S.make_camera((0, 0, 1.5), 0.0, 160, 120, 150.0, t_rs=0.03, ego_vel_world=(10.0, 0, 0),
                               n_channels=16)
        cams, lids = [sensor], []
    else:
        mu = S.uniform_box(rng, 6000, (-25, -25, -2), (25, 25, 2))
        sensor = S.make_lidar((0, 0, 0), 0.0, 32, -20.0, 10.0, 512, t_sweep=0.1, ego_vel_world=(10.0, 0, 0),
                              feat_offset=3, n_channels=8)
        cams, lids = [], [sensor]
    g = S.random_gaussians(rng, mu, 16, rgb=True, moving_frac=1.0)
    # poison copies of Gaussians the sensor sees, so every one is inside the depth / range limits
    # (except the non-finite means, which fail those tests)
    bad, tags = _poison(g, rng, 40)
    gg = _cat(g, bad)
    rig = b.Rig(cams, lids)
    outs, grads = [], []
    up = np.random.default_rng(62)
    R, C = sensor.n_rays, sensor.n_channels
    dF = torch.from_numpy(up.normal(size=R * C).astype(np.float32)).cuda()
    dD = torch.from_numpy((0.1 * up.normal(size=R)).astype(np.float32)).cuda()
    dA = torch.from_numpy(up.normal(size=R).astype(np.float32)).cuda()
    for scene in (g, gg):
        G = b.GaussTensors.from_numpy(scene)
        sp = b.SensorPass(rig, 0, 1, scene.n, 1)
        sp.fit_capacity(G)
        sp.status.zero_()
        sp.render(G)
        gr = b.zeros_like_grads(G)
        sp.raster_bwd(G, dF, dD, dA, gr)
        torch.cuda.synchronize()
        outs.append((gpu_outputs(sp, 0), b.read_status(sp.status)))
        grads.append(gr)
    (clean, st0), (poisoned, st1) = outs
    assert st0.n_nonfinite == 0
    # every poisoned copy is counted once: means fail the frame test, the others the projection
    print(f"[status] {kind}: n_nonfinite {st1.n_nonfinite} of {len(tags)} poisoned ({sorted(set(tags))})", flush=True)
    assert st1.n_nonfinite == len(tags)
    # the finite Gaussians render exactly as without the poisoned ones (same order, same sums)
    for key in ("F", "D", "A", "T", "last"):
        np.testing.assert_array_equal(clean[key], poisoned[key], err_msg=key)
    # the finite Gaussians' gradients are those of the clean scene; their per-Gaussian sums over
    # tiles are float atomics whose order follows the schedule, so two runs agree to the
    # run-to-run bar of the adjoint (1e-4 relative per element, 1e-5 of the largest), not bit for bit
    n = g.n
    for name in ("means", "log_scales", "quats", "opacities", "velocities", "features"):
        a = getattr(grads[0], name).cpu().numpy()
        p = getattr(grads[1], name).cpu().numpy()
        bad = grad_mismatch(p[:n], a, rtol=1e-4, afloor=1e-5)
        assert not bad.any(), (name, int(bad.sum()))
        assert (p[n:] == 0).all(), name                      # culled: no gradient at all


def test_ray_time_outside_the_sweep_counted_and_rendered():
    """Rays whose time lies beyond +-t_rs/2 are counted in n_rays_time and rendered at their
    own time, as the oracle renders them (rolling-shutter mean at that time)."""
    b = _binding()
    rng = np.random.default_rng(63)
    mu = S.uniform_box(rng, 3000, (-20, -20, -2), (20, 20, 2))
    g = S.random_gaussians(rng, mu, 16, rgb=True, moving_frac=0.5)
    lid = S.make_lidar((0, 0, 0), 0.0, 16, -20.0, 10.0, 256, t_sweep=0.1, ego_vel_world=(15.0, 0, 0),
                       feat_offset=3, n_channels=8)
    lid.ray_t = lid.ray_t.copy()
    late = rng.choice(lid.n_rays, size=77, replace=False)
    lid.ray_t[late] = np.where(rng.uniform(size=77) < 0.5, -1, 1).astype(np.float32) * \
        rng.uniform(0.051, 0.2, 77).astype(np.float32)
    inside = np.setdiff1d(np.arange(lid.n_rays), late)[:5]
    lid.ray_t[inside[:3]] = np.float32(0.05)                 # exactly t_rs / 2: not counted
    lid.ray_t[inside[3:5]] = np.float32(-0.05)
    rig = b.Rig([], [lid])
    G = b.GaussTensors.from_numpy(g)
    sp = b.SensorPass(rig, 0, 1, g.n, 1)
    sp.fit_capacity(G)
    sp.status.zero_()
    sp.render(G)
    torch.cuda.synchronize()
    st = b.read_status(sp.status)
    assert st.n_rays_time == 77 and st.n_rays_invalid == 0
    out = gpu_outputs(sp, 0)
    idx = np.sort(np.concatenate([late, inside]))
    ref = rd.render_sensor(g, lid, idx)
    ok = ~ref["near"]
    for key in ("F", "D", "A"):
        bad = rtol_check(out[key][idx], ref[key].detach().numpy(), 1e-4, 1e-5, ok)
        assert not bad.any(), (key, int(bad.sum()))
