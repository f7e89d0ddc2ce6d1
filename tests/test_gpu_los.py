"""Lidar line-of-sight sum (the loss term L_los of the training-details appendix: the alphas of
the Gaussians a ray blends whose corrected range lies in front of its measured range minus a
margin) through the C ABI against the FP64 oracle: the forward sums within 1e-4 relative /
1e-5 absolute on every ray whose decisions are not within float32 reach of a threshold, and
the Gaussian gradients of a loss that includes the sum (SplatRenderOut.d_los) within 1e-3
relative, per sensor and batched with a camera."""
import numpy as np
import pytest
import torch

from oracle import geometry as geo
from oracle import grad as ogr
from oracle import render as rd
from scenes import synthetic as S
from tests.gpu_helpers import assert_grad_close

pytestmark = pytest.mark.gpu


def _binding():
    from paper_2411_16816_amd import binding
    binding.load()
    return binding


def _scene(seed):
    rng = np.random.default_rng(seed)
    n = 500
    mu = np.stack([rng.uniform(-14, 14, n), rng.uniform(-14, 14, n), rng.uniform(-1.5, 1.5, n)], 1)
    return S.random_gaussians(rng, mu, 8, moving_frac=0.4, log_scale_mean=-0.6)


def _lidar(seed, tile_az=16):
    lid = S.make_lidar((0, 0, 0), 0.0, 16, -15.0, 15.0, 512, tile_az=tile_az, tile_el=8, t_sweep=0.1,
                       ego_vel_world=(10.0, 1.0, 0), ego_yaw_rate=0.2, n_channels=8)
    # measured ranges over the depth span of the scene: part of each ray's Gaussians lie in front
    lid.ray_range = np.random.default_rng(seed).uniform(0.5, 16.0, lid.n_rays).astype(np.float32)
    lid.los_eps = 0.8
    return lid


def _camera():
    return S.make_camera((0, 0, 0), 0.0, 64, 48, 60.0, t_rs=0.04, ego_vel_world=(6.0, 0.5, 0), n_channels=8)


@pytest.mark.parametrize("tile_az", [16, 64])
def test_los_forward(tile_az):
    b = _binding()
    g = _scene(21)
    lid = _lidar(5, tile_az)
    print(f"[los] forward tile_az={tile_az}", flush=True)
    rig = b.Rig([], [lid])
    G = b.GaussTensors.from_numpy(g)
    sp = b.SensorPass(rig, 0, 1, g.n, 1)
    sp.fit_capacity(G)
    sp.render(G)
    torch.cuda.synchronize()
    ref = rd.render_sensor(g, lid)
    ok = ~ref["near"]
    assert ok.mean() > 0.9
    r = ref["los"].numpy()
    a = sp.outputs()["los"].cpu().numpy().astype(np.float64)
    assert (r[ok] > 0).mean() > 0.2 and (r[ok] == 0).mean() > 0.05   # both sides of the threshold
    err = np.abs(a[ok] - r[ok]) / (1e-5 + 1e-4 * np.abs(r[ok]))
    assert err.max() <= 1.0, float(err.max())
    # without measured ranges the sum is zero on every ray
    bare = _lidar(5, tile_az)
    bare.ray_range = None
    rig2 = b.Rig([], [bare])
    sp2 = b.SensorPass(rig2, 0, 1, g.n, 1)
    sp2.fit_capacity(G)
    sp2.render(G)
    torch.cuda.synchronize()
    assert float(sp2.outputs()["los"].abs().max()) == 0.0


def _upstream(sensor, seed, keep=None, with_los=True):
    up = np.random.default_rng(seed)
    R, C = sensor.n_rays, sensor.n_channels
    dF = up.normal(size=(R, C)).astype(np.float32)
    dD = (0.1 * up.normal(size=R)).astype(np.float32)
    dA = up.normal(size=R).astype(np.float32)
    dl = up.normal(size=R).astype(np.float32) if with_los else None
    if keep is not None:
        dF, dD, dA = dF * keep[:, None], dD * keep, dA * keep
        dl = None if dl is None else dl * keep
    return dF, dD, dA, dl


@pytest.mark.parametrize("batched", [False, True])
def test_los_gradients(batched):
    b = _binding()
    g = _scene(22)
    cam, lid = _camera(), _lidar(6)
    print(f"[los] gradients batched={batched}", flush=True)
    G = b.GaussTensors.from_numpy(g)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a).reshape(-1)).cuda()
    refs, ups = [], []
    for k, sensor in enumerate((cam, lid)):
        is_lid = k == 1
        dF, dD, dA, dl = _upstream(sensor, 60 + k, with_los=is_lid)
        _, out = ogr.reference_grads(g, sensor, np.arange(sensor.n_rays), dF, dD, dA, dlos=dl)
        keep = ~out["near"]
        assert keep.mean() > 0.9
        dF, dD, dA, dl = _upstream(sensor, 60 + k, keep, with_los=is_lid)   # near-decision rays: no gradient
        ref, _ = ogr.reference_grads(g, sensor, np.arange(sensor.n_rays), dF, dD, dA, dlos=dl)
        refs.append(ref)
        ups.append((dF, dD, dA, dl if is_lid else np.zeros(sensor.n_rays, np.float32)))
    rig = b.Rig([cam], [lid])
    if batched:
        passes = [(b.SensorPass(rig, 0, 2, g.n, 1, batched=True), [0, 1])]
    else:
        passes = [(b.SensorPass(rig, 0, 1, g.n, 1), [0]), (b.SensorPass(rig, 1, 1, g.n, 1), [1])]
    got = []
    for sp, ks in passes:
        sp.fit_capacity(G)
        sp.render(G)
        dF = np.concatenate([ups[k][0].reshape(-1) for k in ks])
        dD = np.concatenate([ups[k][1] for k in ks])
        dA = np.concatenate([ups[k][2] for k in ks])
        dl = np.concatenate([ups[k][3] for k in ks])
        grads = b.zeros_like_grads(G)
        sp.raster_bwd(G, t(dF), t(dD), t(dA), grads, d_los=t(dl))
        torch.cuda.synchronize()
        got.append(grads)
    want = {name: refs[0][name] + refs[1][name] for name in geo.Params.names}
    for name in geo.Params.names:
        gg = sum(getattr(gr, name).cpu().numpy().astype(np.float64) for gr in got)
        rr = want[name]
        assert_grad_close(gg, rr, name)
    # the line-of-sight term is present: the lidar's opacity gradient moves with it
    ref_no, _ = ogr.reference_grads(g, lid, np.arange(lid.n_rays), *ups[1][:3])
    assert np.linalg.norm(ref_no["opacities"] - refs[1]["opacities"]) > 1e-3 * np.linalg.norm(refs[1]["opacities"])
