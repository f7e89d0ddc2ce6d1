"""Full-size configurations in the batched launch form that bench.py times (one call per stage
for all sensors of the scene, persistent queue rasterisers), against the FP64 oracle on
sampled rays:

* C2 (500k Gaussians, 1080p rolling-shutter camera), C3 (2M Gaussians, 128 x 2048 lidar sweep),
  C4 (1.5M Gaussians, 6 cameras of uneven sizes + a 64 x 1800 lidar): forward values of sampled
  rays of every sensor, and gradients.  For the gradients the upstream gradient is nonzero only
  on the sampled rays, so the exact gradient is a sum over those rays that the oracle evaluates
  over all Gaussians, element by element.
* C5 (3M Gaussians, 48 lidar sweeps of 32 / 64 / 128 beams and 12 cameras) in one call per
  stage (about 1.9e9 list entries): forward values of sampled rays and gradients, as above.

Bars as in test_gpu_parity: 1e-5 + 1e-4 |ref| per rendered element on rays without a
near-threshold decision; gradients within 1e-3 relative per tensor and per element."""
import numpy as np
import pytest
import torch

from oracle import geometry as geo
from oracle import grad as ogr
from oracle import render as rd
from scenes import synthetic as S
from tests.gpu_helpers import assert_grad_close, gpu_outputs, grad_mismatch, rtol_check

pytestmark = pytest.mark.gpu


def _binding():
    from paper_2411_16816_amd import binding
    binding.load()
    return binding


def _render(sc):
    b = _binding()
    rig = b.Rig(sc.cameras, sc.lidars)
    G = b.GaussTensors.from_numpy(sc.gaussians)
    n_s = len(rig.sensors)
    sp = b.SensorPass(rig, 0, n_s, sc.gaussians.n, 1, batched=True)
    sp.fit_capacity(G, 1.1)
    sp.status.zero_()
    sp.render(G)
    torch.cuda.synchronize()
    st = b.read_status(sp.status)
    assert st.overflow == 0 and st.n_nonfinite == 0
    return b, rig, G, sp


def _check_forward(sp, rig, g, k, idx):
    return _check_forward_at(sp, rig, g, 0, k, idx)


def _check_forward_at(sp, rig, g, first, k, idx):
    """Sampled rays of sensor k of a call starting at rig sensor `first`, against the oracle;
    returns the oracle's near mask."""
    sensor = rig.sensors[first + k]
    out = gpu_outputs(sp, k)
    ref = rd.render_sensor(g, sensor, idx)
    ok = ~ref["near"]
    # a sanity bound: the exclusion must leave most sampled rays to compare
    assert ref["near"].sum() <= max(2, 0.15 * len(idx)), (first + k, int(ref["near"].sum()), len(idx))
    for key, refv in (("F", ref["F"]), ("D", ref["D"]), ("A", ref["A"])):
        got = out[key][idx]
        bad = rtol_check(got, refv.numpy(), mask=ok)
        assert not bad.any(), (k, key, int(bad.sum()))
    if "median" in out and hasattr(sensor, "ray_az"):
        bad = rtol_check(out["median"][idx], ref["median"].numpy(), mask=ok)
        assert not bad.any(), (k, "median", int(bad.sum()))
    return ref["near"]


def _config(name):
    return {"c2": S.config_2, "c3": S.config_3, "c4": S.config_4, "c5": S.config_5}[name]()


@pytest.mark.parametrize("cfg,rays", [("c2", 24), ("c3", 24), ("c4", 6)])
def test_full_size_forward_and_gradients(cfg, rays):
    sc = _config(cfg)
    print(f"[configs] {sc.name}: {sc.gaussians.n} Gaussians, {len(sc.cameras)} cameras, {len(sc.lidars)} lidars",
          flush=True)
    b, rig, G, sp = _render(sc)
    g = sc.gaussians
    rng = np.random.default_rng(404)
    up = np.random.default_rng(405)
    dF = np.zeros(sp.n_feat, np.float32)
    dD = np.zeros(sp.n_rays, np.float32)
    dA = np.zeros(sp.n_rays, np.float32)
    picks = []
    for k, sensor in enumerate(rig.sensors):
        idx = np.sort(rng.choice(sensor.n_rays, size=rays, replace=False))
        near = _check_forward(sp, rig, g, k, idx)
        keep = idx[~near]                       # near-threshold rays get no upstream gradient
        rs, fs, C = sp.sensor_slices(k)
        dFk = up.normal(size=(len(keep), C)).astype(np.float32)
        dDk = (0.1 * up.normal(size=len(keep))).astype(np.float32)
        dAk = up.normal(size=len(keep)).astype(np.float32)
        dF[fs.start:fs.stop].reshape(-1, C)[keep] = dFk
        dD[rs.start + keep] = dDk
        dA[rs.start + keep] = dAk
        picks.append((sensor, keep, dFk, dDk, dAk))
    grads = b.zeros_like_grads(G)
    t = lambda a: torch.from_numpy(a).cuda()
    sp.raster_bwd(G, t(dF), t(dD), t(dA), grads)
    torch.cuda.synchronize()
    ref = None
    for sensor, keep, dFk, dDk, dAk in picks:
        r, _ = ogr.reference_grads(g, sensor, keep, dFk, dDk, dAk)
        ref = r if ref is None else {n: ref[n] + r[n] for n in ref}
    got = dict(means=grads.means, log_scales=grads.log_scales, quats=grads.quats, opacities=grads.opacities,
               velocities=grads.velocities, features=grads.features)
    for name in geo.Params.names:
        assert_grad_close(got[name].cpu().numpy(), ref[name], f"{cfg} {name}")


def test_full_size_c5_one_call():
    """C5's 60 sensors in one batched call per stage: about 1.9e9 (tile, Gaussian) entries (list
    positions beyond 2^31), so the adjoint keeps no per-entry rows and adds atomically.  Forward
    values of sampled rays of cameras and of 32-, 64- and 128-beam sweeps against the oracle,
    one sensor against its own per-sensor call (bit-identical), and the gradients of upstream
    gradients placed on the sampled rays only, element by element against the oracle."""
    b = _binding()
    sc = _config("c5")
    g = sc.gaussians
    n_cam, n_lid = len(sc.cameras), len(sc.lidars)
    print(f"[configs] {sc.name}: {g.n} Gaussians, {n_cam} cameras, {n_lid} lidars", flush=True)
    rig = b.Rig(sc.cameras, sc.lidars)
    G = b.GaussTensors.from_numpy(g)
    n_s = n_cam + n_lid
    sp = b.SensorPass(rig, 0, n_s, g.n, 1, batched=True)
    K = sp.fit_capacity(G, 1.05)
    print(f"[configs] one call: {K} entries, capacity {sp.k_cap}", flush=True)
    assert K <= sp.k_cap < (1 << 32) and sp.k_cap > b.ADJOINT_ROW_LIMIT
    sp.status.zero_()
    sp.render(G)
    torch.cuda.synchronize()
    st = b.read_status(sp.status)
    assert st.overflow == 0 and st.n_nonfinite == 0
    rng = np.random.default_rng(505)
    up = np.random.default_rng(506)
    dF = np.zeros(sp.n_feat, np.float32)
    dD = np.zeros(sp.n_rays, np.float32)
    dA = np.zeros(sp.n_rays, np.float32)
    sample = [0, n_cam - 1, n_cam, n_cam + 16, n_s - 1]   # cameras; sweeps of each beam group
    picks = []
    for k in sample:
        sensor = rig.sensors[k]
        idx = np.sort(rng.choice(sensor.n_rays, size=4, replace=False))
        near = _check_forward(sp, rig, g, k, idx)
        keep = idx[~near]
        rs, fs, C = sp.sensor_slices(k)
        dFk = up.normal(size=(len(keep), C)).astype(np.float32)
        dDk = (0.1 * up.normal(size=len(keep))).astype(np.float32)
        dAk = up.normal(size=len(keep)).astype(np.float32)
        dF[fs.start:fs.stop].reshape(-1, C)[keep] = dFk
        dD[rs.start + keep] = dDk
        dA[rs.start + keep] = dAk
        picks.append((sensor, keep, dFk, dDk, dAk))
    # one sensor of the call against its own per-sensor call
    one = b.SensorPass(rig, n_cam + 16, 1, g.n, 1)
    one.fit_capacity(G, 1.1)
    one.render(G)
    torch.cuda.synchronize()
    a_, p_ = gpu_outputs(sp, n_cam + 16), gpu_outputs(one, 0)
    for key in ("F", "D", "A", "T"):
        np.testing.assert_array_equal(a_[key], p_[key], err_msg=key)
    del one
    grads = b.zeros_like_grads(G)
    t = lambda x: torch.from_numpy(x).cuda()
    sp.raster_bwd(G, t(dF), t(dD), t(dA), grads)
    torch.cuda.synchronize()
    print("[configs] adjoint done; oracle gradients", flush=True)
    per_pick = [ogr.reference_grads(g, sensor, keep, dFk, dDk, dAk)[0] for sensor, keep, dFk, dDk, dAk in picks]
    ref = {n: sum(r[n] for r in per_pick) for n in geo.Params.names}
    got = dict(means=grads.means, log_scales=grads.log_scales, quats=grads.quats, opacities=grads.opacities,
               velocities=grads.velocities, features=grads.features)
    n_ill = 0
    for name in geo.Params.names:
        gg = got[name].cpu().numpy().astype(np.float64)
        assert_grad_close(gg, ref[name], f"c5 {name}", rtol=1e-3, afloor=1e-5, norm_tol=1e-3, per_element=False)
        bad = grad_mismatch(gg, ref[name], rtol=1e-3, afloor=1e-5).reshape(g.n, -1)
        rows = np.unique(np.nonzero(bad)[0])
        assert len(rows) <= 4, (name, rows[:16])
        for i in rows:
            # An element outside the bar passes only if the FP64 oracle's own value for it moves by
            # more than the GPU's error when the Gaussian's float32 inputs move by one ulp: the
            # gradient is ill-conditioned at FP32 precision (seen for Gaussians a few decimetres
            # outside a lidar's minimum range, whose angular footprint spans most of the sphere).
            spread = _ulp_spread(g, picks, per_pick, int(i), name)
            err = np.abs(gg.reshape(g.n, -1)[i] - ref[name].reshape(g.n, -1)[i])
            print(f"[configs] c5 {name}: Gaussian {i} outside the bar: error {err.max():.3g}, oracle one-ulp "
                  f"spread {spread.max():.3g}", flush=True)
            assert (err <= 2.0 * spread).all(), (name, int(i), err, spread)
            n_ill += 1
    print(f"[configs] c5: {n_ill} ill-conditioned gradient rows", flush=True)


def _ulp_spread(g, picks, per_pick, i, name):
    """Largest change of the oracle's gradient `name` of Gaussian i when each of its float32
    inputs (mean, log-scales, quaternion, opacity, velocity) moves one ulp up, or one ulp down."""
    import copy
    out = 0.0
    for direction in (np.inf, -np.inf):
        g2 = copy.deepcopy(g)
        for f in ("means", "log_scales", "quats", "opacities", "velocities"):
            a = getattr(g2, f)
            if a is not None:
                a[i] = np.nextafter(a[i], np.float32(direction))
        for (sensor, keep, dFk, dDk, dAk), base in zip(picks, per_pick):
            if not np.any(base[name].reshape(g.n, -1)[i]):
                continue   # this sensor's rays give Gaussian i no gradient
            r, _ = ogr.reference_grads(g2, sensor, keep, dFk, dDk, dAk)
            out = np.maximum(out, np.abs(r[name].reshape(g.n, -1)[i] - base[name].reshape(g.n, -1)[i]))
    return np.asarray(out)
