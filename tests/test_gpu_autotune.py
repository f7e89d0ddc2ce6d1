"""Tile-shape autotuner: every candidate layout renders the same result (BOX candidate rule), so
the tuner's choice is free; it must return one of the candidates."""
import json

import numpy as np
import pytest
import torch

from scenes import synthetic as S
from tests.gpu_helpers import gpu_outputs, last_ids_gpu

pytestmark = pytest.mark.gpu


def _binding():
    from paper_2411_16816_amd import binding
    binding.load()
    return binding


def _scene():
    rng = np.random.default_rng(307)
    mu = S.road_slab(rng, 5000, (0.5, 40.0), (-15.0, 15.0), 5.0)
    g = S.random_gaussians(rng, mu, 16, rgb=True, moving_frac=0.3)
    cam = S.make_camera((0, 0, 1.5), 1.0, 200, 120, 170.0, t_rs=0.03, ego_vel_world=(12.0, 0, 0),
                        ego_yaw_rate=0.2, n_channels=16)
    lid = S.make_lidar((0, 0, 1.8), 3.0, 32, -25.0, 15.0, 512, t_sweep=0.1, ego_vel_world=(12.0, 0, 0),
                       ego_yaw_rate=0.2, tile_az=32, tile_el=8, feat_offset=3, n_channels=8)
    return g, cam, lid


def _render(b, G, sensor, is_camera, up):
    rig = b.Rig([sensor], []) if is_camera else b.Rig([], [sensor])
    sp = b.SensorPass(rig, 0, 1, G.n, 1, batched=True)
    sp.fit_capacity(G, 1.3)
    sp.render(G)
    grads = b.zeros_like_grads(G)
    dF, dD, dA = (torch.from_numpy(a).cuda() for a in up(sp))
    sp.raster_bwd(G, dF, dD, dA, grads)
    torch.cuda.synchronize()
    assert b.read_status(sp.status).overflow == 0
    o = gpu_outputs(sp, 0)
    # `last` is a position in the ray's tile list, which depends on the layout: compare the
    # Gaussian it names instead
    o["last"] = last_ids_gpu(sp, 0, sensor, np.arange(sensor.n_rays), o["last"])
    return o, grads


@pytest.mark.parametrize("kind", ["camera", "lidar"])
def test_candidate_layouts_render_identically(kind):
    b = _binding()
    from paper_2411_16816_amd import autotune as at
    g, cam, lid = _scene()
    G = b.GaussTensors.from_numpy(g)
    is_camera = kind == "camera"
    sensor = cam if is_camera else lid
    cands = at.camera_candidates(sensor) if is_camera else at.lidar_candidates(sensor)
    assert len(cands) >= 4

    def up(sp):
        r = np.random.default_rng(9)
        return (r.normal(size=sp.n_feat).astype(np.float32), (0.1 * r.normal(size=sp.n_rays)).astype(np.float32),
                r.normal(size=sp.n_rays).astype(np.float32))

    ref_o, ref_g = _render(b, G, cands[0], is_camera, up)
    for c in cands[1:]:
        print(f"[autotune] {kind} layout {at._shape(c, is_camera)}", flush=True)
        o, gr = _render(b, G, c, is_camera, up)
        for key in ref_o:
            np.testing.assert_array_equal(o[key], ref_o[key], err_msg=f"{kind} {at._shape(c, is_camera)} {key}")
        for name in ("means", "log_scales", "quats", "opacities", "velocities", "features"):
            x = getattr(gr, name).cpu().numpy().astype(np.float64)
            y = getattr(ref_g, name).cpu().numpy().astype(np.float64)
            assert np.linalg.norm(x - y) <= 1e-5 * np.linalg.norm(y), (kind, name)


def test_tune_rig_picks_a_candidate(tmp_path, monkeypatch):
    b = _binding()
    from paper_2411_16816_amd import autotune as at
    monkeypatch.setattr(at, "CACHE_PATH", str(tmp_path / "autotune_cache.json"))
    monkeypatch.setattr(at, "_cache", {})
    monkeypatch.setattr(at, "_loaded", False)
    g, cam, lid = _scene()
    G = b.GaussTensors.from_numpy(g)
    cams, lids, report = at.tune_rig([cam], [lid], G, steps=2, warmup=1)
    assert (cams[0].tile_w, cams[0].tile_h) in at.CAMERA_TILES
    assert at._shape(lids[0], False) in [at._shape(c, False) for c in at.lidar_candidates(lid)]
    assert len(report[0][1]) == len(at.CAMERA_TILES)
    # cached: a second call returns the same choice without timing
    cams2, lids2, report2 = at.tune_rig([cam], [lid], G)
    assert report2[0][1] == [] and report2[1][1] == []
    assert (cams2[0].tile_w, cams2[0].tile_h) == (cams[0].tile_w, cams[0].tile_h)
    # persisted: a fresh process state reads the same choices back from the JSON file
    stored = json.loads((tmp_path / "autotune_cache.json").read_text())
    assert len(stored) == 2 and all(k.startswith(at._arch() + "|") for k in stored)
    monkeypatch.setattr(at, "_cache", {})
    monkeypatch.setattr(at, "_loaded", False)
    cams3, lids3, report3 = at.tune_rig([cam], [lid], G)
    assert report3[0][1] == [] and report3[1][1] == []
    assert at._shape(lids3[0], False) == at._shape(lids[0], False)
