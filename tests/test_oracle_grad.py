"""Pins of the oracle's reference gradient: central finite differences of the FP64 forward
against autograd (every parameter kind, camera and lidar, rolling shutter on), and the closed
form of the over-operator derivative dO/dalpha_i = T_i f_i - sum_{j>i} f_j alpha_j T_j / (1 - alpha_i)."""
import math

import numpy as np
import pytest
import torch

from oracle import geometry as geo
from oracle import grad as gr
from oracle import render as rd
from scenes import synthetic as S


def _scene(kind, seed):
    rng = np.random.default_rng(seed)
    if kind == "camera":
        sensor = S.make_camera((0, 0, 0), 0.0, 24, 18, 30.0, t_rs=0.04, ego_vel_world=(6.0, 0.5, 0),
                               ego_yaw_rate=0.3, n_channels=4, tile=(8, 8))
        n = 30
        means = np.stack([rng.uniform(2, 10, n), rng.uniform(-2.5, 2.5, n), rng.uniform(-2, 2, n)], 1)
        ids = np.arange(sensor.n_rays)
    else:
        sensor = S.make_lidar((0, 0, 0), 0.0, 8, -15.0, 15.0, 96, tile_az=8, tile_el=4, t_sweep=0.1,
                              ego_vel_world=(10.0, 1.0, 0), n_channels=4, feat_offset=1)
        n = 40
        means = np.stack([rng.uniform(-8, 8, n), rng.uniform(-8, 8, n), rng.uniform(-1, 1, n)], 1)
        ids = np.arange(sensor.n_rays)
    g = S.random_gaussians(rng, means, 6, moving_frac=0.6, log_scale_mean=-0.3)
    R = ids.shape[0]
    up = np.random.default_rng(seed + 100)
    dF = up.normal(size=(R, sensor.n_channels))
    dD = 0.1 * up.normal(size=R)
    dA = up.normal(size=R)
    return g, sensor, ids, dF, dD, dA


@pytest.mark.parametrize("kind", ["camera", "lidar"])
def test_autograd_matches_finite_differences(kind):
    g, sensor, ids, dF, dD, dA = _scene(kind, 11 if kind == "camera" else 12)
    ref, out = gr.reference_grads(g, sensor, ids, dF, dD, dA)
    rng = np.random.default_rng(0)
    coords = []
    for name in geo.Params.names:
        arr = ref[name]
        nz = np.nonzero(np.abs(arr.reshape(-1)) > 0)[0]
        pick = rng.choice(nz, size=min(8, nz.shape[0]), replace=False)
        coords += [(name, int(k)) for k in pick]
    fd, ok = gr.finite_diff(g, sensor, ids, dF, dD, dA, coords)
    assert ok.mean() > 0.8
    checked = 0
    for (name, k), v, good in zip(coords, fd, ok):
        if not good:
            continue
        a = ref[name].reshape(-1)[k]
        assert v == pytest.approx(a, rel=2e-5, abs=1e-7 * max(1.0, np.abs(ref[name]).max())), (name, k)
        checked += 1
    assert checked >= 30


def test_over_operator_closed_form():
    """Build a projection by hand with every Gaussian centred on the ray (alpha_i = o_eff_i)."""
    K = 5
    rng = np.random.default_rng(1)
    a = torch.tensor(rng.uniform(0.05, 0.8, K), dtype=torch.float64, requires_grad=True)
    f = torch.tensor(rng.normal(size=(K, 3)), dtype=torch.float64)
    z = torch.arange(K, dtype=torch.float64) + 1.0
    zeros2 = torch.zeros(K, 2, dtype=torch.float64)
    conic = torch.tensor([[1.0, 0.0, 1.0]] * K, dtype=torch.float64)
    big = torch.full((K, 2), 10.0, dtype=torch.float64)
    proj = geo.Projection(zeros2, zeros2, torch.zeros(K, dtype=torch.float64), None, conic, a, z, z,
                          big, -big, big, torch.ones(K, dtype=torch.bool), "camera",
                          torch.zeros(K, dtype=torch.bool))
    rays = rd.Rays(torch.zeros(1, 2, dtype=torch.float64), torch.zeros(1, dtype=torch.float64),
                   np.zeros(1, np.int64), np.ones(1, bool))

    class _S:
        feat_offset, n_channels = 0, 3
    out = rd.render(proj, _S(), f, rays)
    w = torch.tensor([0.3, -1.2, 0.7], dtype=torch.float64)
    L = (out["F"][0] * w).sum()
    (g,) = torch.autograd.grad(L, [a], retain_graph=True)
    av = a.detach().numpy()
    fv = f.numpy() @ w.numpy()
    T = np.concatenate([[1.0], np.cumprod(1 - av)[:-1]])
    want = np.array([T[i] * fv[i] - sum(fv[j] * av[j] * T[j] for j in range(i + 1, K)) / (1 - av[i])
                     for i in range(K)])
    np.testing.assert_allclose(g.numpy(), want, rtol=1e-12, atol=1e-14)
    # and the opacity output: dA/dalpha_i = T_final / (1 - alpha_i)
    (gA,) = torch.autograd.grad(out["A"][0], [a])
    Tf = np.prod(1 - av)
    np.testing.assert_allclose(gA.numpy(), Tf / (1 - av), rtol=1e-12)
