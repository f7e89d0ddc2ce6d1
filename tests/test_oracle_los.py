"""Pins of the oracle's line-of-sight sum (oracle/render.py; the loss term L_los of the
training-details appendix: the alphas of the Gaussians a lidar ray blends in front of its
measured range minus a margin): against the ray's own opacity for one Gaussian, the margin's
strict threshold, additivity against each Gaussian rendered alone, and gradients against central
differences."""
import dataclasses

import numpy as np
import torch

from oracle import geometry as geo
from oracle import render as rd
from scenes import synthetic as S


def _lidar(**kw):
    return S.make_lidar((0, 0, 0), 0.0, 16, -15.0, 15.0, 256, tile_az=16, tile_el=4, rolling_shutter=False,
                        n_channels=3, **kw)


def _g(means, log_scale=-1.0, opac=0.6):
    means = np.asarray(means, np.float32).reshape(-1, 3)
    n = means.shape[0]
    return S.Gaussians(means, np.full((n, 3), log_scale, np.float32), np.tile(np.float32([1, 0, 0, 0]), (n, 1)),
                       np.full(n, opac, np.float32), None, np.ones((n, 3), np.float32))


def _ray_towards(lid, x, y, z):
    """Index of the ray closest to the direction of (x, y, z)."""
    az = np.arctan2(y, x) % (2 * np.pi)
    el = np.arcsin(z / np.sqrt(x * x + y * y + z * z))
    d = np.abs(((lid.ray_az - az + np.pi) % (2 * np.pi)) - np.pi) + np.abs(lid.ray_el - el)
    return int(np.argmin(d))


def _with_range(lid, r):
    return dataclasses.replace(lid, ray_range=np.full(lid.n_rays, r, np.float32), los_eps=0.8)


def test_one_gaussian_in_front_contributes_its_alpha():
    lid = _lidar()
    g = _g([[10.0, 0.5, 0.2]])
    k = _ray_towards(lid, 10.0, 0.5, 0.2)
    r = float(np.linalg.norm([10.0, 0.5, 0.2]))
    out = rd.render_sensor(g, _with_range(lid, r + 0.8 + 0.5), [k])
    assert float(out["A"][0]) > 0.1
    np.testing.assert_allclose(out["los"].numpy(), out["A"].numpy(), rtol=1e-12)   # one blend: A = alpha
    behind = rd.render_sensor(g, _with_range(lid, r + 0.8 - 0.5), [k])
    assert float(behind["los"][0]) == 0.0
    none = rd.render_sensor(g, lid, [k])   # no measured range: no line-of-sight sum
    assert float(none["los"][0]) == 0.0


def test_margin_is_a_strict_threshold():
    lid = _lidar()
    g = _g([[10.0, 0.0, 0.0]])
    k = _ray_towards(lid, 10.0, 0.0, 0.0)
    # r_p = 10.75 and eps = 0.75 are exact in float32: corrected range == r_p - eps exactly
    on = rd.render_sensor(g, dataclasses.replace(_with_range(lid, 10.75), los_eps=0.75), [k])
    assert float(on["los"][0]) == 0.0
    just = rd.render_sensor(g, dataclasses.replace(_with_range(lid, 10.7501), los_eps=0.75), [k])
    assert float(just["los"][0]) > 0.0


def test_sum_over_gaussians_equals_each_alone():
    """Two Gaussians on one ray, both blended and in front: the sum is the sum of the opacities
    each produces alone (unlike A, which composites them)."""
    lid = _lidar()
    a, b = [8.0, 0.3, 0.1], [12.0, 0.35, 0.1]
    k = _ray_towards(lid, 8.0, 0.3, 0.1)
    both = rd.render_sensor(_g([a, b], log_scale=-0.3, opac=0.5), _with_range(lid, 30.0), [k])
    alone = [rd.render_sensor(_g([m], log_scale=-0.3, opac=0.5), _with_range(lid, 30.0), [k])["A"] for m in (a, b)]
    assert float(alone[0][0]) > 0.05 and float(alone[1][0]) > 0.01
    np.testing.assert_allclose(both["los"].numpy(), (alone[0] + alone[1]).numpy(), rtol=1e-12)
    assert float(both["los"][0]) > float(both["A"][0])


def test_gradients_against_central_differences():
    rng = np.random.default_rng(8)
    n = 60
    means = np.stack([rng.uniform(-12, 12, n), rng.uniform(-12, 12, n), rng.uniform(-1.5, 1.5, n)], 1)
    g = S.random_gaussians(rng, means, 3, moving_frac=0.3, log_scale_mean=-0.7)
    lid = dataclasses.replace(_lidar(), ray_range=rng.uniform(3.0, 15.0, 256 * 16).astype(np.float32))
    idx = np.arange(0, lid.n_rays, 3)
    p = geo.Params.from_gaussians(g, requires_grad=True)
    w = torch.from_numpy(rng.normal(size=len(idx)))
    out = rd.render_sensor(p, lid, idx)
    assert float(out["los"].abs().sum()) > 0
    (out["los"] * w).sum().backward()
    h = 1e-6
    for name in ("means", "opacities", "log_scales"):
        ten = getattr(p, name)
        flat = ten.grad.view(-1)
        for j in rng.choice(flat.numel(), 6, replace=False):
            vals = []
            for sgn in (1.0, -1.0):
                q = geo.Params.from_gaussians(g)
                getattr(q, name).view(-1)[j] += sgn * h
                with torch.no_grad():
                    vals.append(float((rd.render_sensor(q, lid, idx)["los"] * w).sum()))
            fd = (vals[0] - vals[1]) / (2 * h)
            np.testing.assert_allclose(float(flat[j]), fd, rtol=1e-4, atol=1e-7, err_msg=f"{name}[{j}]")
