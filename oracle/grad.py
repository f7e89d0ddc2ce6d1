"""Oracle, steps 11-12: reference gradients.

Plain FP64 torch (CPU).  Test infrastructure only.

  * reference_grads -- autograd through the FP64 projection + compositing of geometry/render;
    every discrete decision (culling, box candidacy, the 1/255 skip, the T < 1e-4 stop, the
    0.99 clamp, the Jacobian clamp) enters only through masks or clamps, so the gradient is
    that of the piecewise-smooth function with those decisions held fixed.
  * finite_diff -- central differences of the same FP64 forward, h = h_rel * max(1, |theta|);
    a coordinate is skipped (and reported) when any decision differs between theta +- h.

The training-style scalar is L = sum(dF * F) + sum(dD * D) + sum(dA * A) for given upstream
weights, so dL/dtheta equals the vector-Jacobian product the GPU adjoint computes.
Pins: finite differences against autograd, and the closed-form dO/dalpha_i of the over operator
(tests/test_oracle_grad.py).
"""
from __future__ import annotations

import numpy as np
import torch

from . import geometry as geo
from . import render as rd


def weighted_loss(out, dF, dD, dA, dlos=None):
    """Sum of the outputs weighted by upstream gradients; `dlos` weights the lidar line-of-sight
    sum (the loss term L_los of the training-details appendix)."""
    L = (out["F"] * dF).sum() + (out["D"] * dD).sum() + (out["A"] * dA).sum()
    if dlos is not None:
        L = L + (out["los"] * dlos).sum()
    return L


def reference_grads(g, sensor, ray_idx, dF, dD, dA, mode="box", dlos=None):
    """Returns ({name: grad [N,...] float64 numpy}, forward dict)."""
    p = geo.Params.from_gaussians(g, requires_grad=True)
    out = rd.render_sensor(p, sensor, ray_idx, mode)
    L = weighted_loss(out, geo.t64(dF), geo.t64(dD), geo.t64(dA), None if dlos is None else geo.t64(dlos))
    grads = torch.autograd.grad(L, p.tensors(), allow_unused=True)
    res = {}
    for name, gr, ten in zip(geo.Params.names, grads, p.tensors()):
        res[name] = np.zeros(tuple(ten.shape)) if gr is None else gr.detach().numpy()
    return res, out


def reference_sensor_grads(g, sensor, ray_idx, dF, dD, dA, mode="box"):
    """Gradients of the weighted loss with respect to the sensor's linear and angular velocity
    (sensor frame) and, for a camera, its time offset: {name: float64 numpy}, by FP64 autograd
    with the sensor parameters as leaves (candidacy decisions do not depend on them
    differentiably)."""
    import dataclasses
    leaves = {"lin_vel": geo.t64(sensor.lin_vel).clone().requires_grad_(True),
              "ang_vel": geo.t64(sensor.ang_vel).clone().requires_grad_(True)}
    if not hasattr(sensor, "ray_az"):
        leaves["time_offset"] = geo.t64(getattr(sensor, "time_offset", 0.0)).clone().requires_grad_(True)
    s2 = dataclasses.replace(sensor, **leaves)
    p = geo.Params.from_gaussians(g)
    out = rd.render_sensor(p, s2, ray_idx, mode)
    L = weighted_loss(out, geo.t64(dF), geo.t64(dD), geo.t64(dA))
    grads = torch.autograd.grad(L, list(leaves.values()), allow_unused=True)
    return {k: (np.zeros(tuple(v.shape)) if gr is None else gr.detach().numpy())
            for (k, v), gr in zip(leaves.items(), grads)}, out


def sensor_finite_diff(g, sensor, ray_idx, dF, dD, dA, name, index=None, h=1e-6, mode="box"):
    """Central difference of the weighted loss in one sensor parameter (FP64 forward)."""
    import dataclasses
    base = np.asarray(getattr(sensor, name), dtype=np.float64)
    dF, dD, dA = geo.t64(dF), geo.t64(dD), geo.t64(dA)
    p = geo.Params.from_gaussians(g)
    vals = []
    for sgn in (1.0, -1.0):
        x = base.copy()
        if index is None:
            x = x + sgn * h
        else:
            x[index] += sgn * h
        s2 = dataclasses.replace(sensor, **{name: x if x.ndim else float(x)})
        with torch.no_grad():
            out = rd.render_sensor(p, s2, ray_idx, mode)
            vals.append(float(weighted_loss(out, dF, dD, dA)))
    return (vals[0] - vals[1]) / (2 * h)


def _forward_value(p, sensor, ray_idx, dF, dD, dA, mode):
    with torch.no_grad():
        out = rd.render_sensor(p, sensor, ray_idx, mode)
        L = weighted_loss(out, dF, dD, dA)
    return float(L), out["proj"].valid.clone(), out["sig"].clone()


def finite_diff(g, sensor, ray_idx, dF, dD, dA, coords, mode="box", h_rel=1e-6):
    """coords: list of (param_name, flat_index).  Returns (values [n], ok mask [n])."""
    base = geo.Params.from_gaussians(g)
    dF, dD, dA = geo.t64(dF), geo.t64(dD), geo.t64(dA)
    _, valid0, sig0 = _forward_value(base, sensor, ray_idx, dF, dD, dA, mode)
    vals = np.zeros(len(coords))
    ok = np.ones(len(coords), bool)
    for k, (name, flat) in enumerate(coords):
        ten = getattr(base, name)
        theta = float(ten.view(-1)[flat])
        h = h_rel * max(1.0, abs(theta))
        res = []
        for sgn in (+1.0, -1.0):
            pp = geo.Params(*[t.clone() for t in base.tensors()])
            getattr(pp, name).view(-1)[flat] = theta + sgn * h
            L, valid, sig = _forward_value(pp, sensor, ray_idx, dF, dD, dA, mode)
            if not torch.equal(valid, valid0) or not torch.equal(sig, sig0):
                ok[k] = False
            res.append(L)
        vals[k] = (res[0] - res[1]) / (2.0 * h)
    return vals, ok
