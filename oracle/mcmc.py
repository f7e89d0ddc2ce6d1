"""Oracle, MCMC regulariser (training-details appendix: the opacity and scale regularisation of
the MCMC densification strategy the paper adopts).

Plain FP64 torch (CPU).  Test infrastructure only.

    L = lambda_o * sum_i |o_i| + lambda_S * sum_i sum_j |sqrt(eig_j(Sigma_i))|

with the paper's weights lambda_o = 0.005 and lambda_S = 0.001.  Sigma_i is the Gaussian's 3D
covariance (Sec. 3.1, built by oracle.geometry.covariance); its eigenvalues are taken with a
library symmetric eigensolver, and the gradients follow by autograd through that solver.  The
opacities are the values the rasteriser blends (in (0, 1)).

Pins (tests/test_oracle_mcmc.py): the eigenvalues of R diag(s^2) R^T are s^2 for any rotation
(so the scale term equals the sum of the scales), invariance under rotation of the Gaussian,
hand values, and gradients against central differences.

Relocation of dead Gaussians (the MCMC densification strategy the paper adopts unchanged, with
at most 5M Gaussians): a Gaussian whose opacity is at most 0.005 is dead; each dead Gaussian
takes the place of an alive one drawn with probability proportional to opacity, and a target
shared by N Gaussians (itself and its N - 1 copies) gets

    o' = 1 - (1 - o)^(1/N),   s' = s * o / sum_{k=1..N} C(N, k) (-1)^(k+1) o'^k / sqrt(k)

(every scale axis alike; N capped at 51).  The scale rule keeps the integral of the composited
profile of the N copies, 1 - (1 - o' g')^N along an axis, equal to that of the original o g.
Readings (listed in the design notes): the draw is an input, one 32-bit integer u per Gaussian;
the weights are the opacities in fixed point, floor(o * 2^24), so that the draw is exact integer
arithmetic (r = floor(u * total / 2^32), the target is the first Gaussian whose inclusive weight
sum exceeds r; a Gaussian is alive when o > 0.005 and its weight is at most 2^24); the copies take the target's mean, rotation, velocity and features and the new
opacity and scales; o' is not clamped; with no alive Gaussian nothing moves.

Relocation pins: a hand-worked draw, the opacity identity 1 - (1 - o')^N = o, the profile
integral by numerical quadrature, N = 1 leaving a Gaussian unchanged, and the copies.
"""
import copy
import math

import numpy as np
import torch

from . import geometry as geo

LAMBDA_O = 0.005
LAMBDA_S = 0.001


def regulariser(opacities, log_scales, quats, lambda_o=LAMBDA_O, lambda_s=LAMBDA_S):
    """Scalar L of the appendix's MCMC regularisation (torch float64, differentiable)."""
    o = geo.t64(opacities)
    Sig = geo.covariance(geo.t64(log_scales), geo.t64(quats))
    Sig = 0.5 * (Sig + Sig.transpose(-1, -2))   # exactly symmetric for the solver
    ev = torch.linalg.eigvalsh(Sig)
    return lambda_o * o.abs().sum() + lambda_s * torch.sqrt(ev.clamp_min(0.0)).abs().sum()


DEAD_OPACITY = 0.005
N_MAX = 51
WEIGHT_ONE = 1 << 24      # opacities as fixed-point sampling weights


def relocated_opacity_scale(o, n):
    """(o', scale factor) of a Gaussian of opacity o shared by n copies (FP64)."""
    o = float(o)
    on = 1.0 - (1.0 - o) ** (1.0 / n)
    denom = 0.0
    for k in range(1, n + 1):
        denom += math.comb(n, k) * (-1.0) ** (k + 1) * on ** k / math.sqrt(k)
    return on, o / denom


def draw_targets(opacities, u, dead_opacity=DEAD_OPACITY):
    """Target index of every dead Gaussian (-1 for alive ones, and for all when none is alive)."""
    o = np.asarray(opacities, np.float32)
    dead = ~(o > np.float32(dead_opacity))
    w = np.where(dead, 0, np.minimum(np.floor(o.astype(np.float64) * WEIGHT_ONE), WEIGHT_ONE)).astype(np.int64)
    incl = np.cumsum(w)
    total = int(incl[-1]) if len(incl) else 0
    tgt = np.full(len(o), -1, np.int64)
    if total == 0:
        return tgt
    for i in np.nonzero(dead)[0]:
        r = (int(u[i]) * total) >> 32
        tgt[i] = int(np.searchsorted(incl, r, side="right"))
    return tgt


def relocate(g, u, dead_opacity=DEAD_OPACITY, n_max=N_MAX):
    """Relocated copy of a scenes.Gaussians-like object (opacities and log-scales as float64)
    and the targets."""
    tgt = draw_targets(g.opacities, u, dead_opacity)
    out = copy.deepcopy(g)
    counts = np.bincount(tgt[tgt >= 0], minlength=len(tgt))
    o64 = np.asarray(g.opacities, np.float64)
    ls64 = np.asarray(g.log_scales, np.float64)
    new_o, new_ls = o64.copy(), ls64.copy()
    for t in np.nonzero(counts)[0]:
        on, f = relocated_opacity_scale(o64[t], min(int(counts[t]) + 1, n_max))
        new_o[t] = on
        new_ls[t] = ls64[t] + math.log(f)
    dead_moved = tgt >= 0
    src = np.where(dead_moved, tgt, np.arange(len(tgt)))
    for name in ("means", "quats", "velocities", "features"):
        arr = getattr(g, name)
        if arr is not None:
            setattr(out, name, np.asarray(arr)[src].copy())
    out.opacities = new_o[src]
    out.log_scales = new_ls[src]
    return out, tgt
