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
"""
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
