"""Pins of the oracle's MCMC regulariser (oracle/mcmc.py; training-details appendix): a hand
value, the spectrum of R diag(s^2) R^T, invariance under rotation, and gradients against central
differences."""
import numpy as np
import torch
from scipy.spatial.transform import Rotation

from oracle import mcmc


def _q(rng, n):
    q = Rotation.random(n, random_state=int(rng.integers(1 << 30))).as_quat()   # (x, y, z, w)
    return np.concatenate([q[:, 3:], q[:, :3]], 1)


def test_hand_value():
    L = mcmc.regulariser([0.5], np.log([[1.0, 2.0, 3.0]]), [[1.0, 0, 0, 0]])
    assert abs(float(L) - (0.005 * 0.5 + 0.001 * 6.0)) < 1e-15


def test_scale_term_is_the_sum_of_scales_for_any_rotation():
    rng = np.random.default_rng(1)
    n = 200
    ls = rng.normal(-1.0, 0.8, (n, 3))
    op = rng.uniform(0.01, 0.99, n)
    for q in (np.tile([1.0, 0, 0, 0], (n, 1)), _q(rng, n), 3.0 * _q(rng, n)):   # unnormalised too
        L = float(mcmc.regulariser(op, ls, q))
        want = 0.005 * op.sum() + 0.001 * np.exp(ls).sum()
        assert abs(L - want) <= 1e-12 * want


def test_gradients_against_central_differences():
    rng = np.random.default_rng(2)
    n = 30
    leaves = [torch.tensor(rng.uniform(0.05, 0.95, n), dtype=torch.float64, requires_grad=True),
              torch.tensor(rng.normal(-1.0, 0.5, (n, 3)), dtype=torch.float64, requires_grad=True),
              torch.tensor(_q(rng, n), dtype=torch.float64, requires_grad=True)]
    mcmc.regulariser(*leaves).backward()
    h = 1e-6
    for k, leaf in enumerate(leaves):
        flat = leaf.grad.view(-1)
        for j in rng.choice(flat.numel(), 8, replace=False):
            vals = []
            for sgn in (1.0, -1.0):
                args = [x.detach().clone() for x in leaves]
                args[k].view(-1)[j] += sgn * h
                vals.append(float(mcmc.regulariser(*args)))
            fd = (vals[0] - vals[1]) / (2 * h)
            np.testing.assert_allclose(float(flat[j]), fd, rtol=1e-5, atol=1e-10, err_msg=f"leaf {k} [{j}]")
    # rotations leave the spectrum unchanged: no quaternion gradient
    assert float(leaves[2].grad.abs().max()) < 1e-12
