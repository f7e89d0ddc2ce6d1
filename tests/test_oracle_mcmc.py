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


# ---- relocation ------------------------------------------------------------------------------
import math  # noqa: E402

from scipy import integrate  # noqa: E402

from scenes import synthetic as S  # noqa: E402


def test_hand_worked_draw():
    # weights floor(o * 2^24): 8388608, 0 (dead), 4194304, 0 (dead); inclusive sums 8388608,
    # 8388608, 12582912, 12582912; total 12582912
    o = np.array([0.5, 0.001, 0.25, 0.002], np.float32)
    for u, want in ((1 << 31, 0), (3 << 30, 2), (0, 0), ((1 << 32) - 1, 2), (2863311531, 2)):
        t = mcmc.draw_targets(o, np.array([0, u, 0, u], np.uint64))
        # r = u * total >> 32: 2^31 -> 6291456 (< 8388608: Gaussian 0); 0.75 -> 9437184 (Gaussian 2)
        assert t[0] == -1 and t[2] == -1 and t[1] == want and t[3] == want, (u, t)
    assert (mcmc.draw_targets(np.full(3, 0.004, np.float32), np.zeros(3, np.uint64)) == -1).all()   # none alive


def test_opacity_identity_and_single_copy():
    for o in (0.006, 0.05, 0.3, 0.7, 0.99):
        on, f = mcmc.relocated_opacity_scale(o, 1)
        assert abs(on - o) < 1e-14 and abs(f - 1.0) < 1e-14
        for n in (2, 3, 10, 51):
            on, _ = mcmc.relocated_opacity_scale(o, n)
            assert abs(1.0 - (1.0 - on) ** n - o) < 1e-13


def test_scale_rule_keeps_the_profile_integral():
    """N copies of (o', s') composited at one place integrate to the original's o s sqrt(2 pi)
    along an axis (quadrature, independent of the closed form)."""
    for o in (0.02, 0.3, 0.9):
        for n in (2, 3, 7, 20, 51):
            on, f = mcmc.relocated_opacity_scale(o, n)
            s = 1.7
            val, _ = integrate.quad(lambda x: 1.0 - (1.0 - on * math.exp(-0.5 * (x / (f * s)) ** 2)) ** n,
                                    -60 * s, 60 * s, limit=400, epsabs=1e-13, epsrel=1e-12)
            assert abs(val - o * s * math.sqrt(2 * math.pi)) < 1e-9 * val, (o, n)


def test_relocate_copies_targets():
    rng = np.random.default_rng(6)
    n = 500
    g = S.random_gaussians(rng, rng.uniform(-5, 5, (n, 3)), 6)
    g.opacities[rng.choice(n, 120, replace=False)] = rng.uniform(0.0, 0.005, 120).astype(np.float32)
    u = rng.integers(0, 1 << 32, n, dtype=np.uint64)
    out, tgt = mcmc.relocate(g, u)
    dead = g.opacities <= np.float32(0.005)
    assert (tgt[dead] >= 0).all() and (tgt[~dead] == -1).all() and not dead[tgt[dead]].any()
    counts = np.bincount(tgt[dead], minlength=n)
    for i in np.nonzero(dead)[0]:
        t = tgt[i]
        for name in ("means", "quats", "velocities", "features"):
            np.testing.assert_array_equal(getattr(out, name)[i], getattr(g, name)[t])
        assert out.opacities[i] == out.opacities[t] and (out.log_scales[i] == out.log_scales[t]).all()
        on, f = mcmc.relocated_opacity_scale(g.opacities[t], counts[t] + 1)
        assert abs(out.opacities[t] - on) < 1e-15
        np.testing.assert_allclose(out.log_scales[t], g.log_scales[t].astype(np.float64) + math.log(f), rtol=1e-14)
    untouched = ~dead & (counts == 0)
    np.testing.assert_array_equal(out.opacities[untouched], g.opacities[untouched])
