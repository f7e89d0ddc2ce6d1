"""MCMC regulariser (splat_mcmc_regularizer; training-details appendix) through the C ABI
against the FP64 oracle (oracle/mcmc.py, eigenvalues of the 3D covariance by a symmetric
eigensolver): the value within 1e-4 relative, the opacity and log-scale gradients within
1e-4 relative / 1e-5 absolute element by element; accumulation into existing buffers, optional
outputs, an empty call, and the 2M-Gaussian headline scene."""
import numpy as np
import pytest
import torch

from oracle import mcmc
from scenes import synthetic as S

pytestmark = pytest.mark.gpu


def _binding():
    from paper_2411_16816_amd import binding
    binding.load()
    return binding


def _oracle(g, idx=None):
    sel = (lambda a: a) if idx is None else (lambda a: a[idx])
    leaves = [torch.tensor(sel(g.opacities), dtype=torch.float64, requires_grad=True),
              torch.tensor(sel(g.log_scales), dtype=torch.float64, requires_grad=True)]
    L = mcmc.regulariser(leaves[0], leaves[1], torch.tensor(sel(g.quats), dtype=torch.float64))
    L.backward()
    return float(L), leaves[0].grad.numpy(), leaves[1].grad.numpy()


def _close(a, r, what):
    err = np.abs(a.astype(np.float64) - r) / (1e-5 + 1e-4 * np.abs(r))
    assert float(err.max(initial=0.0)) <= 1.0, (what, float(err.max()))


def test_mcmc_regulariser_matches_oracle():
    b = _binding()
    rng = np.random.default_rng(3)
    n = 100003
    g = S.random_gaussians(rng, rng.uniform(-50, 50, (n, 3)), 4)
    print(f"[mcmc] n={n}", flush=True)
    G = b.GaussTensors.from_numpy(g)
    val = torch.zeros(1, device="cuda")
    gr = b.zeros_like_grads(G)
    gr.opacities.fill_(1.0)   # gradients accumulate
    b.mcmc_regularizer(G, val, gr)
    b.mcmc_regularizer(G, val)   # value only: the value accumulates too
    torch.cuda.synchronize()
    L, d_o, d_l = _oracle(g)
    assert abs(float(val) - 2 * L) <= 1e-4 * 2 * L
    _close(gr.opacities.cpu().numpy() - 1.0, d_o, "opacities")
    _close(gr.log_scales.cpu().numpy(), d_l, "log_scales")
    assert float(gr.means.abs().max()) == 0.0 and float(gr.quats.abs().max()) == 0.0   # untouched


def test_mcmc_regulariser_edge_cases():
    b = _binding()
    rng = np.random.default_rng(4)
    g = S.random_gaussians(rng, rng.uniform(-5, 5, (0, 3)), 4)
    G = b.GaussTensors.from_numpy(g)
    val = torch.zeros(1, device="cuda")
    b.mcmc_regularizer(G, val, b.zeros_like_grads(G))   # no Gaussians
    torch.cuda.synchronize()
    assert float(val) == 0.0
    g = S.random_gaussians(rng, rng.uniform(-5, 5, (7, 3)), 4)
    g.log_scales[:] = np.log(np.float32(0.25))   # equal scales (a degenerate spectrum)
    G = b.GaussTensors.from_numpy(g)
    gr = b.zeros_like_grads(G)
    b.mcmc_regularizer(G, None, gr)   # gradients only
    torch.cuda.synchronize()
    L, d_o, d_l = _oracle(g)
    _close(gr.opacities.cpu().numpy(), d_o, "opacities")
    _close(gr.log_scales.cpu().numpy(), d_l, "log_scales")
    with pytest.raises(b.SplatError):
        b.mcmc_regularizer(G, val, gr, lambda_o=float("nan"))


def test_mcmc_regulariser_headline_scene():
    b = _binding()
    sc = S.headline()
    g = sc.gaussians
    print(f"[mcmc] headline n={g.n}", flush=True)
    G = b.GaussTensors.from_numpy(g)
    val = torch.zeros(1, device="cuda")
    gr = b.zeros_like_grads(G)
    b.mcmc_regularizer(G, val, gr)
    torch.cuda.synchronize()
    with torch.no_grad():
        L = float(mcmc.regulariser(g.opacities, g.log_scales, g.quats))
    assert abs(float(val) - L) <= 1e-4 * L
    idx = np.sort(np.random.default_rng(5).choice(g.n, 4096, replace=False))
    _, d_o, d_l = _oracle(g, idx)
    _close(gr.opacities.cpu().numpy()[idx], d_o, "opacities")
    _close(gr.log_scales.cpu().numpy()[idx], d_l, "log_scales")
