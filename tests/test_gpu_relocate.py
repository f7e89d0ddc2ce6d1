"""MCMC relocation of dead Gaussians (splat_mcmc_relocate) through the C ABI against the oracle
(oracle/mcmc.py): the drawn targets bit-exact (the draw is integer arithmetic on both sides),
copied rows bit-exact, the new opacities and log-scales within 1e-4 relative / 1e-5 absolute;
ragged sizes, the cap on copies, no dead and no alive Gaussians, and the 2M-Gaussian scene."""
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


def _scene(seed, n, dead_frac, n_feat=6):
    rng = np.random.default_rng(seed)
    g = S.random_gaussians(rng, rng.uniform(-50, 50, (n, 3)), n_feat, moving_frac=0.3)
    k = int(dead_frac * n)
    idx = rng.choice(n, k, replace=False)
    g.opacities[idx] = rng.uniform(0.0, 0.005, k).astype(np.float32)
    if k:
        g.opacities[idx[0]] = np.float32(0.005)   # on the threshold: dead
    u = rng.integers(0, 1 << 32, n, dtype=np.uint64)
    return g, u


def _run(b, g, u, n_max=51):
    G = b.GaussTensors.from_numpy(g)
    ud = torch.from_numpy(u.astype(np.uint32).view(np.int32)).cuda()
    tgt, moved = b.mcmc_relocate(G, ud, n_max=n_max)
    torch.cuda.synchronize()
    return G, tgt.cpu().numpy(), int(moved)


def _check(G, tgt, g, u, n_max=51):
    ref, rt = mcmc.relocate(g, u, n_max=n_max)
    np.testing.assert_array_equal(tgt, rt)
    for name in ("means", "quats", "velocities", "features"):
        np.testing.assert_array_equal(getattr(G, name).cpu().numpy(), getattr(ref, name), err_msg=name)
    for name in ("opacities", "log_scales"):
        a = getattr(G, name).cpu().numpy().astype(np.float64)
        r = np.asarray(getattr(ref, name), np.float64)
        err = np.abs(a - r) / (1e-5 + 1e-4 * np.abs(r))
        assert err.max() <= 1.0, (name, float(err.max()))


@pytest.mark.parametrize("n,dead", [(100003, 0.2), (4097, 0.6), (1, 0.0), (300, 0.9)])
def test_relocate_matches_oracle(n, dead):
    b = _binding()
    g, u = _scene(n, n, dead)
    print(f"[relocate] n={n} dead={dead}", flush=True)
    G, tgt, moved = _run(b, g, u)
    assert moved == int((tgt >= 0).sum()) == int((g.opacities <= np.float32(0.005)).sum())
    _check(G, tgt, g, u)


def test_relocate_cap_and_degenerate_cases():
    b = _binding()
    # 95 % dead: many copies per target, capped at N = 3
    g, u = _scene(7, 2000, 0.95)
    G, tgt, _ = _run(b, g, u, n_max=3)
    _check(G, tgt, g, u, n_max=3)
    # none alive: nothing moves
    g, u = _scene(8, 500, 0.0)
    g.opacities[:] = np.float32(0.001)
    G, tgt, moved = _run(b, g, u)
    assert moved == 0 and (tgt == -1).all()
    np.testing.assert_array_equal(G.opacities.cpu().numpy(), g.opacities)
    # none dead: nothing moves
    g, u = _scene(9, 500, 0.0)
    G, tgt, moved = _run(b, g, u)
    assert moved == 0
    np.testing.assert_array_equal(G.log_scales.cpu().numpy(), g.log_scales)


def test_relocate_few_alive_small_total():
    # total weight below one entry per four Gaussians: every value of r has a lookup-table entry of
    # its own; and a few alive near the threshold scattered through a large dead set
    b = _binding()
    for seed, n, alive in ((11, 500_000, [123_457]), (12, 300_001, [0, 17, 150_000, 300_000])):
        g, u = _scene(seed, n, 1.0)
        g.opacities[alive] = np.float32(0.006)
        print(f"[relocate] few alive n={n} alive={alive}", flush=True)
        G, tgt, moved = _run(b, g, u, n_max=51)
        np.testing.assert_array_equal(tgt, mcmc.draw_targets(g.opacities, u))
        assert moved == n - len(alive)
        assert set(np.unique(tgt[tgt >= 0])) <= set(alive)


def test_relocate_headline_scene():
    b = _binding()
    g = S.headline().gaussians
    rng = np.random.default_rng(10)
    idx = rng.choice(g.n, g.n // 10, replace=False)
    g.opacities[idx] = rng.uniform(0.0, 0.005, len(idx)).astype(np.float32)
    u = rng.integers(0, 1 << 32, g.n, dtype=np.uint64)
    print(f"[relocate] headline n={g.n}", flush=True)
    G, tgt, moved = _run(b, g, u)
    rt = mcmc.draw_targets(g.opacities, u)
    np.testing.assert_array_equal(tgt, rt)
    assert moved == len(idx)
    sample = np.random.default_rng(2).choice(g.n, 4096, replace=False)
    sample = np.union1d(sample, idx[:512])
    ref, _ = mcmc.relocate(g, u)
    for name in ("means", "features"):
        np.testing.assert_array_equal(getattr(G, name).cpu().numpy()[sample], getattr(ref, name)[sample])
    a = G.opacities.cpu().numpy().astype(np.float64)[sample]
    r = ref.opacities[sample]
    assert (np.abs(a - r) / (1e-5 + 1e-4 * np.abs(r))).max() <= 1.0
