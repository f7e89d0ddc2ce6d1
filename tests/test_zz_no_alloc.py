"""The composition adjoint's entry point that allocates nothing (splat_compose_bwd_noalloc)
against the workspace entry point (splat_compose_bwd), through the C ABI: two calls in a row on
one GPU, the second with fewer Gaussians and fewer actors, so that accumulators left over from
the first call would show in the second.  Per-Gaussian gradients carry no atomics and must be
bit-equal; per-actor sums are float atomics, so they agree to the adjoint's run-to-run bar
(1e-4 relative per element, 1e-5 of the largest).  Also: an actor count above the array's
maximum is refused before anything is launched."""
import numpy as np
import pytest
import torch

from scenes import synthetic as S
from tests.gpu_helpers import grad_mismatch

pytestmark = pytest.mark.gpu


def _binding():
    from paper_2411_16816_amd import binding
    binding.load()
    return binding


def _inputs(b, sc, seed):
    f = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    g = sc.gaussians
    A = b.ActorTensors(f(sc.rot), f(sc.trans), f(sc.rot_offset), f(sc.trans_offset), f(sc.lin_vel),
                       f(sc.lin_vel_offset), f(sc.ang_vel))
    n = g.n
    r = np.random.default_rng(seed)
    ups = [f(r.normal(size=(n, 3))), f(r.normal(size=(n, 4))), f(r.normal(size=(n, 3)))]
    return f(g.means), f(g.quats), torch.from_numpy(sc.actor_id).cuda(), A, ups


def _grads(b, mu, q, A):
    d = (torch.zeros_like(mu), torch.zeros_like(q), torch.zeros_like(mu))
    da = {k: torch.zeros_like(getattr(A, k)) for k in b.ACTOR_GRAD_FIELDS if getattr(A, k) is not None}
    return d, da


def test_compose_bwd_noalloc_matches_workspace_entry_point():
    b = _binding()
    for call, (seed, n, n_actors) in enumerate(((71, 200_003, 300), (72, 50_001, 37))):
        print(f"[no_alloc] call {call}: n={n} actors={n_actors}", flush=True)
        sc = S.actor_scene(seed, n, n_actors, contiguous=False)
        mu, q, aid, A, (gm, gq, gv) = _inputs(b, sc, seed + 100)
        (dm0, dq0, dv0), da0 = _grads(b, mu, q, A)
        (dm1, dq1, dv1), da1 = _grads(b, mu, q, A)
        b.compose_bwd(mu, q, aid, A, gm, gq, gv, dm0, dq0, dv0, da0)
        b.compose_bwd_noalloc(mu, q, aid, A, gm, gq, gv, dm1, dq1, dv1, da1)
        torch.cuda.synchronize()
        for name, x, y in (("means", dm1, dm0), ("quats", dq1, dq0), ("velocities", dv1, dv0)):
            assert torch.equal(x, y), name
        for k in da0:
            ref = da0[k].cpu().numpy()
            got = da1[k].cpu().numpy()
            assert np.abs(ref).max() > 0, k
            bad = grad_mismatch(got, ref, rtol=1e-4, afloor=1e-5)
            assert not bad.any(), (call, k, int(bad.sum()))


def test_compose_bwd_noalloc_refuses_too_many_actors():
    b = _binding()
    n_actors = b.COMPOSE_NOALLOC_MAX_ACTORS + 1
    sc = S.actor_scene(73, 1000, n_actors)
    mu, q, aid, A, (gm, gq, gv) = _inputs(b, sc, 173)
    (dm, dq, dv), da = _grads(b, mu, q, A)
    with pytest.raises(b.SplatError, match="capacity|CAPACITY"):
        b.compose_bwd_noalloc(mu, q, aid, A, gm, gq, gv, dm, dq, dv, da)
    torch.cuda.synchronize()
    assert not dm.any() and not dq.any() and not dv.any()
    assert all(not x.any() for x in da.values())
