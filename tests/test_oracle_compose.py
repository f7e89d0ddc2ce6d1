"""Pins of the scene-graph composition oracle (oracle/compose.py) against what the paper and the
mathematics fix: identity poses, scipy rotations, a spinning rigid body, rigid distances, the
time derivative of explicitly moved poses, and central finite differences of the gradients."""
import numpy as np
import torch
from scipy.spatial.transform import Rotation

from oracle import compose as oc

D = torch.float64


def _t(x):
    return torch.as_tensor(np.asarray(x, dtype=np.float64))


def _scipy_quat(q):
    """(w, x, y, z) -> scipy Rotation (which takes x, y, z, w)."""
    q = np.asarray(q, dtype=np.float64)
    return Rotation.from_quat(np.concatenate([q[..., 1:], q[..., :1]], -1))


def _scene(rng, n=12, actors=3):
    means = rng.normal(size=(n, 3)) * 2.0
    quats = rng.normal(size=(n, 4))
    aid = rng.integers(-1, actors, size=n)
    aid[0], aid[1] = -1, 0
    rot = rng.normal(size=(actors, 4))
    trans = rng.normal(size=(actors, 3)) * 5.0
    rot_off = np.array([1.0, 0.0, 0.0, 0.0]) + 0.2 * rng.normal(size=(actors, 4))
    trans_off = 0.3 * rng.normal(size=(actors, 3))
    lin = rng.normal(size=(actors, 3)) * 3.0
    lin_off = 0.2 * rng.normal(size=(actors, 3))
    ang = rng.normal(size=(actors, 3)) * 0.5
    vel = rng.normal(size=(n, 3))
    return means, quats, aid, rot, trans, rot_off, trans_off, lin, lin_off, ang, vel


def _call(s, **over):
    means, quats, aid, rot, trans, rot_off, trans_off, lin, lin_off, ang, vel = s
    kw = dict(rot_offset=_t(rot_off), trans_offset=_t(trans_off), lin_vel=_t(lin), lin_vel_offset=_t(lin_off),
              ang_vel=_t(ang), velocities=_t(vel))
    kw.update(over)
    return oc.compose(_t(means), _t(quats), aid, _t(rot), _t(trans), **kw)


def test_identity_pose_passes_gaussians_through():
    rng = np.random.default_rng(1)
    s = _scene(rng)
    means, quats, aid = s[0], s[1], s[2]
    A = s[3].shape[0]
    ident = np.tile([1.0, 0.0, 0.0, 0.0], (A, 1))
    mu, q, v = oc.compose(_t(means), _t(quats), aid, _t(ident), torch.zeros(A, 3, dtype=D))
    np.testing.assert_allclose(mu.numpy(), means, atol=1e-14)
    np.testing.assert_allclose(q.numpy(), quats, atol=1e-14)
    np.testing.assert_allclose(v.numpy(), 0.0, atol=1e-14)


def test_static_gaussians_keep_values_and_velocity():
    rng = np.random.default_rng(2)
    s = _scene(rng)
    mu, q, v = _call(s)
    st = s[2] < 0
    np.testing.assert_array_equal(mu.numpy()[st], s[0][st])
    np.testing.assert_array_equal(q.numpy()[st], s[1][st])
    np.testing.assert_array_equal(v.numpy()[st], s[10][st])


def test_pose_against_scipy_rotations():
    """mu_w = R_b R_off mu + t_b + dt and R(q_w) = R_b R_off R(q), rotations composed by scipy
    (non-commuting rotations: a reversed product fails)."""
    rng = np.random.default_rng(3)
    s = _scene(rng)
    means, quats, aid, rot, trans, rot_off, trans_off = s[:7]
    mu, q, _ = _call(s)
    for i in np.nonzero(aid >= 0)[0]:
        a = aid[i]
        Ra = _scipy_quat(rot[a]) * _scipy_quat(rot_off[a])
        np.testing.assert_allclose(mu.numpy()[i], Ra.apply(means[i]) + trans[a] + trans_off[a], rtol=1e-12, atol=1e-12)
        Rw = (Ra * _scipy_quat(quats[i])).as_matrix()
        np.testing.assert_allclose(_scipy_quat(q.numpy()[i]).as_matrix(), Rw, atol=1e-12)


def test_spinning_actor_point_velocity():
    """A point at radius r on an actor spinning about its z axis with rate w moves with speed
    |w| r, tangentially (counter-clockwise for w > 0)."""
    r, w = 2.5, 0.7
    means = np.array([[r, 0.0, 0.0], [0.0, r, 1.0]])
    mu, q, v = oc.compose(_t(means), _t([[1.0, 0, 0, 0]] * 2), np.array([0, 0]), _t([[1.0, 0, 0, 0]]),
                          _t([[0.0, 0, 0]]), ang_vel=_t([[0.0, 0.0, w]]))
    np.testing.assert_allclose(v.numpy(), [[0.0, w * r, 0.0], [-w * r, 0.0, 0.0]], atol=1e-14)


def test_rigid_distances_preserved():
    rng = np.random.default_rng(4)
    s = _scene(rng, n=40, actors=2)
    mu, _, _ = _call(s)
    for a in range(2):
        idx = np.nonzero(s[2] == a)[0]
        if len(idx) < 2:
            continue
        d0 = np.linalg.norm(s[0][idx][:, None] - s[0][idx][None], axis=-1)
        d1 = np.linalg.norm(mu.numpy()[idx][:, None] - mu.numpy()[idx][None], axis=-1)
        np.testing.assert_allclose(d1, d0, rtol=1e-12, atol=1e-12)


def test_velocity_is_time_derivative_of_moved_pose():
    """Move each actor explicitly for a time dt: rotation R_a exp(dt [w]x) (w in the actor
    frame, scipy's rotation vector) and translation t_a + dt R_a v_a; the central difference of
    the composed means over +-dt equals the composed velocity."""
    rng = np.random.default_rng(5)
    s = _scene(rng, n=20, actors=3)
    means, quats, aid, rot, trans, rot_off, trans_off, lin, lin_off, ang, vel = s
    _, _, v = _call(s)
    h = 1e-5
    for i in np.nonzero(aid >= 0)[0]:
        a = aid[i]
        Ra = _scipy_quat(rot[a]) * _scipy_quat(rot_off[a])
        ta = trans[a] + trans_off[a]
        va = lin[a] + lin_off[a]

        def at(tau):
            R = Ra * Rotation.from_rotvec(tau * ang[a])
            return R.apply(means[i]) + ta + tau * Ra.apply(va)

        fd = (at(h) - at(-h)) / (2 * h)
        np.testing.assert_allclose(v.numpy()[i], fd, rtol=1e-7, atol=1e-7)


def test_gradients_against_central_differences():
    rng = np.random.default_rng(6)
    s = _scene(rng, n=8, actors=2)
    means, quats, aid, rot, trans, rot_off, trans_off, lin, lin_off, ang, vel = s
    w_mu, w_q, w_v = (rng.normal(size=(8, 3)), rng.normal(size=(8, 4)), rng.normal(size=(8, 3)))

    def loss(arrs):
        mu, q, v = oc.compose(arrs["means"], arrs["quats"], aid, _t(rot), _t(trans), rot_offset=arrs["rot_off"],
                              trans_offset=arrs["trans_off"], lin_vel=_t(lin), lin_vel_offset=arrs["lin_off"],
                              ang_vel=arrs["ang"], velocities=_t(vel))
        return (mu * _t(w_mu)).sum() + (q * _t(w_q)).sum() + (v * _t(w_v)).sum()

    base = {"means": means, "quats": quats, "rot_off": rot_off, "trans_off": trans_off, "lin_off": lin_off,
            "ang": ang}
    arrs = {k: _t(v).clone().requires_grad_(True) for k, v in base.items()}
    loss(arrs).backward()
    h = 1e-6
    for k, x in base.items():
        g = arrs[k].grad.numpy()
        fd = np.zeros_like(x)
        for idx in np.ndindex(x.shape):
            xp, xm = x.copy(), x.copy()
            xp[idx] += h
            xm[idx] -= h
            fp = loss({**{kk: _t(vv) for kk, vv in base.items()}, k: _t(xp)}).item()
            fm = loss({**{kk: _t(vv) for kk, vv in base.items()}, k: _t(xm)}).item()
            fd[idx] = (fp - fm) / (2 * h)
        np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-7, err_msg=k)
