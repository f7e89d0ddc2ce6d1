"""Oracle, scene-graph composition at a capture time (Sec. 3.1 "Scene representation"; Sec. 3.2
"Rolling shutter", the actor velocity term of Eq. (pixel_velocity); App. D "Rolling shutter
details").

Plain FP64 torch (CPU).  Test infrastructure only.

The scene is a static background plus rigid actors.  A Gaussian with actor id a >= 0 has its
mean and rotation expressed in the frame of its actor's box; at the capture time the actor has
a pose (rotation R_a, translation t_a: actor frame -> world) and a rigid motion (linear velocity
v_a and angular velocity w_a, both in the actor frame).  Composition gives the world mean,
world rotation and world velocity that the projection consumes:

    mu_w = R_a mu + t_a
    q_w  = q_a (x) q                 (rotation composition: R(q_w) = R_a R(q))
    v_w  = R_a (w_a x mu + v_a)      (the velocity of a point of a rigid body, App. D, rotated
                                      from the actor frame to the world frame)

Gaussians of the static background (id < 0) keep their mean and rotation, and their world
velocity is the per-Gaussian input velocity (zero when none is given).

Pose and velocity estimates carry learnable offsets (Sec. 3.1).  Readings (not fixed by the
paper; listed in the design notes):
  * the effective rotation is q_a = q_b (x) dq / |dq| with the base rotation q_b normalised:
    the rotation offset acts in the actor's own frame;
  * the effective translation is t_a = t_b + dt (world frame);
  * the effective linear velocity is v_a = v_b + dv (actor frame); the angular velocity w_a is
    used as given (and differentiated).

Pins (tests/test_oracle_compose.py): identity poses pass Gaussians through; rotations and
their products against scipy's Rotation; a point on a spinning actor moves with speed |w| r
tangentially; rigid-body distances are preserved; the velocity equals the time derivative of
the composed mean under the actor's rigid motion (central differences of explicitly moved
poses, independent of the velocity formula); gradients against central finite differences.
"""
from __future__ import annotations

import torch

from .geometry import quat_to_rotmat

D = torch.float64


def quat_mul(a: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    """Hamilton product a (x) b of quaternions (w, x, y, z): R(a (x) b) = R(a) R(b)."""
    aw, ax, ay, az = a.unbind(-1)
    bw, bx, by, bz = b.unbind(-1)
    return torch.stack([aw * bw - ax * bx - ay * by - az * bz,
                        aw * bx + ax * bw + ay * bz - az * by,
                        aw * by - ax * bz + ay * bw + az * bx,
                        aw * bz + ax * by - ay * bx + az * bw], -1)


def normalize(q: torch.Tensor) -> torch.Tensor:
    return q / torch.linalg.norm(q, dim=-1, keepdim=True)


def actor_state(rot, trans, rot_offset=None, trans_offset=None, lin_vel=None, lin_vel_offset=None,
                ang_vel=None):
    """Effective pose and motion of every actor: (q_a unit [A,4], R_a [A,3,3], t_a [A,3],
    v_a [A,3], w_a [A,3]) from the base values and the learnable offsets (None = identity /
    zero)."""
    qb = normalize(rot)
    A = qb.shape[0]
    dq = torch.tensor([1.0, 0.0, 0.0, 0.0], dtype=D).expand(A, 4) if rot_offset is None else normalize(rot_offset)
    qa = quat_mul(qb, dq)
    ta = trans if trans_offset is None else trans + trans_offset
    zero = torch.zeros(A, 3, dtype=D)
    va = (zero if lin_vel is None else lin_vel) + (zero if lin_vel_offset is None else lin_vel_offset)
    wa = zero if ang_vel is None else ang_vel
    return qa, quat_to_rotmat(qa), ta, va, wa


def compose(means, quats, actor_id, rot, trans, rot_offset=None, trans_offset=None, lin_vel=None,
            lin_vel_offset=None, ang_vel=None, velocities=None):
    """World means [N,3], rotations [N,4] and velocities [N,3] of the composed scene.

    means, quats: per-Gaussian, in the actor frame for actor Gaussians (world frame for the
    static background); actor_id [N] int (< 0: static); the actor arrays as in actor_state;
    velocities [N,3]: world velocity of static Gaussians (None = zero)."""
    N = means.shape[0]
    qa, Ra, ta, va, wa = actor_state(rot, trans, rot_offset, trans_offset, lin_vel, lin_vel_offset, ang_vel)
    aid = torch.as_tensor(actor_id, dtype=torch.long)
    dyn = aid >= 0
    a = aid.clamp(min=0)
    R = Ra[a]                                              # [N,3,3]
    mu_w = torch.einsum("nij,nj->ni", R, means) + ta[a]
    q_w = quat_mul(qa[a], quats)
    u = torch.linalg.cross(wa[a], means, dim=-1) + va[a]   # rigid-body velocity, actor frame
    v_dyn = torch.einsum("nij,nj->ni", R, u)
    v_static = torch.zeros(N, 3, dtype=D) if velocities is None else velocities
    m = dyn[:, None]
    return (torch.where(m, mu_w, means), torch.where(m, q_w, quats), torch.where(m, v_dyn, v_static))
