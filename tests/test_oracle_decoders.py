"""Pins of the oracle's lidar decoder (oracle/decoders.py; Sec. 3.3 and the training-details
appendix): a hand-worked network, axis directions, and gradients against central
differences."""
import math

import numpy as np
import torch

from oracle import decoders as dec


def test_hand_worked_network():
    # C = 1; hidden units: relu(F), relu(-F), relu(d_y); intensity from unit 0, drop from unit 2
    w1 = np.zeros((32, 4))
    w1[0, 0], w1[1, 0], w1[2, 2] = 1.0, -1.0, 1.0
    b1 = np.zeros(32)
    w2 = np.zeros((2, 32))
    w2[0, 0], w2[0, 1], w2[1, 2] = 1.0, 5.0, 2.0
    b2 = np.array([0.0, math.log(3.0)])
    F = np.array([[2.0], [-1.0]])
    az = np.array([0.0, math.pi / 2])
    el = np.array([0.0, 0.0])
    I, P = dec.lidar_mlp(F, az, el, w1, b1, w2, b2)
    # ray 0: h = (2, 0, 0) -> z = (2, ln 3); ray 1: h = (0, 1, 1) -> z = (5, 2 + ln 3)
    s = lambda v: 1.0 / (1.0 + math.exp(-v))
    np.testing.assert_allclose(I.numpy(), [s(2.0), s(5.0)], rtol=1e-14)
    np.testing.assert_allclose(P.numpy(), [0.75, s(2.0 + math.log(3.0))], rtol=1e-14)


def test_axis_directions():
    d = dec.ray_direction([0.0, math.pi / 2, math.pi, 0.3], [0.0, 0.0, 0.0, math.pi / 2]).numpy()
    np.testing.assert_allclose(d, [[1, 0, 0], [0, 1, 0], [-1, 0, 0], [0, 0, 1]], atol=1e-15)


def test_gradients_against_central_differences():
    rng = np.random.default_rng(1)
    R, C = 20, 8
    vals = [rng.normal(size=(R, C)), rng.normal(0, 0.4, (32, C + 3)), rng.normal(0, 0.1, 32),
            rng.normal(0, 0.4, (2, 32)), rng.normal(0, 0.1, 2)]
    az, el = rng.uniform(0, 2 * np.pi, R), rng.uniform(-0.4, 0.3, R)
    up = rng.normal(size=(2, R))
    leaves = [torch.tensor(v, dtype=torch.float64, requires_grad=True) for v in vals]

    def loss(ls):
        I, P = dec.lidar_mlp(ls[0], az, el, *ls[1:])
        return (I * torch.from_numpy(up[0])).sum() + (P * torch.from_numpy(up[1])).sum()

    loss(leaves).backward()
    h = 1e-6
    for k, leaf in enumerate(leaves):
        flat = leaf.grad.view(-1)
        for j in rng.choice(flat.numel(), min(8, flat.numel()), replace=False):
            fs = []
            for sgn in (1.0, -1.0):
                ls = [x.detach().clone() for x in leaves]
                ls[k].view(-1)[j] += sgn * h
                fs.append(float(loss(ls)))
            np.testing.assert_allclose(float(flat[j]), (fs[0] - fs[1]) / (2 * h), rtol=1e-5, atol=1e-9,
                                       err_msg=f"leaf {k} [{j}]")
