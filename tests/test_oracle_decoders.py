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


# ---- camera decoder ------------------------------------------------------------------------
from scenes import synthetic as S   # noqa: E402


def _cam(w=6, h=4, yaw=0.0):
    return S.make_camera((0, 0, 0), yaw, w, h, 5.0, n_channels=3)


def test_conv3x3_against_brute_force_loops():
    rng = np.random.default_rng(3)
    H, W, Ci, Co = 5, 7, 3, 2
    x = rng.normal(size=(H, W, Ci))
    w = rng.normal(size=(Co, Ci, 3, 3))
    b = rng.normal(size=Co)
    want = np.zeros((H, W, Co))
    for y in range(H):
        for xx in range(W):
            for o in range(Co):
                s = b[o]
                for i in range(3):
                    for j in range(3):
                        yy, xj = y + i - 1, xx + j - 1
                        if 0 <= yy < H and 0 <= xj < W:
                            s += float(np.dot(w[o, :, i, j], x[yy, xj]))
                want[y, xx, o] = s
    got = dec.conv3x3(torch.from_numpy(x), torch.from_numpy(w), torch.from_numpy(b)).numpy()
    np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-13)


def _centre(co, ci, nci, n_co=32):
    w = np.zeros((n_co, nci, 3, 3))
    for o, i in zip(co, ci):
        w[o, i, 1, 1] = 1.0
    return w


def test_camera_cnn_closed_forms():
    """D_f = 3, E = 1, x = [F_r, F_g, F_b, d_x, d_y, d_z, e].  Stem: channel 0 <- F_r, channel
    1 <- e, channel 2 <- d_x (centre taps).
    With both block convolutions centre-tap identities each block doubles h (r = h, h' = h + h),
    so h_2 = 4 h_0; with zero blocks h_2 = h_0."""
    cam = _cam()
    rng = np.random.default_rng(4)
    F = rng.normal(size=(cam.height, cam.width, 3))
    e = np.array([0.7])
    w_in, b_in = _centre([0, 1, 2], [0, 6, 3], 3 + 3 + 1), np.zeros(32)
    w_out, b_out = np.zeros((6, 32)), np.array([0.0, 0.0, 0.0, 0.5, 0.25, 0.0])
    w_out[0, 0], w_out[2, 1], w_out[4, 2] = 1.0, 1.0, 1.0   # M_r = h_0, M_b = h_1, b_g = 0.25 + h_2
    ident = _centre(range(32), range(32), 32)
    dx = np.maximum(dec.camera_directions(cam)[..., 0].numpy(), 0.0)
    assert dx.min() > 0.5   # the camera looks along the world x axis
    for blocks, gain in (([np.zeros((32, 32, 3, 3))] * 4, 1.0), ([ident] * 4, 4.0)):
        I = dec.camera_cnn(F, cam, e, w_in, b_in, blocks, [np.zeros(32)] * 4, w_out, b_out).numpy()
        np.testing.assert_allclose(I[..., 0], gain * np.maximum(F[..., 0], 0) * F[..., 0] + 0.5, rtol=1e-13, atol=1e-14)
        np.testing.assert_allclose(I[..., 1], 0.25 + gain * dx, rtol=1e-13)
        np.testing.assert_allclose(I[..., 2], gain * 0.7 * F[..., 2], rtol=1e-13, atol=1e-14)


def test_camera_directions():
    cam = _cam(6, 4)                      # cx = 3, cy = 2: the pixel (2.5.., ..) grid straddles the axis
    d = dec.camera_directions(cam).numpy()
    np.testing.assert_allclose(np.linalg.norm(d, axis=-1), 1.0, rtol=1e-14)
    # pixel centre (u, v) = (3.5, 2.5): camera-frame direction (0.5/5, 0.5/5, 1) normalised, rotated to the world
    dc = np.array([0.1, 0.1, 1.0]) / np.linalg.norm([0.1, 0.1, 1.0])
    np.testing.assert_allclose(d[2, 3], np.asarray(cam.R, np.float64).T @ dc, rtol=1e-7)
    yawed = _cam(6, 4, yaw=30.0)
    d2 = dec.camera_directions(yawed).numpy()
    np.testing.assert_allclose(d2[2, 3], np.asarray(yawed.R, np.float64).T @ dc, rtol=1e-7)
    assert not np.allclose(d2[2, 3], d[2, 3])


def test_camera_cnn_gradients_against_central_differences():
    rng = np.random.default_rng(5)
    cam = _cam(5, 4, yaw=10.0)
    Df, E = 4, 2
    shapes = [(cam.height, cam.width, Df), (E,), (32, Df + 3 + E, 3, 3), (32,)] + [(32, 32, 3, 3)] * 4 + [(32,)] * 4 + \
        [(6, 32), (6,)]
    vals = [rng.normal(0, 0.3, s) for s in shapes]
    up = rng.normal(size=(cam.height, cam.width, 3))
    leaves = [torch.tensor(v, dtype=torch.float64, requires_grad=True) for v in vals]

    def loss(ls):
        I = dec.camera_cnn(ls[0], cam, ls[1], ls[2], ls[3], ls[4:8], ls[8:12], ls[12], ls[13])
        return (I * torch.from_numpy(up)).sum()

    loss(leaves).backward()
    h = 1e-6
    for k in (0, 1, 2, 3, 4, 7, 8, 11, 12, 13):
        leaf = leaves[k]
        flat = leaf.grad.view(-1)
        for j in rng.choice(flat.numel(), min(4, flat.numel()), replace=False):
            fs = []
            for sgn in (1.0, -1.0):
                ls = [x.detach().clone() for x in leaves]
                ls[k].view(-1)[j] += sgn * h
                fs.append(float(loss(ls)))
            np.testing.assert_allclose(float(flat[j]), (fs[0] - fs[1]) / (2 * h), rtol=1e-5, atol=1e-8,
                                       err_msg=f"leaf {k} [{j}]")
