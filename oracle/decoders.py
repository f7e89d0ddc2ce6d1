"""Oracle, decoders of the rendered features (Sec. 3.3: the lidar MLP; training-details
appendix: 2 layers, hidden dimension 32).

Plain FP64 torch (CPU).  Test infrastructure only.

Lidar decoder.  A lidar ray's rendered feature row F (C channels) is concatenated with the ray's
direction and decoded to intensity and ray-drop probability by a two-layer MLP:

    d = (cos(el) cos(az), cos(el) sin(az), sin(el))      unit direction, sensor frame
    x = [F, d]                                           C + 3 inputs
    h = ReLU(W1 x + b1)                                  W1 [32, C+3], b1 [32]
    z = W2 h + b2                                        W2 [2, 32],   b2 [2]
    intensity = sigmoid(z_0),   drop probability = sigmoid(z_1)

Readings (the paper names only the layer count and width; listed in the design notes): the
direction is the unit vector of the ray's azimuth and elevation in the lidar frame, the hidden
activation is ReLU, and both outputs pass through a sigmoid (an intensity normalised to [0, 1]
and the probability the ray-drop cross-entropy takes).  Weights are inputs (no trained model is
needed to define the operation).

Camera decoder (Sec. 3.2: a small CNN maps the feature image F, the ray directions d and a
camera embedding e to a per-pixel affine map of the rendered colour; training-details appendix:
two residual blocks of width 32 and kernel size 3, then a final linear layer):

    x  = [F, d, e]                      per pixel; d the unit ray direction through the pixel
                                        centre in the world frame, e broadcast to every pixel
    h0 = ReLU(conv_in(x))               3x3, D_f + 3 + E -> 32
    r_k = ReLU(conv_k1(h_{k-1}))        3x3, 32 -> 32          (k = 1, 2)
    h_k = ReLU(h_{k-1} + conv_k2(r_k))  3x3, 32 -> 32
    (M, b) = W_out h_2 + b_out          1x1, 32 -> 6 (M: channels 0-2, b: 3-5)
    I  = M * F_rgb + b                  F_rgb = the first three feature channels

Every convolution has a bias, zero padding and stride 1 and is a cross-correlation
(out[y, x] = sum_{i, j} w[i, j] in[y + i - 1, x + j - 1]).  Readings (not fixed by the paper;
listed in the design notes): the stem convolution from the input to width 32, the ReLU places
(inside each block and after the residual sum), M and b taken linearly from the final layer,
and the world-frame direction.  Weights and the embedding are inputs.

Pins (tests/test_oracle_decoders.py): a hand-worked network with closed-form outputs, the unit
directions of axis rays, gradients against central differences; for the camera decoder a
brute-force loop convolution on a small image, closed forms of a network whose blocks are
switched off, the pinhole directions, and gradients against central differences.
"""
import torch

from . import geometry as geo

HIDDEN = 32


def ray_direction(az, el):
    az, el = geo.t64(az), geo.t64(el)
    return torch.stack([torch.cos(el) * torch.cos(az), torch.cos(el) * torch.sin(az), torch.sin(el)], -1)


def lidar_mlp(F, az, el, w1, b1, w2, b2):
    """(intensity [R], drop probability [R]) of feature rows F [R, C] (float64, differentiable in
    F and the weights)."""
    x = torch.cat([geo.t64(F), ray_direction(az, el)], -1)
    h = torch.relu(x @ geo.t64(w1).T + geo.t64(b1))
    z = h @ geo.t64(w2).T + geo.t64(b2)
    return torch.sigmoid(z[:, 0]), torch.sigmoid(z[:, 1])


def camera_directions(cam):
    """[H, W, 3] unit world-frame directions of the rays through the pixel centres
    (x_c = R x_w + t; camera x right, y down, z forward)."""
    H, W = cam.height, cam.width
    v, u = torch.meshgrid(torch.arange(H, dtype=torch.float64) + 0.5, torch.arange(W, dtype=torch.float64) + 0.5,
                          indexing="ij")
    dc = torch.stack([(u - float(cam.cx)) / float(cam.fx), (v - float(cam.cy)) / float(cam.fy), torch.ones_like(u)], -1)
    dc = dc / torch.linalg.norm(dc, dim=-1, keepdim=True)
    return dc @ geo.t64(cam.R)          # R^T d_c, row-vector form


def conv3x3(x, w, b):
    """[H, W, Ci] -> [H, W, Co]: cross-correlation with w [Co, Ci, 3, 3], bias b, zero padding
    (a library 2-D convolution)."""
    y = torch.nn.functional.conv2d(x.permute(2, 0, 1)[None], w, b, padding=1)
    return y[0].permute(1, 2, 0)


def camera_cnn(F, cam, embed, w_in, b_in, w_blocks, b_blocks, w_out, b_out):
    """Decoded image I [H, W, 3] from the feature image F [H, W, D_f] (float64, differentiable
    in F, the embedding and every weight).  w_blocks / b_blocks: the four block convolutions in
    order (block 1 first, block 2 second)."""
    F = geo.t64(F)
    H, W, _ = F.shape
    e = geo.t64(embed)
    x = torch.cat([F, camera_directions(cam), e.expand(H, W, e.shape[0])], -1)
    h = torch.relu(conv3x3(x, geo.t64(w_in), geo.t64(b_in)))
    for k in range(2):
        r = torch.relu(conv3x3(h, geo.t64(w_blocks[2 * k]), geo.t64(b_blocks[2 * k])))
        h = torch.relu(h + conv3x3(r, geo.t64(w_blocks[2 * k + 1]), geo.t64(b_blocks[2 * k + 1])))
    z = h @ geo.t64(w_out).T + geo.t64(b_out)
    return z[..., 0:3] * F[..., 0:3] + z[..., 3:6]
