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

Pins (tests/test_oracle_decoders.py): a hand-worked network with closed-form outputs, the unit
directions of axis rays, and gradients against central differences.
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
