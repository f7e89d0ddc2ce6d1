"""MI355X-native differentiable camera + lidar Gaussian rasterizer (SplatAD, arXiv 2411.16816).

The compute path is libsplat.so (hand-written HIP for gfx950) behind the C ABI of
include/splat.h; `binding` marshals arguments to it from PyTorch tensors.
"""
from . import structs  # noqa: F401

__all__ = ["binding", "structs", "build"]
