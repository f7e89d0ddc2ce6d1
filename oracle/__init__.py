"""FP64 CPU oracle for the SplatAD camera + lidar Gaussian rasterizer (arXiv 2411.16816).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously-correct reference written
from the paper's equations.  Only the test suite, the smoke check and the benchmark's CPU
baseline leg may import it; the product library never calls it and shares no code with it.

Layout:
  geometry  -- Gaussian covariance, sensor frames, camera / lidar projection, rolling-shutter
               velocities, EWA dilation and boxes (Sec. 3.1-3.3, App. D)
  tiles     -- camera and lidar tile ranges (Sec. 3.2, App. A) in FP64, plus an FP32 emulation
               of the library's documented tile arithmetic for bit-exact stage checks
  render    -- brute-force per-ray compositing over every Gaussian (Eqs. t_pix, alpha_blend,
               alpha, delta; expected and median range), BOX and TILE candidate rules
  grad      -- reference gradients by FP64 autograd and by central finite differences
  compose   -- scene-graph composition at a capture time: actor-frame Gaussians to world means,
               rotations and rigid-body velocities (Sec. 3.1, Eq. pixel_velocity, App. D)
  points    -- lidar points to rasterisation rays: ego-motion compensation removed, spherical
               coordinates (App. A)
  mcmc      -- the MCMC opacity and scale regulariser of the training-details appendix
  decoders  -- the lidar MLP decoding rendered features to intensity and ray-drop probability

Parity status of every function is listed in each module header.  "Parity unpinned" items:
the value of the lidar dilation s_L and the Jacobian clamp constant are conventions passed in
as inputs (the paper prints no worked values for them).
"""
from . import geometry, tiles, render, grad, compose, points, mcmc, decoders  # noqa: F401
