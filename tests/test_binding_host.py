"""Host-side guards of the Python binding, on the CPU (no GPU call is reached): the saved-state
check of the differentiable render and the argument checks of the MCMC relocation."""
from types import SimpleNamespace

import pytest
import torch

from paper_2411_16816_amd import binding as B


def test_backward_refuses_state_newer_than_its_forward():
    sp = SimpleNamespace(generation=7)
    B.check_saved_state(sp, 7)                       # unchanged: accepted
    sp.generation = 8                                # the pass rendered again
    with pytest.raises(B.SplatError, match="used again"):
        B.check_saved_state(sp, 7)
    # backward itself checks first, before touching any device buffer
    ctx = SimpleNamespace(sp=sp, g=None, support=0, has_vel=False, generation=3)
    with pytest.raises(B.SplatError):
        B.SplatRenderFn.backward(ctx, None, None, None)


def test_every_state_changing_call_bumps_the_generation():
    """project, bin_sort, raster_fwd and set_capacity each bump the counter before any library
    call (checked with a library stub that records the calls)."""
    calls = []

    class Lib:
        def __getattr__(self, name):
            def f(*a):
                calls.append(name)
                return 0 if name != "splat_workspace_bytes" else 1024
            return f

    sp = B.SensorPass.__new__(B.SensorPass)
    sp.lib, sp.rig, sp.first, sp.count, sp.n_gauss = Lib(), SimpleNamespace(handle=None), 0, 1, 4
    sp.device = "cpu"
    sp.generation = 0
    sp.set_capacity(16)
    assert sp.generation == 1
    sp.batched, sp.lidar = True, False
    sp.status = torch.zeros(64, dtype=torch.uint8)
    for name, bump in (("project", lambda: sp.project(SimpleNamespace(struct=lambda: B.st.SplatGaussians()))),
                       ("bin_sort", lambda: sp.bin_sort())):
        before = sp.generation
        try:
            bump()
        except Exception:
            pass                                     # the stub cannot marshal every struct
        assert sp.generation == before + 1, name


def _gauss(n=10, c=5, **over):
    f = dict(dtype=torch.float32)
    g = dict(means=torch.zeros(n, 3, **f), log_scales=torch.zeros(n, 3, **f), quats=torch.zeros(n, 4, **f),
             opacities=torch.zeros(n, **f), velocities=torch.zeros(n, 3, **f), features=torch.zeros(n, c, **f))
    g.update(over)
    return B.GaussTensors(**g)


def test_relocate_arguments_checked_on_host():
    u = torch.zeros(10, dtype=torch.int32)
    B.check_relocate_args(_gauss(), u)                                   # valid
    B.check_relocate_args(_gauss(velocities=None), u)                    # velocities optional
    B.check_relocate_args(_gauss(), torch.zeros(12, dtype=torch.uint32))  # longer u, uint32
    bad = [
        (_gauss(), torch.zeros(9, dtype=torch.int32)),                   # u too short
        (_gauss(), torch.zeros(10, dtype=torch.int64)),                  # u wrong type
        (_gauss(), torch.zeros(20, dtype=torch.int32)[::2]),             # u not contiguous
        (_gauss(opacities=torch.zeros(9)), u),                           # short opacities
        (_gauss(quats=torch.zeros(10, 3)), u),                           # quats of 3 columns
        (_gauss(means=torch.zeros(10, 3, dtype=torch.float64)), u),      # float64 means
        (_gauss(features=torch.zeros(5, 10).t()), u),                    # non-contiguous features
        (_gauss(log_scales=torch.zeros(11, 3)), u),                      # row count differs
        (_gauss(features=None), u),                                      # features missing
    ]
    for g, uu in bad:
        with pytest.raises(B.SplatError):
            B.check_relocate_args(g, uu)
    # the public call refuses before loading or launching anything
    with pytest.raises(B.SplatError):
        B.mcmc_relocate(_gauss(), torch.zeros(3, dtype=torch.int32))
