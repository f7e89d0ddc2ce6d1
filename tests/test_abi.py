"""CPU checks of the C ABI: the library loads, exports every function include/splat.h declares,
and validates sensor descriptions on the host (no device call)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from scenes import synthetic as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2411_16816_amd import binding
    try:
        return binding.load()
    except RuntimeError as e:
        pytest.fail(str(e))


def test_exports_every_declared_function():
    lib = _lib()
    hdr = open(os.path.join(ROOT, "include", "splat.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    names = set(re.findall(r"\b(splat_[a-z0-9_]+)\s*\(", hdr))
    assert len(names) >= 16
    for n in sorted(names):
        assert hasattr(lib, n), n


def test_status_strings():
    lib = _lib()
    assert lib.splat_status_string(0) == b"ok"
    assert lib.splat_status_string(1) == b"invalid argument"
    assert lib.splat_status_string(99) == b"unknown status"


def test_camera_validation_on_host():
    from paper_2411_16816_amd import structs as st
    lib = _lib()
    cam = S.make_camera((0, 0, 1.5), 0.0, 1920, 1080, 1500.0, t_rs=0.03)
    assert lib.splat_check_camera(C.byref(st.camera_struct(cam))) == 0
    for field, val in [("width", 0), ("fx", -1.0), ("tile_w", 0), ("near", 0.0), ("eps2d", -0.1), ("n_channels", 65)]:
        bad = S.make_camera((0, 0, 1.5), 0.0, 1920, 1080, 1500.0, t_rs=0.03)
        setattr(bad, field, val)
        assert lib.splat_check_camera(C.byref(st.camera_struct(bad))) == 1, field
    big = S.make_camera((0, 0, 1.5), 0.0, 1920, 1080, 1500.0, tile=(32, 16))   # 512 px per tile
    assert lib.splat_check_camera(C.byref(st.camera_struct(big))) == 1
    assert lib.splat_check_camera(None) == 1


def test_lidar_validation_on_host():
    from paper_2411_16816_amd import structs as st
    lib = _lib()
    lid = S.make_lidar((0, 0, 0), 0.0, 32, -25.0, 10.0, 1024)
    keep = []
    s = st.lidar_struct(lid, (1, 1, 1), keep)
    assert lib.splat_check_lidar(C.byref(s)) == 0
    # non-monotone elevation boundaries
    bad = S.make_lidar((0, 0, 0), 0.0, 32, -25.0, 10.0, 1024)
    bad.elev_bounds = bad.elev_bounds[::-1].copy()
    assert lib.splat_check_lidar(C.byref(st.lidar_struct(bad, (1, 1, 1), keep))) == 1
    # azimuth tiles that do not cover a full turn
    bad = S.make_lidar((0, 0, 0), 0.0, 32, -25.0, 10.0, 1024)
    bad.n_az_tiles = 31
    assert lib.splat_check_lidar(C.byref(st.lidar_struct(bad, (1, 1, 1), keep))) == 1
    # rays without arrays
    assert lib.splat_check_lidar(C.byref(st.lidar_struct(lid, (None, None, None), keep))) == 1


def test_rig_create_rejects_bad_counts_without_device():
    lib = _lib()
    h = C.c_void_p()
    assert lib.splat_rig_create(0, 0, C.byref(h)) == 1
    assert lib.splat_rig_create(-1, 2, C.byref(h)) == 1
    assert lib.splat_rig_create(2000, 0, C.byref(h)) == 1
    assert lib.splat_workspace_bytes(None, 0, 1, 10, 10) == 0
