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
    # valid but beyond the binning kernels' limits (unsupported, code 4): 65536 tiles across a
    # row, and 2^24 tiles in total
    wide = S.make_camera((0, 0, 1.5), 0.0, 65536, 4, 1500.0, tile=(1, 1))
    assert lib.splat_check_camera(C.byref(st.camera_struct(wide))) == 4
    many = S.make_camera((0, 0, 1.5), 0.0, 4096, 4096, 1500.0, tile=(1, 1))
    assert lib.splat_check_camera(C.byref(st.camera_struct(many))) == 4
    edge = S.make_camera((0, 0, 1.5), 0.0, 65535, 4, 1500.0, tile=(1, 1))
    assert lib.splat_check_camera(C.byref(st.camera_struct(edge))) == 0


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


def test_struct_layouts_match_header(tmp_path):
    """sizeof / offsetof of every public struct, compiled from include/splat.h with gcc, against
    the ctypes mirrors the binding passes across the ABI."""
    from paper_2411_16816_amd import structs as st
    mirrors = [st.SplatStatus, st.SplatGaussians, st.SplatCamera, st.SplatLidar, st.SplatRigLayout,
               st.SplatProjected, st.SplatTileLists, st.SplatRenderOut, st.SplatGrads, st.SplatStep,
               st.SplatActors, st.SplatActorGrads, st.SplatLidarMLP, st.SplatLidarMLPGrads, st.SplatCameraCNN,
               st.SplatCameraCNNGrads, st.SplatGaussianState]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "splat.h"', "int main(void) {"]
    for m in mirrors:
        n = m.__name__
        lines.append(f'  printf("{n} size %zu\\n", sizeof({n}));')
        for f in m._fields_:
            lines.append(f'  printf("{n} {f[0]} %zu\\n", offsetof({n}, {f[0]}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    import subprocess
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            a, b, v = line.split()
            got[(a, b)] = int(v)
    for m in mirrors:
        n = m.__name__
        assert got[(n, "size")] == C.sizeof(m), n
        for f in m._fields_:
            assert got[(n, f[0])] == getattr(m, f[0]).offset, (n, f[0])
