"""The C ABI's host side under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only): every
library source is compiled with the sanitizers on its host code (device code unchanged) and
linked with tests/host/abi_host_check.cpp, which drives sensor validation, workspace sizing and
the entry points' argument checks (no device is touched).  Any sanitizer report or failed
expectation fails the test."""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2411_16816_amd", "csrc")
sys.path.insert(0, ROOT)
from paper_2411_16816_amd.build import SOURCES  # noqa: E402

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# sanitizers on the host code only: each -fsanitize= follows -Xarch_host
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined"]
FLAGS = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
         "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), "-w"]


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    out = tmp_path_factory.mktemp("hostsan")
    objs = [str(out / s.replace(".hip", ".o")) for s in SOURCES]

    def compile_one(args):
        src, obj = args
        r = subprocess.run([HIPCC, *FLAGS, *SAN, "-c", os.path.join(CSRC, src), "-o", obj],
                           capture_output=True, text=True)
        return src, r.returncode, r.stdout + r.stderr

    with ThreadPoolExecutor(max_workers=min(4, os.cpu_count() or 1)) as ex:
        for src, rc, log in ex.map(compile_one, zip(SOURCES, objs)):
            assert rc == 0, f"{src}: {log[-2000:]}"
    exe = str(out / "abi_host_check")
    r = subprocess.run([HIPCC, "-O1", "-g", "-std=c++17", "--offload-arch=gfx950", "-I", os.path.join(ROOT, "include"),
                        *SAN, *objs, os.path.join(ROOT, "tests", "host", "abi_host_check.cpp"), "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    yield exe
    shutil.rmtree(out, ignore_errors=True)


def test_host_abi_under_sanitizers(checker):
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1"   # the GPU runtime's own allocations are not ours
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["HIP_VISIBLE_DEVICES"] = ""
    r = subprocess.run([checker], capture_output=True, text=True, env=env, timeout=300)
    log = r.stdout + r.stderr
    assert "runtime error" not in log and "AddressSanitizer" not in log, log[-4000:]
    assert r.returncode == 0, log[-4000:]
    assert "0 failed" in log, log[-4000:]
