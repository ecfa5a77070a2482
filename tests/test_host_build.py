"""Host-only build of the library's host runtime (api.cpp) under AddressSanitizer and
UndefinedBehaviorSanitizer, run against a fake HIP runtime (tests/hostbuild/): argument
validation before any work, injected device-allocation failures (NV_E_NOMEM, nothing
half-built left behind, the context and streams usable afterwards), ordering of the
shared workspace and of a clip stream's state across HIP streams, and no leaked
allocation.  No GPU and no kernel is involved; the launchers are stubs that check every
device pointer they receive against the fake allocation registry."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HB = os.path.join(ROOT, "tests", "hostbuild")
CXX = "/opt/rocm/llvm/bin/clang++"


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    cxx = CXX if os.path.exists(CXX) else shutil.which("clang++")
    if cxx is None:
        pytest.skip("no clang++ with _Float16 support for the host-only build")
    exe = str(tmp_path_factory.mktemp("hostbuild") / "host_driver")
    cmd = [cxx, "-std=c++17", "-g", "-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer", "-I" + os.path.join(HB, "fake_hip"), "-I" + os.path.join(ROOT, "include"),
           os.path.join(ROOT, "paper_2308_03121_amd", "csrc", "api.cpp"), os.path.join(HB, "fake_runtime.cpp"),
           os.path.join(HB, "host_driver.cpp"), "-o", exe]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-4000:]
    return exe


def test_host_runtime_under_sanitizers(driver):
    env = dict(os.environ)
    env.pop("NNVISR_FAULT_ALLOC_MIN_BYTES", None)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0"
    res = subprocess.run([driver], capture_output=True, text=True, env=env, timeout=300)
    out = res.stdout + res.stderr
    assert res.returncode == 0, out[-4000:]
    for case in ("validation_before_any_work", "workspace_nomem_then_retry", "stream_open_nomem_then_clip",
                 "batch_nomem_stream_usable", "ordering_across_streams", "nothing_leaks"):
        assert f"ok {case}" in res.stdout, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out
