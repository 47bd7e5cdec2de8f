"""The C ABI's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

`ebv_api.cpp` (argument checks, workspace sizing, skyline planning, batch
order, handles, the tuning-table reader) is rebuilt with the sanitizers on
its host side only (each -fsanitize= behind -Xarch_host; no device code is
instrumented), linked with the library's kernel object, and the host ABI
tests (`test_abi_host.py`, no GPU needed) run against that build in a child
process with the sanitizer runtime preloaded.  The test passes when they all
pass and the sanitizers report nothing (no recovery: the first finding
aborts the child).
"""
import glob
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

CHILD = r"""
import sys
sys.path.insert(0, sys.argv[2])
from paper_1907_05767_amd import ebv
ebv.LIB_PATH = sys.argv[1]
import pytest
sys.exit(pytest.main(["-q", "-p", "no:cacheprovider", "-m", "not gpu",
                      sys.argv[2] + "/tests/test_abi_host.py"]))
"""


def _asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="needs hipcc")
def test_host_abi_under_asan_and_ubsan(tmp_path):
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("no AddressSanitizer runtime for hipcc's clang")
    from paper_1907_05767_amd import build

    kernels_o = os.path.join(build.BUILD, "ebv_kernels.hip.o")
    if not os.path.exists(kernels_o):
        build.build()
    api_o, so = str(tmp_path / "ebv_api_san.o"), str(tmp_path / "libebv_san.so")
    subprocess.check_call([
        "hipcc", "-x", "hip", "-O1", "-g", "-std=c++17", "-fPIC", f"--offload-arch={build.ARCH}",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", os.path.join(ROOT, "paper_1907_05767_amd", "csrc"), "-I", os.path.join(ROOT, "include"),
        "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
        "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
        "-c", os.path.join(ROOT, "paper_1907_05767_amd", "csrc", "ebv_api.cpp"), "-o", api_o])
    subprocess.check_call([
        "hipcc", f"--offload-arch={build.ARCH}", "-shared", "-fPIC",
        "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-shared-libsan",
        api_o, kernels_o, "-o", so])
    logs = str(tmp_path / "san")
    env = dict(os.environ)
    env["LD_PRELOAD"] = rt
    env["ASAN_OPTIONS"] = f"detect_leaks=0:exitcode=23:log_path={logs}"
    env["UBSAN_OPTIONS"] = f"print_stacktrace=1:halt_on_error=1:log_path={logs}"
    res = subprocess.run([sys.executable, "-c", CHILD, so, ROOT], env=env, capture_output=True, text=True,
                         timeout=900)
    reports = ""
    for f in glob.glob(logs + "*"):
        with open(f) as fh:
            reports += fh.read()
    assert res.returncode == 0 and not reports, (res.stdout[-3000:] + res.stderr[-2000:] + reports[-4000:])
    assert " passed" in res.stdout
