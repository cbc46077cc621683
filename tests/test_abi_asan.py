"""The host side of libptrt under AddressSanitizer, without a GPU.

The library's sources are compiled with the sanitizer on the host code
only (device code as usual) into a separate library, and the C driver in
tests/asan/abi_driver.c runs every host path that needs no device against
it: argument checks, handle life cycle with every setter, tables, error
messages, and the error paths of the calls that would allocate device
memory (they fail cleanly here).  Any heap or stack error or leak report
fails the test.  CPU only (about a minute of compilation).
"""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

from conftest import ROOT

ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
CSRC = os.path.join(ROOT, "paper_2602_06686_amd", "csrc")
SOURCES = ["ptrt_single.hip", "step_d2q9.hip", "step_d3q19.hip", "step_d3q27.hip",
           "ptrt_batch.hip"]


@pytest.mark.slow
def test_host_code_under_address_sanitizer(tmp_path):
    hipcc = os.path.join(ROCM, "bin", "hipcc")
    clang = os.path.join(ROCM, "llvm", "bin", "clang")
    if not (os.path.exists(hipcc) and os.path.exists(clang) and shutil.which("gcc")):
        pytest.skip("ROCm toolchain not found")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]

    def compile_one(src):
        obj = str(tmp_path / (os.path.splitext(src)[0] + ".o"))
        cmd = [hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
               "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer",
               *inc, "-c", os.path.join(CSRC, src), "-o", obj]
        res = subprocess.run(cmd, capture_output=True, text=True)
        assert res.returncode == 0, res.stderr[-2000:]
        return obj

    with ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    lib = str(tmp_path / "libptrt_asan.so")
    link = [os.path.join(ROCM, "llvm", "bin", "clang++"), "-shared", "-fPIC",
            "-fsanitize=address", "-o", lib, *objs, "-L", os.path.join(ROCM, "lib"),
            "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    res = subprocess.run(link, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-2000:]
    exe = str(tmp_path / "abi_driver")
    res = subprocess.run([clang, "-g", "-O1", "-fsanitize=address", "-fno-omit-frame-pointer",
                          *inc, os.path.join(ROOT, "tests", "asan", "abi_driver.c"), "-o", exe,
                          lib, "-Wl,-rpath," + str(tmp_path)], capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:abort_on_error=0")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    out = run.stdout + run.stderr
    print(out[-3000:])
    assert "AddressSanitizer" not in out and "LeakSanitizer" not in out
    assert run.returncode == 0 and "\n0 failed" in out
