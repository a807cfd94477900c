"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the host code:
the C oracle, and the library's host paths (argument checks, planners,
workspace sizes, tuning files, quantizer tables). The library is compiled
with the sanitizers on its host code only (device code is built as usual)
and loaded by a small driver with dlopen; nothing here needs a GPU. A
sanitizer report aborts the driver with a non-zero status."""
import glob
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]


def _run(cmd, **kw):
    p = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert p.returncode == 0, f"{' '.join(cmd[:3])} ... failed ({p.returncode}):\n{p.stdout[-2000:]}\n{p.stderr[-4000:]}"
    return p


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_asan")
    _run(["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fopenmp",
          os.path.join(ROOT, "oracle", "tde_oracle.c"), os.path.join(ROOT, "tests", "asan", "oracle_driver.c"),
          "-lm", "-o", exe])
    p = _run([exe], env=ENV, timeout=300)
    assert "oracle driver: ok" in p.stdout


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="ROCm toolchain not available")
def test_library_host_code_under_sanitizers(tmp_path):
    srcs = sorted(glob.glob(os.path.join(ROOT, "paper_2509_19974_amd", "csrc", "*.hip")))
    flags = ["--offload-arch=gfx950", "-O2", "-g", "-std=c++17", "-fPIC", "-Xclang", "-target-feature", "-Xclang",
             "-packed-fp32-ops", "-fno-omit-frame-pointer", "-Wno-unused-command-line-argument",
             "-I", os.path.join(ROOT, "include")] + SAN

    def compile_one(s):
        o = str(tmp_path / (os.path.basename(s)[:-4] + ".o"))
        _run([HIPCC] + flags + ["-c", s, "-o", o])
        return o

    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, srcs))
    lib = str(tmp_path / "libtde_san.so")
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + SAN + objs + ["-o", lib])
    drv = str(tmp_path / "host_driver")
    _run([CLANG, "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
          "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "asan", "host_driver.c"),
          "-o", drv, "-ldl"])
    tune = os.path.join(ROOT, "paper_2509_19974_amd", "weights", "tune_mi355x.txt")
    p = _run([drv, lib, str(tmp_path), tune], env=ENV, timeout=600)
    assert "host driver:" in p.stdout
