"""Sanitizer builds of the host code (no GPU): the C oracle under
AddressSanitizer + UndefinedBehaviorSanitizer, and libaerl's host code
(validation, multi-threaded packing, launch planning, the evolution loop's
breeding) under ASan + UBSan and under ThreadSanitizer, each driven by a
small program in tests/sanitize/.  The library's device code is built as
usual; only its host side carries the instrumentation."""
import concurrent.futures as cf
import glob
import os
import subprocess

import pytest

from paper_2406_01821_amd.build_lib import SOURCES

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2406_01821_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang++"


def _run(cmd, env=None, timeout=600):
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=timeout)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-3000:]}\n{r.stderr[-6000:]}"
    return r.stdout


def _clang_rt_dir():
    hits = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    return os.path.dirname(hits[0]) if hits else None


def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_asan")
    _run(["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
          "-fno-omit-frame-pointer", "-fopenmp", "-ffp-contract=off", "-std=gnu11",
          os.path.join(ROOT, "oracle", "aerl_oracle.c"),
          os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"), "-lm", "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", OMP_NUM_THREADS="4")
    assert "all calls returned 0" in _run([exe], env=env)


def _build_library(out, sanitizers):
    os.makedirs(out, exist_ok=True)
    fl = ["--offload-arch=gfx950", "-O1", "-g", "-fPIC", "-std=c++17", "-ffp-contract=off",
          "-fno-fast-math", "-fno-gpu-flush-denormals-to-zero", "-Xclang", "-target-feature",
          "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
          "-Xarch_host", "-fno-omit-frame-pointer"]
    for s in sanitizers:
        fl += ["-Xarch_host", f"-fsanitize={s}"]

    def one(src):
        obj = os.path.join(out, os.path.splitext(src)[0] + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        _run([HIPCC, *fl, *lang, "-c", os.path.join(CSRC, src), "-o", obj])
        return obj

    with cf.ThreadPoolExecutor(max_workers=8) as ex:
        objs = list(ex.map(one, SOURCES))
    lk = ["--offload-arch=gfx950", "-shared", "-fPIC", "-shared-libsan"]
    for s in sanitizers:
        lk += ["-Xarch_host", f"-fsanitize={s}"]
    lib = os.path.join(out, "libaerl_san.so")
    _run([HIPCC, *lk, "-o", lib, *objs, "-lpthread"])
    exe = os.path.join(out, "driver")
    _run([CLANG, "-g", "-O1", "-std=c++17", *[f"-fsanitize={s}" for s in sanitizers],
          "-shared-libsan", "-I", os.path.join(ROOT, "include"), "-D__HIP_PLATFORM_AMD__",
          "-I", "/opt/rocm/include", os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp"),
          "-L", out, "-laerl_san", f"-Wl,-rpath,{out}", "-o", exe])
    return exe


@pytest.mark.skipif(not os.path.exists(HIPCC) or _clang_rt_dir() is None,
                    reason="needs hipcc and the clang sanitizer runtimes")
@pytest.mark.parametrize("sanitizers,opts", [
    (("address", "undefined"), {"ASAN_OPTIONS": "detect_leaks=0",
                                "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}),
    (("thread",), {"TSAN_OPTIONS": "halt_on_error=1"}),
])
def test_library_host_code_under_sanitizers(tmp_path, sanitizers, opts):
    exe = _build_library(str(tmp_path / "_".join(sanitizers)), sanitizers)
    env = dict(os.environ, LD_LIBRARY_PATH=_clang_rt_dir(), **opts)
    assert "all checks passed" in _run([exe], env=env)
