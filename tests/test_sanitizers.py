"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

1. The FP64 oracle: oracle/sanitize_check.c (which includes lbm_oracle.c)
   built with gcc and both sanitizers, every entry point exercised on small
   cavities of every wall type and force model.
2. The C-ABI's host paths: the HIP library rebuilt with the sanitizers on its
   host code only (each sanitizer flag right after -Xarch_host), loaded into
   a Python subprocess with the sanitizer runtime preloaded, and driven by
   tests/sanitize_abi_host.py through every call that returns before device
   work (parameter validation, sizes, error strings, NULL handles, rejected
   kernel shapes).
A finding aborts the run (no recovery), so a zero exit status means clean.
"""
import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "sanitize_check")
    subprocess.check_call(
        ["gcc", "-std=c99", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
         "-fno-omit-frame-pointer", "-ffp-contract=off", "-fopenmp", "-Wall", "-Wextra", "-o", exe,
         os.path.join(ROOT, "oracle", "sanitize_check.c"), "-lm"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", OMP_NUM_THREADS="2")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr[-4000:]
    assert "ran clean" in r.stdout


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_abi_host_paths_under_asan_ubsan(tmp_path):
    runtime = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not runtime:
        pytest.skip("clang AddressSanitizer runtime not found")
    host_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-sanitize-recover=all"]
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", os.path.join(ROOT, "include")] + host_san
    srcs = [os.path.join(ROOT, "paper_1511_04633_amd", "csrc", f)
            for f in ("lbmx.hip", "batch.hip", "nn.hip")]

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        subprocess.check_call([HIPCC, *flags, "-c", "-o", obj, src], stderr=subprocess.DEVNULL)
        return obj

    with ThreadPoolExecutor(max_workers=3) as ex:
        objs = list(ex.map(compile_one, srcs))
    lib = str(tmp_path / "liblbmx_sanitized.so")
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *host_san[:4],
                           "-o", lib, *objs])
    env = dict(os.environ, LD_PRELOAD=runtime[-1], ASAN_OPTIONS="detect_leaks=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "sanitize_abi_host.py"), lib],
                       capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr[-4000:]
    assert "ran clean" in r.stdout
