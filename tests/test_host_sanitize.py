"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only): the
oracle and the input generator (gcc), the serving arena allocator (g++), and the
library's host-side C ABI paths -- option resolution, layout arithmetic, argument
and error checks -- with every HIP source built for the host with the sanitizers
(the device code is compiled as usual, and no device work is done)."""
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

from conftest import ROOT

SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang"
CSRC = os.path.join(ROOT, "paper_2605_29604_amd", "csrc")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def run(cmd, **kw):
    res = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert res.returncode == 0, f"{' '.join(cmd)}\n{res.stdout}\n{res.stderr}"
    return res.stdout


def test_oracle_and_generator_sanitized(tmp_path):
    exe = str(tmp_path / "oracle_gen_check")
    run(["gcc", "-std=c11", "-g", "-O1", *SAN, os.path.join(ROOT, "oracle", "mis_oracle.c"),
         os.path.join(ROOT, "paper_2605_29604_amd", "gen", "graphgen.c"),
         os.path.join(ROOT, "tests", "host", "oracle_gen_check.c"), "-lpthread", "-lm", "-o", exe])
    assert run([exe], env=ENV, timeout=120).startswith("ok")


def test_arena_sanitized(tmp_path):
    exe = str(tmp_path / "arena_check")
    run(["g++", "-std=c++17", "-g", "-O1", *SAN, os.path.join(ROOT, "tests", "host", "arena_check.cpp"), "-o", exe])
    assert run([exe], env=ENV, timeout=120).startswith("ok")


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="ROCm toolchain not found")
def test_c_abi_host_paths_sanitized(tmp_path):
    srcs = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip")) + ["rcm.cpp"]
    host_san = []
    for f in SAN:   # host side only: each sanitizer flag goes to the host compilation
        host_san += ["-Xarch_host", f]

    def compile_one(src):
        obj = str(tmp_path / (os.path.splitext(src)[0] + ".o"))
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        run([HIPCC, *lang, "-O1", "-g", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature",
             "-Xclang", "-packed-fp32-ops", *host_san, "-c", os.path.join(CSRC, src), "-o", obj])
        return obj

    with ThreadPoolExecutor(min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, srcs))
    drv = str(tmp_path / "abi_check.o")
    run([CLANG, "-g", "-O1", *SAN, "-c", os.path.join(ROOT, "tests", "host", "abi_check.c"), "-o", drv])
    exe = str(tmp_path / "abi_check")
    run([CLANG + "++", *SAN, *objs, drv, "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe])
    # the HIP runtime keeps allocations of its own until exit: leak reports are off here
    env = dict(ENV, ASAN_OPTIONS="detect_leaks=0")
    assert run([exe], env=env, timeout=120).startswith("ok")
