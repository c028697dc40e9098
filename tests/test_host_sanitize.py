"""The host code of libwolf (argument validation, buffer and overlap checks, plan validity, launch
set-up, graph recording) built for the CPU with AddressSanitizer and UndefinedBehaviorSanitizer, and
driven through every entry point of include/wolf.h (tests/host/check_host.cpp) against a host-only
stand-in of the HIP runtime (tests/host/hip_stub.cpp): no GPU, no kernel runs. Each library source is
compiled host-only (its device code is not built); the sanitizers apply to the host compilation only."""
from __future__ import annotations

import os
import re
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2203_02734_amd", "csrc")
HOSTDIR = os.path.join(HERE, "host")
HIPCC = "/opt/rocm/bin/hipcc"
CLANGXX = "/opt/rocm/llvm/bin/clang++"


def _sources():
    import importlib.util

    spec = importlib.util.spec_from_file_location("wolf_build", os.path.join(ROOT, "paper_2203_02734_amd", "build.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return [os.path.join(CSRC, s) for s in m.SOURCES]


def _host_compile(src, obj):
    # Each sanitizer flag applies to the host compilation only (-Xarch_host before it).
    cmd = [HIPCC, "-x", "hip", "--cuda-host-only", "-O1", "-g", "-std=c++17", "-fPIC", "-fno-omit-frame-pointer",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-I", HOSTDIR,
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-c", src, "-o", obj]
    return subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANGXX)), reason="ROCm compilers not installed")
def test_host_code_under_asan_ubsan(tmp_path):
    srcs = _sources() + [os.path.join(HOSTDIR, "hip_stub.cpp"), os.path.join(HOSTDIR, "check_host.cpp")]
    objs, procs = [], []
    for s in srcs:
        o = str(tmp_path / (os.path.basename(s) + ".o"))
        objs.append(o)
        procs.append((s, _host_compile(s, o)))
    for s, p in procs:
        out, err = p.communicate()
        assert p.returncode == 0, f"host compile of {s} failed:\n{err[-3000:]}"
    # Host-only objects refer to the device code objects they were built without; the stand-in's
    # registration ignores them, so empty definitions satisfy the link.
    nm = subprocess.run(["nm", "-u", *objs], capture_output=True, text=True, check=True).stdout
    names = sorted(set(re.findall(r"\b(__hip_fatbin_[0-9a-f]+)\b", nm)))
    stub_c = tmp_path / "fatbin_stubs.cpp"
    stub_c.write_text("".join(f'extern "C" char {n}[16];\nchar {n}[16] = {{0}};\n' for n in names))
    fat_o = str(tmp_path / "fatbin_stubs.o")
    subprocess.run([CLANGXX, "-c", str(stub_c), "-o", fat_o], check=True)
    exe = str(tmp_path / "check_host")
    link = subprocess.run([CLANGXX, "-fsanitize=address,undefined", "-o", exe, *objs, fat_o, "-lpthread", "-lm"],
                          capture_output=True, text=True)
    assert link.returncode == 0, link.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert run.returncode == 0 and "ALL OK" in run.stdout, (run.stdout[-2000:] + run.stderr[-6000:])
