"""Host code under AddressSanitizer and UBSan, on the CPU.

* librdc's host code (every .hip source compiled host-only, so argument
  checks, launch planning, plane copies, batch tables and graph recording)
  linked against a host-memory stand-in for the HIP runtime
  (host_sanitize/hip_shim.c) and driven through every entry point of
  include/rdc.h by host_sanitize/api_driver.c: expected statuses, write/read
  round trips, launch counts, no launch with an empty or oversized grid, no
  leaked allocation.
* the C oracle, serial and OpenMP, through host_sanitize/oracle_driver.c.

Kernels do not run here; their numerics are the GPU tests' business.
"""
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "host_sanitize")
INC = os.path.join(ROOT, "include")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _tool(name):
    for cand in (shutil.which(name), os.path.join("/opt/rocm/bin", name),
                 os.path.join("/opt/rocm/llvm/bin", name)):
        if cand and os.path.exists(cand):
            return cand
    pytest.skip("%s not found" % name)


def _run(cmd, **kw):
    p = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert p.returncode == 0, "%s\n%s%s" % (" ".join(cmd), p.stdout, p.stderr[-4000:])
    return p.stdout


def test_library_host_code_is_clean_under_asan_and_ubsan(tmp_path):
    hipcc, clang = _tool("hipcc"), _tool("clang")
    clangxx = os.path.join(os.path.dirname(clang), "clang++")
    objs = []
    for src in sorted(glob.glob(os.path.join(ROOT, "paper_1901_06535_amd", "csrc", "*.hip"))):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        # host-only compile: the sanitizer flags reach the host pass only
        _run([hipcc, "-O1", "-g", "-std=c++17", "--cuda-host-only",
              "-Xarch_host", SAN[0], "-Xarch_host", SAN[1], "-I", INC, "-c", src, "-o", obj])
        objs.append(obj)
    for src in ("hip_shim.c", "api_driver.c"):
        obj = str(tmp_path / (src + ".o"))
        _run([clang, "-O1", "-g"] + SAN + ["-I", INC, "-c", os.path.join(HERE, src), "-o", obj])
        objs.append(obj)
    # host-only objects still name their (absent) device code blobs
    syms = set()
    for line in _run(["nm"] + objs).splitlines():
        parts = line.split()
        if len(parts) == 2 and parts[0] == "U" and parts[1].startswith("__hip_fatbin_"):
            syms.add(parts[1])
    stub = tmp_path / "fatbin.c"
    stub.write_text("".join("const char %s[8] = {0};\n" % s for s in sorted(syms)))
    _run([clang, "-c", str(stub), "-o", str(tmp_path / "fatbin.o")])
    exe = str(tmp_path / "api_driver")
    _run([clangxx] + SAN + objs + [str(tmp_path / "fatbin.o"), "-o", exe, "-lm"])
    out = _run([exe], env=ENV)
    print(out)
    assert "ALL OK" in out


@pytest.mark.parametrize("openmp", [False, True])
def test_oracle_is_clean_under_asan_and_ubsan(tmp_path, openmp):
    gcc = _tool("gcc")
    exe = str(tmp_path / "oracle_driver")
    _run([gcc, "-O1", "-g"] + (["-fopenmp"] if openmp else []) + SAN +
         [os.path.join(ROOT, "oracle", "rdc_oracle.c"), os.path.join(HERE, "oracle_driver.c"),
          "-o", exe, "-lm"])
    out = _run([exe], env=dict(ENV, OMP_NUM_THREADS="4"))
    print(out)
    assert "ALL OK" in out
