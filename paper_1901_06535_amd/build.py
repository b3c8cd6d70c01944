"""Build ``librdc.so`` (the C-ABI library of include/rdc.h) with hipcc for
gfx950, in-tree next to this file.

    python -m paper_1901_06535_amd.build
"""
from __future__ import annotations

import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "librdc.so")
ARCH = "gfx950"

HIP_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared",
    "--offload-arch=" + ARCH,
    # Packed FP32 (v_pk_fma_f32 and friends) stays off: every float op is
    # issued unpacked.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


# Per-source hipcc flags.  The row-pipeline kernels are scheduled for
# instruction-level parallelism: each loop body is a long straight-line run
# of independent cell updates, and the scheduler's iterative ILP strategy
# keeps more of them in flight at the same register count (2% faster on the
# 16384^2 workload at T = 11).  Other sources keep the default strategy (the
# compiler fails on some of them with this one).
SOURCE_FLAGS = {"stream.hip": ["-mllvm", "-amdgpu-sched-strategy=iterative-ilp"]}


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    proc = subprocess.run(cmd, capture_output=True, text=True)
    if proc.returncode != 0:
        sys.stderr.write(proc.stdout + proc.stderr)
        raise RuntimeError("hipcc failed: %s" % " ".join(cmd[-3:]))


def build(verbose: bool = False, out: str = LIB, extra=()) -> str:
    """Compile every csrc/*.hip (in parallel, one object each; no device code
    crosses files) and link one shared library at `out`.  `extra` (or the
    RDC_EXTRA_FLAGS environment variable) adds hipcc flags, e.g. the
    build-time tunables -DRDC_STEP1_ROWS=32."""
    import tempfile
    from concurrent.futures import ThreadPoolExecutor
    extra = list(extra) + os.environ.get("RDC_EXTRA_FLAGS", "").split()
    flags = [f for f in HIP_FLAGS if f != "-shared"]
    with tempfile.TemporaryDirectory(prefix="rdc_build_") as tmpd:
        objs = [os.path.join(tmpd, os.path.basename(src) + ".o") for src in sources()]
        cmds = [[hipcc()] + flags + SOURCE_FLAGS.get(os.path.basename(src), []) + extra +
                ["-c", src, "-o", obj] for src, obj in zip(sources(), objs)]
        workers = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
        with ThreadPoolExecutor(max_workers=workers) as ex:
            list(ex.map(lambda c: _run(c, verbose), cmds))
        tmp = out + ".tmp%d" % os.getpid()
        _run([hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs, verbose)
        os.replace(tmp, out)
    return out


if __name__ == "__main__":
    out = sys.argv[1] if len(sys.argv) > 1 else LIB
    print(build(verbose=True, out=out, extra=sys.argv[2:]))
