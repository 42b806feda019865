"""Build the HIP shared library libali.so in-tree for gfx950 (hipcc cross-compiles on a
host without a GPU), and the C-ABI test driver whose host code carries AddressSanitizer and
UndefinedBehaviorSanitizer (tests/sanitize/abi_driver_asan)."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libali.so")
SOURCES = ["ali_capi.hip", "ali_solve.hip", "ali_rays.hip", "ali_adjoint.hip", "ali_refine.hip"]
ASAN_DRIVER_SRC = os.path.join(ROOT, "tests", "sanitize", "abi_driver.cpp")
ASAN_DRIVER = os.path.join(ROOT, "tests", "sanitize", "abi_driver_asan")

HIPFLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no implicit multiply-add contraction: the same estimate must round identically in
    # every kernel that evaluates it (fused operations are written out where wanted)
    "-ffp-contract=off",
    # never emit packed fp32 arithmetic (v_pk_*_f32)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]
# host code only: each sanitizer flag applies to the host compilation (-Xarch_host), the
# device code is built as usual
HOST_SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-omit-frame-pointer", "-g"]


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def _compile_all(jobs, verbose):
    """Compile (cmd, ...) jobs in parallel (at most 8 at a time)."""
    with ThreadPoolExecutor(max_workers=min(8, max(1, len(jobs)))) as ex:
        for f in [ex.submit(_run, cmd, verbose) for cmd in jobs]:
            f.result()


def build(verbose: bool = False, sanitizer_driver: bool = True) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    inc = ["-I", os.path.join(ROOT, "include")]
    jobs, objs, aobjs = [], [], []
    for src in sources():
        obj = os.path.join(CSRC, os.path.basename(src).replace(".hip", ".o"))
        jobs.append([hipcc] + HIPFLAGS + inc + ["-c", src, "-o", obj])
        objs.append(obj)
        if sanitizer_driver:
            aobj = os.path.join(CSRC, os.path.basename(src).replace(".hip", ".asan.o"))
            jobs.append([hipcc] + HIPFLAGS + HOST_SANITIZE + inc + ["-c", src, "-o", aobj])
            aobjs.append(aobj)
    if sanitizer_driver:
        dobj = ASAN_DRIVER + ".o"
        jobs.append([hipcc] + HIPFLAGS + HOST_SANITIZE + inc + ["-c", ASAN_DRIVER_SRC, "-o", dobj])
        aobjs.append(dobj)
    _compile_all(jobs, verbose)
    tmp = LIB + ".tmp%d" % os.getpid()
    _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs, verbose)
    os.replace(tmp, LIB)
    if sanitizer_driver:
        tmpd = ASAN_DRIVER + ".tmp%d" % os.getpid()
        _run([hipcc, "--offload-arch=gfx950"] + HOST_SANITIZE + ["-o", tmpd] + aobjs, verbose)
        os.replace(tmpd, ASAN_DRIVER)
    for o in objs + aobjs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, sanitizer_driver="--no-sanitizer" not in sys.argv))
