"""Build libcq.so (HIP, gfx950) in-tree.

Steps: generate the per-class electron-repulsion kernels (csrc/gen_eri.py ->
csrc/gen/eri_<class>.hip + eri_registry.hpp), compile every translation unit
with hipcc in parallel, and link them into paper_1905_01381_amd/libcq.so.
FP64 atomics are compiled to the hardware instruction (-munsafe-fp-atomics);
packed-FP32 instruction selection is disabled.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
GEN = os.path.join(CSRC, "gen")
OBJ = os.path.join(ROOT, "_build", "obj")
LIB = os.path.join(HERE, "libcq.so")
ARCH = os.environ.get("CQ_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
    "-munsafe-fp-atomics",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-variable", "-Wno-unused-but-set-variable",
]


def generate(verbose: bool = False) -> list[str]:
    cmd = [sys.executable, os.path.join(CSRC, "gen_eri.py"), GEN]
    subprocess.run(cmd, check=True, stderr=None if verbose else subprocess.DEVNULL)
    return sorted(glob.glob(os.path.join(GEN, "eri_*.hip")))


def _headers() -> list[str]:
    return (glob.glob(os.path.join(CSRC, "*.hpp")) + glob.glob(os.path.join(GEN, "*.hpp"))
            + [os.path.join(ROOT, "include", "cq.h"), __file__])


def _fresh(src: str, obj: str) -> bool:
    if not os.path.exists(obj):
        return False
    t = os.path.getmtime(obj)
    deps = _headers()
    if os.path.basename(src).startswith("eri_"):
        # generated class kernels include eri_common.hpp only, not the registry
        deps = [d for d in deps if not d.startswith(GEN)]
    return all(os.path.getmtime(x) <= t for x in [src, *deps])


def _compile(src: str, extra: list[str], incremental: bool = False) -> tuple[str, str]:
    obj = os.path.join(OBJ, os.path.basename(src).replace(".hip", ".o"))
    if incremental and _fresh(src, obj):
        return obj, ""
    tmp = obj + f".tmp{os.getpid()}"
    cmd = ["hipcc", *HIPCC_FLAGS, *extra, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-I", GEN,
           "-c", src, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, obj)
    return obj, r.stderr


def build(verbose: bool = False, extra: list[str] | None = None, jobs: int | None = None,
          incremental: bool = False) -> str:
    """Compile every translation unit (always, unless ``incremental``, which
    skips objects newer than their sources and headers) and link libcq.so."""
    t0 = time.time()
    extra = extra or []
    os.makedirs(OBJ, exist_ok=True)
    srcs = generate(verbose) + [os.path.join(CSRC, "cq_api.hip"), os.path.join(CSRC, "one_electron.hip"),
                                 os.path.join(CSRC, "rt.hip"), os.path.join(CSRC, "eri_hl.hip")]
    jobs = jobs or min(len(srcs), max(1, min(16, os.cpu_count() or 1)))
    objs, logs = [], []
    with cf.ThreadPoolExecutor(jobs) as ex:
        for obj, log in ex.map(lambda s: _compile(s, extra, incremental), srcs):
            objs.append(obj)
            logs.append(log)
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    if verbose:
        for log in logs:
            if log.strip():
                print(log)
        print(f"built {LIB} in {time.time() - t0:.1f}s", flush=True)
    return LIB


if __name__ == "__main__":
    args = sys.argv[1:]
    inc = "--incremental" in args
    args = [a for a in args if a != "--incremental"]
    build(verbose=True, extra=args, incremental=inc)
