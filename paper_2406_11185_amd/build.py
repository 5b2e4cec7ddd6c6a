"""Build libjk.so for gfx950: generate the per-class code, compile, link.

    python -m paper_2406_11185_amd.build [-j N] [--verbose]

Every HIP translation unit is compiled with hipcc for gfx950 only; object files
and generated sources go to _build/ at the repository root, the shared library
to paper_2406_11185_amd/libjk.so.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import fcntl
import os
import shutil
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
GEN = os.path.join(BUILD, "gen")
OBJ = os.path.join(BUILD, "obj")
LIB = os.path.join(PKG, "libjk.so")
ARCH = "gfx950"

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed FP32 instructions stay off in every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics",
    "-Wno-unused-result",
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.sep not in c or os.path.exists(c)):
            return c
    return "hipcc"


def _inc_of(src: str) -> str:
    """Generated class code of a class translation unit (cls_X.hip and its
    erf(omega r12)/r12 twin cls_X_att.hip both include cls_X.inc)."""
    return src.replace("_att.hip", ".hip").replace(".hip", ".inc")


def _deps_newer(src: str, obj: str) -> bool:
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    deps = [src, _inc_of(src), os.path.join(CSRC, "jk_device.hpp"),
            os.path.join(CSRC, "jk_grad_device.hpp"), os.path.join(CSRC, "jk_classes.hpp"),
            os.path.join(INCLUDE, "jk.h")]
    return any(os.path.exists(d) and os.path.getmtime(d) > t for d in deps)


def _compile(src: str, obj: str, verbose: bool, incremental: bool = False) -> tuple[str, float]:
    if incremental and not _deps_newer(src, obj):
        return src, 0.0
    # the temporary object is private to this build process: a compile left over
    # from an interrupted build can never be renamed into place by another one
    tmp = f"{obj}.{os.getpid()}.tmp"
    cmd = [hipcc(), *HIPCC_FLAGS, "-I", INCLUDE, "-I", CSRC, "-I", GEN, "-c", src, "-o", tmp]
    t = time.time()
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, obj)
    return src, time.time() - t


def build(jobs: int = 0, verbose: bool = False, incremental: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    # one build at a time in this tree (generated sources and objects are shared)
    with open(os.path.join(BUILD, ".lock"), "w") as lock:
        fcntl.flock(lock, fcntl.LOCK_EX)
        return _build_locked(jobs, verbose, incremental)


def _build_locked(jobs: int, verbose: bool, incremental: bool) -> str:
    sys.path.insert(0, CSRC)
    try:
        import gen_hgp  # noqa: E402
        import gen_grad  # noqa: E402
    finally:
        sys.path.pop(0)
    gen_hgp.main(GEN)
    gen_grad.main(GEN)
    shutil.copyfile(os.path.join(GEN, "classes.json"), os.path.join(PKG, "classes.json"))
    shutil.copyfile(os.path.join(GEN, "grad_classes.json"), os.path.join(PKG, "grad_classes.json"))
    sources = [os.path.join(CSRC, "jk_host.hip"), os.path.join(CSRC, "jk_pure.hip"),
               os.path.join(CSRC, "jk_scf.hip"), os.path.join(CSRC, "jk_xc.hip"),
               os.path.join(GEN, "jk_classes_table.hip"),
               os.path.join(GEN, "jk_grad_table.hip")]
    sources += sorted(os.path.join(GEN, f) for f in os.listdir(GEN)
                      if (f.startswith("cls_") or f.startswith("gcls_")) and f.endswith(".hip"))
    # largest classes first so the long compiles start early
    sources.sort(key=lambda p: -os.path.getsize(_inc_of(p)) if os.path.exists(_inc_of(p)) else 0)
    objs = [os.path.join(OBJ, os.path.basename(s).replace(".hip", ".o")) for s in sources]
    jobs = jobs or min(8, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = [ex.submit(_compile, s, o, verbose, incremental) for s, o in zip(sources, objs)]
        for f in cf.as_completed(futs):
            src, dt = f.result()
            if verbose:
                print(f"  {os.path.basename(src)}: {dt:.1f}s", flush=True)
    tmp = f"{LIB}.{os.getpid()}.tmp"
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs,
           "-L/opt/rocm/lib", "-lrocsolver", "-lrocblas", "-Wl,-rpath,/opt/rocm/lib"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", type=int, default=0)
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--incremental", action="store_true",
                    help="recompile only sources newer than their objects")
    a = ap.parse_args()
    t = time.time()
    print(build(a.j, a.verbose, a.incremental), f"({time.time() - t:.1f}s)")
