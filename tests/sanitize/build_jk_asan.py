"""Build tests/bin/jk_asan_driver: the library's host translation units (jk_host.hip,
jk_pure.hip) and the driver
(tests/sanitize/jk_driver.cpp) with host-side AddressSanitizer and
UndefinedBehaviorSanitizer, linked with the per-class objects of the regular build
(_build/obj, so run `python -m paper_2406_11185_amd.build` first).  Device code is
compiled as usual; only host code is instrumented.

    python tests/sanitize/build_jk_asan.py
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
HIPCC = "/opt/rocm/bin/hipcc"
OBJ = os.path.join(ROOT, "_build", "obj")
OUT = os.path.join(ROOT, "tests", "bin", "jk_asan_driver")
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
            "-Xarch_host", "-fsanitize-ignorelist=" + os.path.join(HERE, "ubsan_ignore.txt")]


def build() -> str:
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2406_11185_amd", "csrc"),
           "-I", os.path.join(ROOT, "_build", "gen")]
    common = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-munsafe-fp-atomics",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *HOST_SAN, *inc]
    objs = []
    for src, extra in ((os.path.join(ROOT, "paper_2406_11185_amd", "csrc", "jk_host.hip"), []),
                       (os.path.join(ROOT, "paper_2406_11185_amd", "csrc", "jk_pure.hip"), []),
                       (os.path.join(HERE, "jk_driver.cpp"), ["-x", "hip"])):
        obj = os.path.join(os.path.dirname(OUT), os.path.basename(src) + ".asan.o")
        subprocess.run([HIPCC, *common, *extra, "-c", src, "-o", obj], check=True)
        objs.append(obj)
    others = sorted(os.path.join(OBJ, f) for f in os.listdir(OBJ)
                    if f.endswith(".o") and f not in ("jk_host.o", "jk_pure.o"))
    link = [HIPCC, "--offload-arch=gfx950", "-fno-gpu-sanitize", "-fsanitize=address,undefined",
            "-L/opt/rocm/lib", "-lrocsolver", "-lrocblas", "-Wl,-rpath,/opt/rocm/lib"]
    subprocess.run([*link, *objs, *others, "-o", OUT], check=True)
    for o in objs:
        os.remove(o)
    return OUT


if __name__ == "__main__":
    print(build())
    sys.exit(0)
