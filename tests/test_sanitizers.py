"""Host-side sanitizer runs (CPU only).

The CPU oracle, built with AddressSanitizer and UndefinedBehaviorSanitizer, runs
every entry point once on a small s/p/d basis (tests/sanitize/oracle_driver.cpp);
any out-of-bounds access, use after free, leak or undefined behaviour aborts it.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    exe = tmp_path / "oracle_asan"
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fopenmp", *SAN, "-o", str(exe),
                    os.path.join(ROOT, "oracle", "md_oracle.cpp"),
                    os.path.join(HERE, "sanitize", "oracle_driver.cpp")], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="2")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    assert "oracle driver ok" in r.stdout


HIPCC = "/opt/rocm/bin/hipcc"
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
            "-Xarch_host", "-fsanitize-ignorelist=" + os.path.join(HERE, "sanitize", "ubsan_ignore.txt")]


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="needs hipcc")
def test_host_library_under_address_and_undefined_sanitizers(tmp_path):
    """The library's host translation unit with host-side ASan/UBSan (the gfx950
    device code is built as usual and never runs here): option defaults, every
    basis-validation rule, NULL handles and context creation without a device
    (tests/sanitize/host_driver.cpp)."""
    pkg = os.path.join(ROOT, "paper_2406_11185_amd")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(pkg, "csrc")]
    common = ["-O1", "-g", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature",
              "-Xclang", "-packed-fp32-ops", *HOST_SAN, *inc]
    objs = []
    for src, kind in ((os.path.join(pkg, "csrc", "jk_host.hip"), []),
                      (os.path.join(HERE, "sanitize", "host_driver.cpp"), ["-x", "hip"])):
        obj = tmp_path / (os.path.basename(src) + ".o")
        subprocess.run([HIPCC, *common, *kind, "-c", src, "-o", str(obj)], check=True,
                       capture_output=True)
        objs.append(str(obj))
    exe = tmp_path / "host_asan"
    link = [HIPCC, "--offload-arch=gfx950", "-fno-gpu-sanitize", "-fsanitize=address,undefined"]
    subprocess.run([*link, *objs, "-o", str(exe)], check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    assert "host driver ok" in r.stdout
