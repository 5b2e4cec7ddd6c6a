"""The scratch guard's decision (csrc/jk_guard.hpp), compiled for the host with g++."""
import ctypes
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2406_11185_amd", "csrc")

SRC = r'''
#include "jk_guard.hpp"
extern "C" unsigned long long need(unsigned long long p, unsigned long long w, unsigned long long cu,
                                   unsigned long long b, unsigned long long wpb) {
  return jk::launch_scratch_bytes(p, w, cu, b, wpb);
}
extern "C" int ok(unsigned long long need) { return jk::launch_scratch_ok(need) ? 1 : 0; }
extern "C" unsigned long long budget() { return jk::kScratchBudget; }
'''


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    d = tmp_path_factory.mktemp("guard")
    src = d / "g.cpp"
    src.write_text(SRC)
    so = d / "libg.so"
    subprocess.run(["g++", "-O1", "-std=c++17", "-fPIC", "-shared", "-I", CSRC, "-o", str(so),
                    str(src)], check=True)
    L = ctypes.CDLL(str(so))
    u = ctypes.c_ulonglong
    L.need.restype = u
    L.need.argtypes = [u] * 5
    L.ok.argtypes = [u]
    L.budget.restype = u
    return L


def test_no_scratch_always_fits(lib):
    assert lib.need(0, 10**6, 256, 2, 4) == 0 and lib.ok(0) == 1


def test_resident_waves_cap_the_need(lib):
    # 1000 bytes per lane; 256 CUs x 1 workgroup x 4 waves resident = 1024 waves
    assert lib.need(1000, 10**6, 256, 1, 4) == 1000 * 64 * 1024
    # fewer waves launched than can be resident
    assert lib.need(1000, 100, 256, 1, 4) == 1000 * 64 * 100


def test_budget_separates_the_measured_cases(lib):
    # kernels of 7920 and 10464 private bytes per lane at one wavefront per SIMD on
    # 256 CUs (1024 resident waves): the first ran, the second aborted the queue
    ran = lib.need(7920, 10**5, 256, 1, 4)
    aborted = lib.need(10464, 10**5, 256, 1, 4)
    assert lib.ok(ran) == 1 and lib.ok(aborted) == 0
    assert lib.ok(lib.budget()) == 1 and lib.ok(lib.budget() + 1) == 0
