"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer on a
real device.  tests/bin/jk_asan_driver (built by tests/sanitize/build_jk_asan.py: the
host translation unit and the driver instrumented, device code as usual) runs FP64,
mixed, deterministic with a kept setup, the allocation-free entry, the single-copy
path with energies and dE/dD (checked in the driver), FP64 at omega = 0.3, the
pure-function transforms (a trace identity checked in the driver) and timing with
statistics, all through the C ABI; any memory or undefined-behaviour error aborts it.
Its J and K are compared with the oracle."""
import os
import subprocess

import numpy as np
import pytest

import oracle
from gpu_util import say
from paper_2406_11185_amd import molgen

pytestmark = pytest.mark.gpu
EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "bin", "jk_asan_driver")
CASES = ["fp64", "mixed", "deterministic, kept setup", "allocation-free", "one copy", "omega 0.3",
         "fp64 again"]


def write_input(path, mol, tol):
    n_dm = mol.D.shape[0]
    with open(path, "wb") as fh:
        np.array([mol.n_atoms, len(mol.shell_l), len(mol.exps), n_dm, mol.n_bf],
                 dtype=np.int32).tofile(fh)
        np.ascontiguousarray(mol.xyz, dtype=np.float64).tofile(fh)
        for a in (mol.shell_atom, mol.shell_l, mol.shell_nprim, mol.shell_prim0):
            np.ascontiguousarray(a, dtype=np.int32).tofile(fh)
        np.ascontiguousarray(mol.exps, dtype=np.float64).tofile(fh)
        np.ascontiguousarray(mol.coefs, dtype=np.float64).tofile(fh)
        np.ascontiguousarray(mol.D, dtype=np.float64).tofile(fh)
        np.array([tol], dtype=np.float64).tofile(fh)


@pytest.mark.skipif(not os.path.exists(EXE),
                    reason="tests/bin/jk_asan_driver is built by tests/sanitize/build_jk_asan.py")
@pytest.mark.parametrize("nh,nH,seed,n_dm,tol", [(4, 5, 5, 1, 1e-8), (2, 2, 11, 3, 0.0)])
def test_host_code_under_sanitizers_on_device(tmp_path, nh, nH, seed, n_dm, tol):
    mol = molgen.make_molecule(nh, nH, seed, n_dm=n_dm)
    say(f"case host ASan/UBSan driver ({mol.n_bf} functions, {n_dm} densities, tol {tol})")
    inp, out = tmp_path / "in.bin", tmp_path / "out.bin"
    write_input(inp, mol, tol)
    env = dict(os.environ, ASAN_OPTIONS="verify_asan_link_order=0:detect_leaks=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([EXE, str(inp), str(out)], capture_output=True, text=True, env=env,
                       timeout=240)
    say(r.stdout.strip(), r.stderr.strip()[-2000:])
    assert r.returncode == 0 and "jk driver ok" in r.stdout
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
    shape = (len(CASES), 2) + mol.D.shape
    res = np.fromfile(out, dtype=np.float64).reshape(shape)
    Jo, Ko, _ = oracle.jk(mol, tol)
    Jw, Kw, _ = oracle.jk(mol, tol, omega=0.3)
    for c, name in enumerate(CASES):
        jo, ko = (Jw, Kw) if name == "omega 0.3" else (Jo, Ko)
        dj, dk = np.abs(res[c, 0] - jo).max(), np.abs(res[c, 1] - ko).max()
        say(f"  {name}: max|dJ|={dj:.2e} max|dK|={dk:.2e}")
        if name == "mixed":
            assert dj <= 1e-6 * np.abs(Jo).max() and dk <= 1e-6 * np.abs(Ko).max()
        else:
            assert dj <= 1e-10 and dk <= 1e-10
