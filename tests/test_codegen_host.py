"""The generated per-class integral code, compiled for the host with g++, against the
oracle: every energy class on shells of the 4-atom workload, and the full nuclear
gradient of two small molecules.  The recurrence coefficients and the Boys function
in these harnesses are computed directly from their definitions, so a failure here
points at the code generators, not at the device-side setup."""
import ctypes
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
from paper_2406_11185_amd import molgen

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2406_11185_amd", "csrc")
PC = {(0, 0): 0, (1, 0): 1, (1, 1): 2, (2, 0): 3, (2, 1): 4, (2, 2): 5}
dp = ctypes.POINTER(ctypes.c_double)
ip = ctypes.POINTER(ctypes.c_int)


@pytest.fixture(scope="module")
def libs(tmp_path_factory):
    gen = str(tmp_path_factory.mktemp("gen"))
    sys.path.insert(0, CSRC)
    try:
        import gen_grad
        import gen_hgp
    finally:
        sys.path.pop(0)
    gen_hgp.main(gen)
    gen_grad.main(gen)
    out = {}
    procs = []
    for name in ("emu_eri", "emu_grad"):
        so = os.path.join(gen, f"lib{name}.so")
        procs.append((name, so, subprocess.Popen(
            ["g++", "-O0", "-std=c++17", "-fPIC", "-shared", "-D__device__=", "-D_GLIBCXX_ASSERTIONS", "-I", gen, "-o", so,
             os.path.join(HERE, "emu", f"{name}.cpp")], stderr=subprocess.PIPE)))
    for name, so, p in procs:
        _, err = p.communicate()
        assert p.returncode == 0, err.decode()[-2000:]
        out[name] = ctypes.CDLL(so)
    return out


def _p(a, t):
    return a.ctypes.data_as(t)


@pytest.mark.parametrize("entry", ["emu_block", "emu_block32"])
def test_every_energy_class_matches_oracle(libs, entry):
    """Every class (emu_block32: the FP32 layouts of the multi-pass classes,
    evaluated in double precision) against the oracle."""
    lib = libs["emu_eri"]
    fn = getattr(lib, entry)
    mol = molgen.workload("w4")
    b = oracle.Basis(mol)
    ls = mol.shell_l
    inv = {v: k for k, v in PC.items()}

    def pick(la, lb, avoid=None):
        for i in range(mol.n_shells):
            for j in range(mol.n_shells):
                if ls[i] == la and ls[j] == lb and mol.shell_atom[i] != mol.shell_atom[j] \
                        and (i, j) != avoid:
                    return i, j
        raise AssertionError
    q = 0
    for X in range(6):
        for Y in range(X + 1):
            (la, lb), (lc, ld) = inv[X], inv[Y]
            A, B = pick(la, lb)
            C, D = pick(lc, ld, avoid=(A, B))
            sh = [A, B, C, D]
            l = np.array([ls[s] for s in sh], np.int32)
            npr = np.full(4, 3, np.int32)
            cen = np.ascontiguousarray([mol.xyz[mol.shell_atom[s]] for s in sh]).ravel()
            e = np.zeros(32)
            c = np.zeros(32)
            for k, s in enumerate(sh):
                p0 = mol.shell_prim0[s]
                e[8 * k:8 * k + 3] = mol.exps[p0:p0 + 3]
                c[8 * k:8 * k + 3] = mol.coefs[p0:p0 + 3]
            ref = oracle.shell_quartet(b, *sh).ravel()
            out = np.zeros(ref.size)
            rc = fn(q, _p(l, ip), _p(npr, ip), _p(cen, dp), _p(e, dp), _p(c, dp), _p(out, dp))
            if entry == "emu_block32" and rc == -1:   # no separate FP32 layout
                q += 1
                continue
            assert rc == 0
            assert np.abs(out - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max()), (q, sh)
            q += 1


@pytest.mark.parametrize("nh,nH,seed", [(1, 1, 7), (0, 3, 3)])
def test_gradient_classes_match_oracle(libs, nh, nH, seed):
    lib = libs["emu_grad"]
    mol = molgen.make_molecule(nh, nH, seed, heavy_z=None if nh else [])
    l = mol.shell_l.astype(np.int32)
    at = mol.shell_atom.astype(np.int32)
    p0 = mol.shell_prim0.astype(np.int32)
    npr = mol.shell_nprim.astype(np.int32)
    D = np.ascontiguousarray(mol.D[0])
    g = np.zeros((mol.n_atoms, 3))
    lib.emu_grad(mol.n_shells, _p(l, ip), _p(at, ip), _p(np.ascontiguousarray(mol.xyz), dp),
                 _p(mol.exps, dp), _p(mol.coefs, dp), _p(p0, ip), _p(npr, ip), _p(D, dp), mol.n_bf,
                 _p(g, dp))
    go = oracle.grad(mol, 0.0)[0]
    assert np.abs(g - go).max() <= 1e-11


def test_digestion_sweeps_equal_one_sweep(libs):
    """Every single-pass class: the five generated digestion sweeps (one J/K
    block each) give the blocks of the one-sweep digestion."""
    lib = libs["emu_eri"]
    lib.emu_sweeps.restype = ctypes.c_double
    for q in range(21):
        d = lib.emu_sweeps(q)
        assert 0.0 <= d <= 1e-14, (q, d)
