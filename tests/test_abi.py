"""Host-only checks of the C ABI: the library loads, exports what jk.h declares,
and rejects bad arguments before touching a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2406_11185_amd import jk as jkb
from paper_2406_11185_amd import molgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "jk.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(jk_[a-z_]+)\s*\(", text)))


def test_header_declares_the_binding_names():
    assert declared_functions() == sorted(jkb.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = jkb.load()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_opts_default():
    o = jkb.jk_opts_default()
    assert o.precision == jkb.JK_FP64 and o.n_dm == 1 and o.fp32_below == 1e-4
    assert o.boys_fp64_T == 30.0 and o.deterministic == 0 and o.max_scratch_bytes == 0
    assert o.acc_copies == 0 and o.serial == 0 and o.reuse_setup == 0
    assert not o.energy and not o.dEdD and o.omega == 0.0
    assert jkb.load().jk_opts_default(None) == jkb.JK_EINVAL


def test_struct_layouts_match_the_header(tmp_path):
    """Size and field offsets of the binding's ctypes structures equal what a C
    compiler makes of include/jk.h."""
    import json
    import subprocess
    structs = (jkb.jk_basis, jkb.jk_opts, jkb.jk_stats)
    body = []
    for st in structs:
        name = st.__name__
        body.append(f'printf("\\"{name}\\": [%zu", sizeof({name}));')
        for f, _ in st._fields_:
            body.append(f'printf(", %zu", offsetof({name}, {f}));')
        body.append('printf("]%s", ' + ('"\\n"' if st is structs[-1] else '", "') + ');')
    src = tmp_path / "layout.c"
    src.write_text("#include <stddef.h>\n#include <stdio.h>\n#include \"jk.h\"\nint main(void) {\n"
                   'printf("{");\n' + "\n".join(body) + '\nprintf("}\\n");\nreturn 0;\n}\n')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)],
                   check=True)
    got = json.loads(subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout)
    for st in structs:
        want = [ctypes.sizeof(st)] + [getattr(st, f).offset for f, _ in st._fields_]
        assert got[st.__name__] == want, st.__name__


def test_validate_basis_counts_functions():
    for w in ("w4", "w30"):
        mol = molgen.workload(w)
        assert jkb.jk_validate_basis(jkb.Basis(mol)) == mol.n_bf


def _mutated(**kw):
    mol = molgen.workload("w4")
    fields = dict(xyz=mol.xyz.copy(), Z=mol.Z, shell_atom=mol.shell_atom.copy(),
                  shell_l=mol.shell_l.copy(), shell_nprim=mol.shell_nprim.copy(),
                  shell_prim0=mol.shell_prim0.copy(), exps=mol.exps.copy(),
                  coefs=mol.coefs.copy())
    for k, f in kw.items():
        f(fields[k])
    return molgen.Molecule(**fields)


@pytest.mark.parametrize("mut,code", [
    (dict(shell_l=lambda a: a.__setitem__(5, 3)), jkb.JK_EUNSUPPORTED),
    (dict(shell_l=lambda a: a.__setitem__(0, -1)), jkb.JK_EINVAL),
    (dict(shell_nprim=lambda a: a.__setitem__(2, 0)), jkb.JK_EINVAL),
    (dict(shell_nprim=lambda a: a.__setitem__(2, 9)), jkb.JK_EUNSUPPORTED),
    (dict(exps=lambda a: a.__setitem__(4, -0.3)), jkb.JK_EINVAL),
    (dict(exps=lambda a: a.__setitem__(4, 0.0)), jkb.JK_EINVAL),
    (dict(coefs=lambda a: a.__setitem__(1, np.nan)), jkb.JK_EINVAL),
    (dict(shell_atom=lambda a: a.__setitem__(0, 7)), jkb.JK_EINVAL),
    (dict(xyz=lambda a: a.__setitem__((1, 2), np.inf)), jkb.JK_EINVAL),
])
def test_validate_basis_rejects(mut, code):
    b = jkb.Basis(_mutated(**mut))
    with pytest.raises(jkb.JkError) as e:
        jkb.jk_validate_basis(b)
    assert e.value.code == code


def test_null_arguments():
    lib = jkb.load()
    assert lib.jk_validate_basis(None, None) == jkb.JK_EINVAL
    assert lib.jk_build(None, None, None, None, None, 0.0, None, None) == jkb.JK_EINVAL
    assert lib.jk_grad(None, None, None, None, 0.0, None, None) == jkb.JK_EINVAL
    assert lib.jk_get_stats(None, None) == jkb.JK_EINVAL
    assert lib.jk_ctx_destroy(None) == jkb.JK_OK
    assert lib.jk_ctx_create(None, 0) == jkb.JK_EINVAL
    b = jkb.Basis(molgen.workload("w4"))
    b.c.n_shells = 0
    assert lib.jk_validate_basis(ctypes.byref(b.c), None) == jkb.JK_EINVAL


def test_pure_count_on_the_host():
    """jk_pure_count: 2l + 1 functions per shell, a bad basis rejected (no GPU)."""
    for w in ("w4", "w30"):
        mol = molgen.workload(w)
        want = int(sum(2 * int(l) + 1 for l in mol.shell_l))
        assert jkb.jk_pure_count(jkb.Basis(mol)) == want
    assert jkb.load().jk_pure_count(None, None) == jkb.JK_EINVAL
