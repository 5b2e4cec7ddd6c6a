"""Every compiled class kernel takes its launch structure with the size the host
code lays it out with (metadata of the gfx950 code objects in _build/obj against
sizeof on the host): an object compiled from other headers than the host code
would read garbage pointers."""
import os

import pytest

from paper_2406_11185_amd import kernel_resources as kr

OBJ = kr.OBJ


@pytest.mark.skipif(not os.path.isdir(OBJ), reason="library not built (_build/obj missing)")
def test_kernel_arguments_match_host_layout():
    eri, grad = kr.host_arg_sizes()
    n = 0
    for f in sorted(os.listdir(OBJ)):
        if not f.endswith(".o"):
            continue
        for r in kr.kernels_of(os.path.join(OBJ, f)):
            name = r["name"]
            if "grad_kernel" in name:
                assert r["arg0"] == grad, (f, name, r["arg0"], grad)
            elif "eri_jk" in name or "schwarz" in name:
                assert r["arg0"] == eri, (f, name, r["arg0"], eri)
            else:
                continue
            n += 1
    assert n > 100
