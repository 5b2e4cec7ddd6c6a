"""jk_build_noalloc (static device scratch, no allocation in the call) against
jk_build on the same inputs: two calls in a row, the second on a smaller
molecule, both in deterministic mode (bitwise-comparable sums) and in the
default atomic mode (within 1e-10), then a molecule over the 64 MiB limit."""
import numpy as np
import pytest

from gpu_util import say
from paper_2406_11185_amd import molgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    assert torch.cuda.is_available(), "GPU test without a GPU"


def _both(ctx, mol, tol, **kw):
    import torch
    from paper_2406_11185_amd import jk as jkb
    b = jkb.Basis(mol)
    D = torch.as_tensor(np.ascontiguousarray(mol.D), device="cuda")
    n_dm = D.shape[0]
    J1, K1 = torch.empty_like(D), torch.empty_like(D)
    J2, K2 = torch.full_like(D, 3.0), torch.full_like(D, 3.0)
    E1 = torch.empty((n_dm, 3), dtype=torch.float64, device="cuda")
    E2 = torch.empty_like(E1)
    jkb.jk_build(ctx, b, D, J1, K1, tol, jkb.make_opts(n_dm=n_dm, energy=E1, **kw))
    jkb.jk_build_noalloc(ctx, b, D, J2, K2, tol, jkb.make_opts(n_dm=n_dm, energy=E2, **kw))
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in (J1, K1, E1, J2, K2, E2)]


@pytest.mark.parametrize("det", [1, 0])
def test_noalloc_matches_build_twice(det):
    from paper_2406_11185_amd import jk as jkb
    ctx = jkb.Context(0)
    for mol, tol in [(molgen.make_molecule(4, 5, 5, n_dm=2), 1e-8), (molgen.workload("w4"), 0.0)]:
        say(f"case noalloc det={det} ({mol.n_bf} functions, n_dm={mol.D.shape[0]}, tol {tol})")
        J1, K1, E1, J2, K2, E2 = _both(ctx, mol, tol, deterministic=det)
        say("  max|dJ| =", np.abs(J1 - J2).max(), " max|dK| =", np.abs(K1 - K2).max())
        if det:
            assert np.array_equal(J1, J2) and np.array_equal(K1, K2) and np.array_equal(E1, E2)
        else:
            assert np.abs(J1 - J2).max() <= 1e-10 and np.abs(K1 - K2).max() <= 1e-10
            assert np.abs(E1 - E2).max() <= 1e-10
    ctx.close()


def test_noalloc_rejects_what_does_not_fit():
    import torch
    from paper_2406_11185_amd import jk as jkb
    mol = molgen.workload("w120")
    say(f"case noalloc over the limit ({mol.n_bf} functions)")
    ctx = jkb.Context(0)
    b = jkb.Basis(mol)
    D = torch.as_tensor(mol.D, device="cuda")
    J, K = torch.full_like(D, 5.0), torch.full_like(D, 5.0)
    with pytest.raises(jkb.JkError) as e:
        jkb.jk_build_noalloc(ctx, b, D, J, K, 1e-10, jkb.make_opts())
    assert e.value.code == jkb.JK_ENOMEM and "static scratch" in str(e.value)
    torch.cuda.synchronize()
    assert torch.all(J == 5.0) and torch.all(K == 5.0)
    with pytest.raises(jkb.JkError) as e:
        jkb.jk_build_noalloc(ctx, b, D, J, K, 1e-10, jkb.make_opts(timing=True))
    assert e.value.code == jkb.JK_EUNSUPPORTED
    ctx.close()


def test_noalloc_leaves_the_kept_setup_alone():
    """A jk_build_noalloc call between two reuse_setup builds on one context sets up in
    the static array only: the second build still reuses the kept setup, and all three
    agree bit for bit (deterministic mode)."""
    import torch
    from paper_2406_11185_amd import jk as jkb
    mol = molgen.make_molecule(4, 5, 5)
    say(f"case noalloc between reuse_setup builds ({mol.n_bf} functions, tol 1e-8)")
    ctx = jkb.Context(0)
    b = jkb.Basis(mol)
    D = torch.as_tensor(np.ascontiguousarray(mol.D), device="cuda")
    outs = []
    for call in (jkb.jk_build, jkb.jk_build_noalloc, jkb.jk_build):
        J, K = torch.empty_like(D), torch.empty_like(D)
        call(ctx, b, D, J, K, 1e-8, jkb.make_opts(deterministic=1, reuse_setup=True))
        torch.cuda.synchronize()
        outs.append((J.cpu().numpy(), K.cpu().numpy(), ctx.stats().setup_reused))
    assert outs[0][2] == 0 and outs[2][2] == 1
    for J, K, _ in outs[1:]:
        assert np.array_equal(J, outs[0][0]) and np.array_equal(K, outs[0][1])
    ctx.close()
