"""GPU parity of J/K over pure (spherical) d functions: the library's change of
basis (jk_pure_to_cart, jk_cart_to_pure) around jk_build against the oracle's
pure-function build (each quartet block transformed, then digested)."""
import numpy as np
import pytest

import oracle
from gpu_util import say
from paper_2406_11185_amd import molgen

pytestmark = pytest.mark.gpu
TOL_ABS = 1e-10   # plain FP64 path against the FP64 oracle


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    assert torch.cuda.is_available(), "GPU test without a GPU"
    from paper_2406_11185_amd import jk as jkb
    jkb.load()


def _T(mol):
    """[n_cart][n_pure] from the oracle's pure-d table (expected values only)."""
    C = oracle.pure_d()
    ls = [int(l) for l in mol.shell_l]
    nc = [molgen.ncart(l) for l in ls]
    npu = [5 if l == 2 else molgen.ncart(l) for l in ls]
    T = np.zeros((sum(nc), sum(npu)))
    r = c = 0
    for l, a, b in zip(ls, nc, npu):
        T[r:r + a, c:c + b] = C if l == 2 else np.eye(a)
        r, c = r + a, c + b
    return T


def _pure_density(npu, n_dm, seed):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n_dm, npu, max(2, npu // 4))) / np.sqrt(npu)
    return np.einsum("mik,mjk->mij", X, X)


def test_change_of_basis_matches_the_definition():
    """Both directions against T X T^T and T^T X T, three matrices, a basis whose
    shells alternate s, p, d (ragged contraction lengths)."""
    import torch
    from paper_2406_11185_amd import jk as jkb
    mol = molgen.ragged_molecule(2, 3, 5)
    b = jkb.Basis(mol)
    T = _T(mol)
    n, npu = T.shape
    assert jkb.jk_pure_count(b) == npu and jkb.jk_validate_basis(b) == n
    say(f"case change of basis ({n} Cartesian, {npu} pure functions)")
    rng = np.random.default_rng(3)
    P = rng.normal(size=(3, npu, npu))
    X = rng.normal(size=(3, n, n))
    Pd = torch.as_tensor(P, device="cuda")
    Xd = torch.as_tensor(X, device="cuda")
    out_c = torch.full((3, n, n), 7.0, dtype=torch.float64, device="cuda")
    out_p = torch.full((3, npu, npu), 7.0, dtype=torch.float64, device="cuda")
    jkb.jk_pure_to_cart(b, Pd, out_c)
    jkb.jk_cart_to_pure(b, Xd, out_p)
    torch.cuda.synchronize()
    np.testing.assert_allclose(out_c.cpu().numpy(), np.einsum("ia,mab,jb->mij", T, P, T),
                               rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(out_p.cpu().numpy(), np.einsum("ia,mij,jb->mab", T, X, T),
                               rtol=1e-14, atol=1e-14)


CASES = [("m3_3_21", lambda: molgen.make_molecule(3, 3, 21), 1, 0.0),
         ("m4_5_5", lambda: molgen.make_molecule(4, 5, 5), 2, 1e-8),
         ("ragged", lambda: molgen.ragged_molecule(3, 2, 9), 1, 0.0),
         ("one atom", lambda: molgen.make_molecule(1, 0, 13), 1, 0.0)]


@pytest.mark.parametrize("name,make,n_dm,tol", CASES, ids=[c[0] for c in CASES])
def test_pure_jk_against_oracle(name, make, n_dm, tol):
    import torch
    from paper_2406_11185_amd import jk as jkb
    mol = make()
    npu = jkb.jk_pure_count(jkb.Basis(mol))
    P = _pure_density(npu, n_dm, seed=11)
    say(f"case pure {name} ({npu} pure functions, n_dm {n_dm}, tol {tol})")
    J, K, E, G = jkb.jk(mol, torch.as_tensor(P, device="cuda"), tol, energies=True, dEdD=True,
                        pure=True)
    torch.cuda.synchronize()
    J, K, E, G = (t.cpu().numpy() for t in (J, K, E, G))
    Jo, Ko, _ = oracle.jk(mol, tol, D=P, pure=True)
    say("  max|dJ| =", np.abs(J - Jo).max(), " max|dK| =", np.abs(K - Ko).max())
    assert np.abs(J - Jo).max() <= TOL_ABS and np.abs(K - Ko).max() <= TOL_ABS
    np.testing.assert_allclose(G, Jo - 0.5 * Ko, atol=2 * TOL_ABS)
    E = E.reshape(n_dm, 3)
    for m in range(n_dm):
        EJ, EK = 0.5 * np.sum(P[m] * Jo[m]), 0.25 * np.sum(P[m] * Ko[m])
        assert E[m, 0] == pytest.approx(EJ, rel=1e-11) and E[m, 1] == pytest.approx(EK, rel=1e-11)


def test_pure_w30_sampled_blocks_and_mixed():
    """270-function molecule (258 pure functions): sampled blocks of the FP64 pure
    build against the oracle; the mixed pure build's energies within 1e-6 Eh."""
    import torch
    from paper_2406_11185_amd import jk as jkb
    mol = molgen.workload("w30")
    npu = jkb.jk_pure_count(jkb.Basis(mol))
    P = _pure_density(npu, 1, seed=30)
    Pd = torch.as_tensor(P, device="cuda")
    say(f"case pure w30 ({npu} pure functions, tol 1e-10), sampled blocks + mixed")
    J, K, E = jkb.jk(mol, Pd, 1e-10, energies=True, pure=True)
    Jm, Km, Em = jkb.jk(mol, Pd, 1e-10, precision="mixed", energies=True, pure=True)
    torch.cuda.synchronize()
    J, K, E, Em = J.cpu().numpy(), K.cpu().numpy(), E.cpu().numpy(), Em.cpu().numpy()
    pairs = [(0, 5), (7, 7), (12, 40), (3, 99), (60, 2)]
    bf0 = np.concatenate([[0], np.cumsum([5 if l == 2 else molgen.ncart(int(l))
                                          for l in mol.shell_l])])
    for (m, n), (jb, kb) in zip(pairs, oracle.jk_blocks(mol, 1e-10, pairs, D=P, pure=True)):
        gj = J[:, bf0[m]:bf0[m + 1], bf0[n]:bf0[n + 1]]
        gk = K[:, bf0[m]:bf0[m + 1], bf0[n]:bf0[n + 1]]
        say(f"  block ({m},{n}) dJ={np.abs(gj - jb).max():.2e} dK={np.abs(gk - kb).max():.2e}")
        assert np.abs(gj - jb).max() <= TOL_ABS and np.abs(gk - kb).max() <= TOL_ABS
    say(f"  mixed dEJ={Em[0, 0] - E[0, 0]:.2e} dEK={Em[0, 1] - E[0, 1]:.2e}")
    assert abs(Em[0, 0] - E[0, 0]) <= 1e-6 and abs(Em[0, 1] - E[0, 1]) <= 1e-6


def test_pure_argument_checks():
    import torch
    from paper_2406_11185_amd import jk as jkb
    mol = molgen.make_molecule(1, 1, 7)
    b = jkb.Basis(mol)
    n, npu = jkb.jk_validate_basis(b), jkb.jk_pure_count(b)
    X = torch.zeros((1, npu, npu), dtype=torch.float64, device="cuda")
    Y = torch.full((1, n, n), 7.0, dtype=torch.float64, device="cuda")
    lib = jkb.load()
    import ctypes
    assert lib.jk_pure_to_cart(ctypes.byref(b.c), 0, ctypes.c_void_p(X.data_ptr()),
                               ctypes.c_void_p(Y.data_ptr()), None) == jkb.JK_EINVAL
    assert lib.jk_pure_to_cart(ctypes.byref(b.c), 1, None, ctypes.c_void_p(Y.data_ptr()),
                               None) == jkb.JK_EINVAL
    assert lib.jk_cart_to_pure(None, 1, ctypes.c_void_p(Y.data_ptr()),
                               ctypes.c_void_p(X.data_ptr()), None) == jkb.JK_EINVAL
    torch.cuda.synchronize()
    assert bool((Y == 7.0).all())
