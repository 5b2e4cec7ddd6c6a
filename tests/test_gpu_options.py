"""GPU checks of the library's options against the CPU oracle: energies and
dE/dD from the finalize step, the single-copy (in-place) accumulation path,
deterministic mode, serial launches, multi-density gradients, and the FP32
Boys evaluation at the lowest accepted FP64 switch-over."""
import numpy as np
import pytest

import oracle
from gpu_util import GRAD_OFF, say
from paper_2406_11185_amd import molgen

pytestmark = pytest.mark.gpu
TOL_ABS = 1e-10


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    assert torch.cuda.is_available(), "GPU test without a GPU"


def _dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


def _run(mol, tol, **kw):
    import torch
    from paper_2406_11185_amd import jk as jkb
    out = jkb.jk(mol, _dev(mol.D), tol, **kw)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in out]


def test_energies_and_dEdD_from_the_library():
    mol = molgen.make_molecule(2, 2, 11, n_dm=3)
    say(f"case energies + dE/dD, n_dm=3 ({mol.n_bf} functions, tol 0)")
    J, K, E, G = _run(mol, 0.0, energies=True, dEdD=True)
    Jo, Ko, _ = oracle.jk(mol, 0.0)
    EJo, EKo = oracle.energy(Jo, Ko, mol.D)
    say("  dEJ", np.abs(E[:, 0] - EJo).max(), "dEK", np.abs(E[:, 1] - EKo).max())
    assert np.abs(E[:, 0] - EJo).max() <= 1e-10 and np.abs(E[:, 1] - EKo).max() <= 1e-10
    assert np.abs(E[:, 2] - (EJo - EKo)).max() <= 1e-10
    assert np.abs(G - (Jo - 0.5 * Ko)).max() <= TOL_ABS
    assert np.abs(J - Jo).max() <= TOL_ABS and np.abs(K - Ko).max() <= TOL_ABS


@pytest.mark.parametrize("n_dm", [1, 3])
def test_single_copy_in_place_accumulation(n_dm):
    """acc_copies = 1: J and K are the accumulators and the finalize works in place
    (the path large matrices take, e.g. 1800 functions with 10 densities)."""
    mol = molgen.make_molecule(3, 3, 21, n_dm=n_dm)
    say(f"case single accumulator copy, n_dm={n_dm} ({mol.n_bf} functions, tol 1e-8)")
    J, K, E = _run(mol, 1e-8, acc_copies=1, energies=True)
    Jo, Ko, _ = oracle.jk(mol, 1e-8)
    say("  max|dJ| =", np.abs(J - Jo).max(), " max|dK| =", np.abs(K - Ko).max())
    assert np.abs(J - Jo).max() <= TOL_ABS and np.abs(K - Ko).max() <= TOL_ABS
    EJo, EKo = oracle.energy(Jo, Ko, mol.D)
    assert np.abs(E[:, 0] - EJo).max() <= 1e-10 and np.abs(E[:, 1] - EKo).max() <= 1e-10


@pytest.mark.parametrize("copies", [0, 1])
def test_deterministic_mode_is_bitwise_stable(copies):
    mol = molgen.make_molecule(3, 3, 21, n_dm=2)
    say(f"case deterministic, acc_copies={copies} ({mol.n_bf} functions, tol 0)")
    J1, K1 = _run(mol, 0.0, deterministic=1, acc_copies=copies)
    J2, K2 = _run(mol, 0.0, deterministic=1, acc_copies=copies)
    assert np.array_equal(J1, J2) and np.array_equal(K1, K2)
    Ja, Ka = _run(mol, 0.0)
    say("  vs atomic mode: max|dJ| =", np.abs(J1 - Ja).max(), " max|dK| =", np.abs(K1 - Ka).max())
    assert np.abs(J1 - Ja).max() <= 1e-13 * max(1.0, np.abs(Ja).max())
    assert np.abs(K1 - Ka).max() <= 1e-13 * max(1.0, np.abs(Ka).max())
    Jo, Ko, _ = oracle.jk(mol, 0.0)
    assert np.abs(J1 - Jo).max() <= TOL_ABS and np.abs(K1 - Ko).max() <= TOL_ABS


def test_deterministic_multipass_classes_and_mixed():
    """Deterministic mode through the multi-pass (dd-containing) kernels and the
    FP32 kernels: two runs agree bitwise."""
    mol = molgen.workload("w30")
    say("case deterministic w30 mixed (270 functions, tol 1e-10)")
    J1, K1 = _run(mol, 1e-10, precision="mixed", deterministic=1)
    J2, K2 = _run(mol, 1e-10, precision="mixed", deterministic=1)
    assert np.array_equal(J1, J2) and np.array_equal(K1, K2)


def test_serial_launches_match_streams():
    mol = molgen.make_molecule(4, 5, 5)
    say(f"case serial launches ({mol.n_bf} functions, tol 1e-8)")
    J1, K1 = _run(mol, 1e-8, serial=True)
    J2, K2 = _run(mol, 1e-8)
    assert np.abs(J1 - J2).max() <= 1e-13 and np.abs(K1 - K2).max() <= 1e-13


@GRAD_OFF
def test_gradient_multiple_densities_and_deterministic():
    import torch
    from paper_2406_11185_amd import jk as jkb
    mol = molgen.make_molecule(2, 2, 11, n_dm=3)
    say(f"case grad n_dm=3, atomic and deterministic ({mol.n_bf} functions, tol 0)")
    D = _dev(mol.D)
    G = jkb.grad(mol, D, 0.0).cpu().numpy()
    Gd1 = jkb.grad(mol, D, 0.0, deterministic=1).cpu().numpy()
    Gd2 = jkb.grad(mol, D, 0.0, deterministic=1).cpu().numpy()
    torch.cuda.synchronize()
    Go = oracle.grad(mol, 0.0)
    say("  max|dG| =", np.abs(G - Go).max(), " det:", np.abs(Gd1 - Go).max())
    assert G.shape == (3, mol.n_atoms, 3)
    assert np.abs(G - Go).max() <= 1e-9 and np.abs(Gd1 - Go).max() <= 1e-9
    assert np.array_equal(Gd1, Gd2)


def test_fp32_boys_at_lowest_switch_over():
    """boys_fp64_T close to its lower limit: nearly every Boys value of the FP32
    kernels comes from the FP64 evaluation, which is valid at any T."""
    mol = molgen.make_molecule(3, 3, 21)
    say(f"case mixed, all FP32, boys_fp64_T=1e-3 ({mol.n_bf} functions)")
    J, K = _run(mol, 0.0, precision="mixed", fp32_below=1e9, boys_fp64_T=1e-3)
    Jo, Ko, _ = oracle.jk(mol, 0.0)
    say("  max|dJ| =", np.abs(J - Jo).max(), " max|dK| =", np.abs(K - Ko).max())
    assert np.abs(J - Jo).max() <= 1e-6 * np.abs(Jo).max()
    assert np.abs(K - Ko).max() <= 1e-6 * np.abs(Ko).max()


def test_setup_reuse_across_calls():
    """reuse_setup = 1: a second call with the same basis, tol and precision keeps
    the pair data, bounds and work items of the first (stats.setup_reused) and,
    with another D, gives J and K bit for bit equal to a fresh context's
    (deterministic mode) and within the oracle bound; a changed tol or exponent,
    or a call without the option, sets up again."""
    import torch
    from paper_2406_11185_amd import jk as jkb
    mol = molgen.make_molecule(3, 3, 21, n_dm=1)
    say(f"case setup reuse ({mol.n_bf} functions, tol 1e-8)")
    rng = np.random.default_rng(7)
    X = rng.standard_normal(mol.D.shape[1:]) * 0.05
    D2h = mol.D * 0.5 + (X + X.T)[None]
    basis = jkb.Basis(mol)
    D1, D2 = _dev(mol.D), _dev(D2h)
    J, K = torch.empty_like(D1), torch.empty_like(D1)

    def build(ctx, D, tol, reuse, b=basis):
        o = jkb.make_opts("fp64", deterministic=1, reuse_setup=reuse)
        jkb.jk_build(ctx, b, D, J, K, tol, o)
        torch.cuda.synchronize()
        return J.cpu().numpy(), K.cpu().numpy(), ctx.stats().setup_reused

    ctx = jkb.Context(0)
    assert build(ctx, D1, 1e-8, True)[2] == 0
    J2, K2, reused = build(ctx, D2, 1e-8, True)
    assert reused == 1
    J2f, K2f, r = build(jkb.Context(0), D2, 1e-8, False)
    assert r == 0 and np.array_equal(J2, J2f) and np.array_equal(K2, K2f)
    mol2 = molgen.Molecule(**{**mol.__dict__, "D": D2h})
    Jo, Ko, _ = oracle.jk(mol2, 1e-8)
    assert np.abs(J2 - Jo).max() <= TOL_ABS and np.abs(K2 - Ko).max() <= TOL_ABS
    assert build(ctx, D2, 1e-9, True)[2] == 0          # tol changed
    assert build(ctx, D2, 1e-9, True)[2] == 1
    mol3 = molgen.Molecule(**{**mol.__dict__, "exps": mol.exps * 1.01})
    assert build(ctx, D2, 1e-9, True, jkb.Basis(mol3))[2] == 0   # an exponent changed
    assert build(ctx, D2, 1e-9, False)[2] == 0         # no reuse asked: set up again
    assert build(ctx, D2, 1e-9, True)[2] == 0          # ... which replaced the kept setup


def test_largest_density_count():
    """n_dm = 16, the most the library accepts (JK_MAX_NDM), against the oracle; the
    mixed path with every quartet in FP32 takes the per-density row-buffer launches."""
    mol = molgen.make_molecule(2, 2, 11, n_dm=16)
    say(f"case 16 densities ({mol.n_bf} functions, tol 0)")
    J, K = _run(mol, 0.0)
    Jo, Ko, _ = oracle.jk(mol, 0.0)
    say("  max|dJ| =", np.abs(J - Jo).max(), " max|dK| =", np.abs(K - Ko).max())
    assert np.abs(J - Jo).max() <= TOL_ABS and np.abs(K - Ko).max() <= TOL_ABS
    J, K = _run(mol, 0.0, precision="mixed", fp32_below=1e9)
    assert np.abs(J - Jo).max() <= 1e-6 * np.abs(Jo).max()
    assert np.abs(K - Ko).max() <= 1e-6 * np.abs(Ko).max()
