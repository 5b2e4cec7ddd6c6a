"""Mixed FP32/FP64 dispatch: FP32 integrals where Q_AB*Q_CD < fp32_below, FP64
otherwise, FP64 accumulation.  The mixed path is an approximation of the exact
result, so parity is stated as error bounds against FP64: |dE_J|, |dE_K| <= 1e-6
hartree, with the largest element errors printed."""
import numpy as np
import pytest

import oracle
from gpu_util import gpu_jk, say
from paper_2406_11185_amd import molgen

pytestmark = pytest.mark.gpu


def energies(J, K, D):
    return 0.5 * float(np.sum(D * J)), 0.25 * float(np.sum(D * K))


def test_small_mixed_against_oracle():
    """Every quartet in FP32 (threshold above every bound) against the oracle.  This is
    outside the dispatcher's envelope (bounds up to 1 in FP32), so the bound is relative:
    FP32 rounding of O(1) integrals, 1e-7 of the energies and 1e-6 of the largest element."""
    import torch
    from paper_2406_11185_amd import jk as jkb
    mol = molgen.make_molecule(3, 3, 21)
    say(f"case mixed m3_3_21 ({mol.n_bf} functions), all FP32")
    D = torch.as_tensor(mol.D, device="cuda")
    J, K = jkb.jk(mol, D, 0.0, precision="mixed", fp32_below=1e9)
    st = jkb.default_context(0).stats()
    assert sum(st.quartets_fp64) == 0 and sum(st.quartets_fp32) == 378 * 379 // 2
    J, K = J.cpu().numpy(), K.cpu().numpy()
    Jo, Ko, _ = oracle.jk(mol, 0.0)
    EJ, EK = energies(J[0], K[0], mol.D[0])
    EJo, EKo = energies(Jo[0], Ko[0], mol.D[0])
    say(f"  dEJ={EJ - EJo:.2e} dEK={EK - EKo:.2e} max|dJ|={np.abs(J - Jo).max():.2e} "
        f"max|dK|={np.abs(K - Ko).max():.2e}")
    assert abs(EJ - EJo) <= 1e-7 * abs(EJo) and abs(EK - EKo) <= 1e-7 * abs(EKo)
    assert np.abs(J - Jo).max() <= 1e-6 * np.abs(Jo).max()
    assert np.abs(K - Ko).max() <= 1e-6 * np.abs(Ko).max()


@pytest.mark.parametrize("name", ["w30", "w120"])
def test_mixed_against_fp64(name):
    from paper_2406_11185_amd import jk as jkb
    mol = molgen.workload(name)
    say(f"case mixed vs fp64 {name} ({mol.n_bf} functions, tol 1e-10, FP32 below 1e-4)")
    J64, K64 = gpu_jk(mol, 1e-10, "fp64")
    Jm, Km = gpu_jk(mol, 1e-10, "mixed")
    st = jkb.default_context(0).stats()
    n32, n64 = sum(st.quartets_fp32), sum(st.quartets_fp64)
    EJ64, EK64 = energies(J64[0], K64[0], mol.D[0])
    EJm, EKm = energies(Jm[0], Km[0], mol.D[0])
    say(f"  FP32 share {n32 / (n32 + n64):.3f}  dEJ={EJm - EJ64:.2e} dEK={EKm - EK64:.2e} "
        f"max|dJ|={np.abs(Jm - J64).max():.2e} max|dK|={np.abs(Km - K64).max():.2e}")
    assert n32 > n64
    assert abs(EJm - EJ64) <= 1e-6 and abs(EKm - EK64) <= 1e-6
    np.testing.assert_allclose(Jm, Jm.transpose(0, 2, 1), atol=1e-13)


def test_mixed_several_densities_match_one_at_a_time():
    """Several densities in FP32: the light classes take the LDS row buffer once per
    density (integrals recomputed for each); every density must equal its own
    one-density build (up to the order of FP64 atomic adds) and the oracle within
    the all-FP32 bounds above."""
    import torch
    from paper_2406_11185_amd import jk as jkb
    mol = molgen.make_molecule(3, 3, 21, n_dm=3)
    say(f"case mixed, 3 densities ({mol.n_bf} functions), all FP32")
    D = torch.as_tensor(mol.D, device="cuda")
    J, K = jkb.jk(mol, D, 0.0, precision="mixed", fp32_below=1e9)
    J, K = J.cpu().numpy(), K.cpu().numpy()
    Jo, Ko, _ = oracle.jk(mol, 0.0)
    for m in range(3):
        J1, K1 = jkb.jk(mol, D[m:m + 1].contiguous(), 0.0, precision="mixed", fp32_below=1e9)
        J1, K1 = J1.cpu().numpy()[0], K1.cpu().numpy()[0]
        say(f"  density {m}: max|J - J1|={np.abs(J[m] - J1).max():.2e} "
            f"max|K - K1|={np.abs(K[m] - K1).max():.2e} max|dJ|={np.abs(J[m] - Jo[m]).max():.2e}")
        assert np.abs(J[m] - J1).max() <= 1e-12 * np.abs(J1).max()
        assert np.abs(K[m] - K1).max() <= 1e-12 * np.abs(K1).max()
        assert np.abs(J[m] - Jo[m]).max() <= 1e-6 * np.abs(Jo[m]).max()
        assert np.abs(K[m] - Ko[m]).max() <= 1e-6 * np.abs(Ko[m]).max()


def test_ten_densities_mixed_against_fp64():
    """The 30-atom molecule with ten seeded densities (the several-density form of the
    1800-function workload, at a size that runs in a second): mixed against the GPU FP64
    build, |dE_J|, |dE_K| <= 1e-6 hartree per density, J symmetric."""
    import torch
    from paper_2406_11185_amd import jk as jkb
    w = molgen.WORKLOADS["w30"]
    mol = molgen.make_molecule(w["n_heavy"], w["n_h"], w["seed"], w["heavy_z"], n_dm=10)
    say(f"case mixed vs fp64, 10 densities ({mol.n_bf} functions, tol 1e-10)")
    D = torch.as_tensor(mol.D, device="cuda")
    J64, K64, E64 = [t.cpu().numpy() for t in jkb.jk(mol, D, 1e-10, energies=True)]
    Jm, Km, Em = [t.cpu().numpy() for t in jkb.jk(mol, D, 1e-10, precision="mixed", energies=True)]
    dEJ, dEK = np.abs(Em[:, 0] - E64[:, 0]).max(), np.abs(Em[:, 1] - E64[:, 1]).max()
    say(f"  max dEJ={dEJ:.2e} dEK={dEK:.2e} max|dJ|={np.abs(Jm - J64).max():.2e} "
        f"max|dK|={np.abs(Km - K64).max():.2e}")
    assert dEJ <= 1e-6 and dEK <= 1e-6
    np.testing.assert_allclose(Jm, Jm.transpose(0, 2, 1), atol=1e-13)


def test_ten_densities_in_place_mixed_against_oracle():
    """The ten-density, one-accumulator-copy path the 1800-function workload takes
    (J and K are the accumulators, finalized in place), mixed precision inside the
    dispatcher's envelope, against the oracle: |dE_J|, |dE_K| <= 1e-6 hartree per
    density and every element within 1e-6 of the largest."""
    import torch
    from paper_2406_11185_amd import jk as jkb
    mol = molgen.make_molecule(6, 8, 21, n_dm=10)   # 130 functions, a quarter in FP32
    say(f"case mixed, 10 densities, one accumulator copy ({mol.n_bf} functions, tol 1e-10)")
    D = torch.as_tensor(mol.D, device="cuda")
    J, K, E = [t.cpu().numpy() for t in
               jkb.jk(mol, D, 1e-10, precision="mixed", energies=True, acc_copies=1)]
    st = jkb.default_context(0).stats()
    assert sum(st.quartets_fp32) > 0 and sum(st.quartets_fp64) > 0
    Jo, Ko, _ = oracle.jk(mol, 1e-10)
    EJo, EKo = oracle.energy(Jo, Ko, mol.D)
    dEJ, dEK = np.abs(E[:, 0] - EJo).max(), np.abs(E[:, 1] - EKo).max()
    say(f"  max dEJ={dEJ:.2e} dEK={dEK:.2e} max|dJ|={np.abs(J - Jo).max():.2e} "
        f"max|dK|={np.abs(K - Ko).max():.2e}")
    assert dEJ <= 1e-6 and dEK <= 1e-6
    assert np.abs(J - Jo).max() <= 1e-6 * np.abs(Jo).max()
    assert np.abs(K - Ko).max() <= 1e-6 * np.abs(Ko).max()
