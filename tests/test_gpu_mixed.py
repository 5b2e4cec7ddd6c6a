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
