"""GPU parity of the SCF steps beside the build (jk_scf_diag, jk_scf_diis) against
the CPU oracle (oracle/scf_oracle.py), up to the size of the 1080-function
workload, plus properties that hold at any size."""
import math

import numpy as np
import pytest

from gpu_util import say
from oracle import scf_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    assert torch.cuda.is_available(), "GPU test without a GPU"
    from paper_2406_11185_amd import jk as jkb
    jkb.load()


def _spd(n, rng):
    """Overlap-like: unit diagonal, off-diagonal couplings, positive definite."""
    X = rng.normal(size=(n, n)) * 0.3 / math.sqrt(n)
    return np.eye(n) * 1.3 + 0.5 * (X + X.T)


def _sym(n, rng):
    X = rng.normal(size=(n, n)) / math.sqrt(n)
    return 0.5 * (X + X.T)


@pytest.mark.parametrize("n,n_occ", [(64, 17), (301, 80), (1080, 300)])
def test_diag_against_oracle(n, n_occ):
    import torch
    from paper_2406_11185_amd import jk as jkb
    rng = np.random.default_rng(n)
    S, F = _spd(n, rng), _sym(n, rng)
    say(f"case diag n={n} n_occ={n_occ}")
    h = jkb.ScfSteps(n, depth=2)
    Sd, Fd = torch.as_tensor(S, device="cuda"), torch.as_tensor(F, device="cuda")
    eps, C, D = h.diag(Fd, Sd, n_occ)
    torch.cuda.synchronize()
    eps, C, D = eps.cpu().numpy(), C.cpu().numpy(), D.cpu().numpy()
    eo, Co, Do = scf_oracle.roothaan(F, S, n_occ)
    scale = np.abs(eo).max()
    say(f"  max|d eps|={np.abs(eps - eo).max():.2e} max|dD|={np.abs(D - Do).max():.2e} "
        f"gap={eo[n_occ] - eo[n_occ - 1]:.2e}")
    assert np.abs(eps - eo).max() <= 1e-12 * n * scale
    assert np.abs(D - Do).max() <= 1e-9
    # rows of C are S-orthonormal eigenvectors (unique up to sign)
    np.testing.assert_allclose(C @ S @ C.T, np.eye(n), atol=1e-10)
    assert np.abs(F @ C.T - S @ C.T @ np.diag(eps)).max() <= 1e-10
    np.testing.assert_allclose(np.abs(C), np.abs(Co.T), atol=1e-7)


def test_diis_against_oracle_through_the_ring():
    """depth 3, five pairs: the ring drops the oldest pair from the fourth on."""
    import torch
    from paper_2406_11185_amd import jk as jkb
    n, depth = 200, 3
    rng = np.random.default_rng(21)
    S = _spd(n, rng)
    base = _sym(n, rng)
    Fs, Ds = [], []
    h = jkb.ScfSteps(n, depth=depth)
    Sd = torch.as_tensor(S, device="cuda")
    say(f"case DIIS n={n} depth={depth}")
    for k in range(5):
        F = base + 0.05 * _sym(n, rng) / (k + 1)
        _, _, D = scf_oracle.roothaan(base + 0.1 * _sym(n, rng), S, 50)
        Fs.append(F)
        Ds.append(D)
        Fo, err = h.diis(torch.as_tensor(F, device="cuda"), torch.as_tensor(D, device="cuda"), Sd)
        torch.cuda.synchronize()
        Fref, c, emax = scf_oracle.diis(Fs[-depth:], Ds[-depth:], S)
        d = np.abs(Fo.cpu().numpy() - Fref).max()
        say(f"  step {k}: {len(c)} pairs, c={np.round(c, 4)}, max|dF|={d:.2e}")
        assert d <= 1e-10 * np.abs(Fref).max()
        assert float(err.cpu()[0]) == pytest.approx(emax, rel=1e-12)
    h.reset()
    Fo, _ = h.diis(torch.as_tensor(Fs[0], device="cuda"), torch.as_tensor(Ds[0], device="cuda"), Sd)
    torch.cuda.synchronize()
    np.testing.assert_allclose(Fo.cpu().numpy(), Fs[0], atol=0)


def test_scf_argument_checks():
    import torch
    from paper_2406_11185_amd import jk as jkb
    with pytest.raises(jkb.JkError):
        jkb.ScfSteps(0)
    with pytest.raises(jkb.JkError):
        jkb.ScfSteps(10, depth=0)
    h = jkb.ScfSteps(10, depth=2)
    F = torch.eye(10, dtype=torch.float64, device="cuda")
    notpd = -torch.eye(10, dtype=torch.float64, device="cuda")
    with pytest.raises(jkb.JkError) as e:
        h.diag(F, notpd, 3)
    assert e.value.code == jkb.JK_EINVAL
    with pytest.raises(jkb.JkError):
        h.diag(F, F, 11)
