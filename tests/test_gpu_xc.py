"""GPU parity of the XC integration's grid part (jk_xc_rho, jk_xc_vmat) against
the dense oracle definitions (oracle/xc_oracle.py): elementwise on small and
270-function molecules (three batches of points), sampled points of the
1080-function molecule on its full grid, and the identity tr(D V) = sum_g wv_g
rho_g at full size."""
import numpy as np
import pytest

from gpu_util import say
from oracle import xc_oracle
from paper_2406_11185_amd import molgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    assert torch.cuda.is_available(), "GPU test without a GPU"
    from paper_2406_11185_amd import jk as jkb
    jkb.load()


def _wv(pts, w, seed):
    """Grid weight times a smooth synthetic potential."""
    rng = np.random.default_rng(seed)
    c = rng.normal(size=3)
    return w * np.exp(-0.02 * np.sum((pts - c) ** 2, axis=1)) * (1.0 + 0.3 * np.sin(pts[:, 0]))


CASES = [("w4", lambda: molgen.workload("w4"), (30, 50), 1e-14, 1e-11),
         ("ragged", lambda: molgen.ragged_molecule(2, 3, 5), (24, 38), 1e-13, 1e-10),
         ("w30, three batches", lambda: molgen.workload("w30"), (30, 37), 1e-12, 1e-9)]


@pytest.mark.parametrize("name,make,grid,eps,rel", CASES, ids=[c[0] for c in CASES])
def test_xc_against_oracle(name, make, grid, eps, rel):
    import torch
    from paper_2406_11185_amd import jk as jkb
    mol = make()
    pts, w = molgen.atom_grid(mol, *grid)
    wv = _wv(pts, w, 1)
    say(f"case XC {name} ({mol.n_bf} functions, {len(pts)} points, eps {eps})")
    G = torch.as_tensor(pts, device="cuda")
    D = torch.as_tensor(mol.D, device="cuda")
    rho = jkb.xc_rho(mol, G, D, eps).cpu().numpy()
    V = jkb.xc_vmat(mol, G, torch.as_tensor(wv, device="cuda"), eps).cpu().numpy()
    ro = xc_oracle.rho(mol, pts, mol.D)
    Vo = xc_oracle.vmat(mol, pts, wv)
    say(f"  max|drho|={np.abs(rho - ro).max():.2e} (max rho {np.abs(ro).max():.2e}) "
        f"max|dV|={np.abs(V - Vo).max():.2e} (max V {np.abs(Vo).max():.2e})")
    assert np.abs(rho - ro).max() <= rel * np.abs(ro).max()
    assert np.abs(V - Vo).max() <= rel * np.abs(Vo).max()
    np.testing.assert_array_equal(V, V.T)


def test_xc_full_size_sampled_points_and_trace_identity():
    """1080 functions on a 660000-point grid: rho at 3000 sampled points against the
    oracle; tr(D V) = sum_g wv_g rho_g for the library's own rho and V."""
    import torch
    from paper_2406_11185_amd import jk as jkb
    mol = molgen.workload("w120")
    pts, w = molgen.atom_grid(mol, 50, 110)
    wv = _wv(pts, w, 2)
    say(f"case XC w120 ({mol.n_bf} functions, {len(pts)} points, eps 1e-12)")
    G = torch.as_tensor(pts, device="cuda")
    D = torch.as_tensor(mol.D, device="cuda")
    t_rho = torch.zeros(1, dtype=torch.int64, device="cuda")
    t_v = torch.zeros(1, dtype=torch.int64, device="cuda")
    rho = jkb.xc_rho(mol, G, D, tiles=t_rho).cpu().numpy()
    V = jkb.xc_vmat(mol, G, torch.as_tensor(wv, device="cuda"), tiles=t_v).cpu().numpy()
    nr, nv = int(t_rho.cpu()[0]), int(t_v.cpu()[0])
    nIb, nGb = (mol.n_bf + 31) // 32, sum((min(16384, len(pts) - g0) + 31) // 32
                                        for g0 in range(0, len(pts), 16384))
    say(f"  tile products: rho {nr}, V {nv} (dense: {nIb * nIb * nGb}, {nIb * (nIb + 1) // 2 * nGb})")
    assert 0 < nr < nIb * nIb * nGb and 0 < nv < nIb * (nIb + 1) // 2 * nGb
    idx = np.random.default_rng(3).choice(len(pts), 3000, replace=False)
    ro = xc_oracle.rho(mol, pts[idx], mol.D)
    say(f"  sampled max|drho|={np.abs(rho[0, idx] - ro).max():.2e} (max {np.abs(ro).max():.2e})")
    assert np.abs(rho[0, idx] - ro).max() <= 1e-9 * np.abs(ro).max()
    lhs, rhs = float(np.sum(mol.D[0] * V)), float(wv @ rho[0])
    say(f"  tr(DV)={lhs:.12e} sum wv rho={rhs:.12e}")
    assert lhs == pytest.approx(rhs, rel=1e-9)


def test_xc_argument_checks():
    import ctypes
    import torch
    from paper_2406_11185_amd import jk as jkb
    mol = molgen.make_molecule(1, 1, 7)
    b = jkb.Basis(mol)
    G = torch.zeros((10, 3), dtype=torch.float64, device="cuda")
    D = torch.as_tensor(mol.D, device="cuda")
    rho = torch.full((1, 10), 7.0, dtype=torch.float64, device="cuda")
    lib = jkb.load()
    p = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    s = None
    assert lib.jk_xc_rho(ctypes.byref(b.c), p(G), 10, p(D), 1, 0.0, p(rho), None, s) == jkb.JK_EINVAL
    assert lib.jk_xc_rho(ctypes.byref(b.c), p(G), 0, p(D), 1, 1e-12, p(rho), None, s) == jkb.JK_EINVAL
    assert lib.jk_xc_rho(None, p(G), 10, p(D), 1, 1e-12, p(rho), None, s) == jkb.JK_EINVAL
    assert lib.jk_xc_vmat(ctypes.byref(b.c), p(G), 10, None, 1e-12, p(D), None, s) == jkb.JK_EINVAL
    torch.cuda.synchronize()
    assert bool((rho == 7.0).all())


GGA_CASES = [("w4", lambda: molgen.workload("w4"), (30, 50), 1e-14, 1e-11),
             ("w30, three batches", lambda: molgen.workload("w30"), (30, 37), 1e-12, 1e-9)]


@pytest.mark.parametrize("name,make,grid,eps,rel", GGA_CASES, ids=[c[0] for c in GGA_CASES])
def test_xc_gga_against_oracle(name, make, grid, eps, rel):
    """Gradient-corrected terms: rho, grad rho and the GGA matrix against the dense
    oracle (analytic AO derivatives)."""
    import torch
    from paper_2406_11185_amd import jk as jkb
    mol = make()
    pts, w = molgen.atom_grid(mol, *grid)
    wv = _wv(pts, w, 3)
    rng = np.random.default_rng(4)
    wg = np.stack([_wv(pts, w, 5 + c) * rng.uniform(0.5, 1.5) for c in range(3)])
    say(f"case XC GGA {name} ({mol.n_bf} functions, {len(pts)} points, eps {eps})")
    G = torch.as_tensor(pts, device="cuda")
    D = torch.as_tensor(mol.D, device="cuda")
    rho, grad = jkb.xc_rho_gga(mol, G, D, eps)
    V = jkb.xc_vmat_gga(mol, G, torch.as_tensor(wv, device="cuda"),
                        torch.as_tensor(wg, device="cuda").contiguous(), eps)
    rho, grad, V = rho.cpu().numpy(), grad.cpu().numpy(), V.cpu().numpy()
    ro = xc_oracle.rho(mol, pts, mol.D)
    go = xc_oracle.rho_grad(mol, pts, mol.D)
    Vo = xc_oracle.vmat_gga(mol, pts, wv, wg)
    say(f"  max|drho|={np.abs(rho - ro).max():.2e} max|dgrad|={np.abs(grad - go).max():.2e} "
        f"(max {np.abs(go).max():.2e}) max|dV|={np.abs(V - Vo).max():.2e} (max {np.abs(Vo).max():.2e})")
    assert np.abs(rho - ro).max() <= rel * np.abs(ro).max()
    assert np.abs(grad - go).max() <= rel * np.abs(go).max()
    assert np.abs(V - Vo).max() <= rel * np.abs(Vo).max()
    np.testing.assert_array_equal(V, V.T)
