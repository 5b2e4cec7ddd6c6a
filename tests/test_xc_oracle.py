"""Pins of the XC-integration oracle (oracle/xc_oracle.py): on a uniform grid that
integrates Gaussians to near machine precision (trapezoidal rule on a box, which
converges faster than any power of the spacing for such integrands), the matrix
of weight 1 must be the overlap matrix, computed here independently from exact
Gauss-Hermite moments, and the density must integrate to tr(D S)."""
import math

import numpy as np
import pytest

from oracle import xc_oracle
from paper_2406_11185_amd import molgen

CART = {l: xc_oracle.cart_powers(l) for l in range(3)}


def _tight_molecule():
    """Two atoms, s, p and d shells of two primitives, exponents 0.8-3 (decay to
    1e-15 within 6.5 bohr, so a box of +-9 bohr around the atoms holds them)."""
    rng = np.random.default_rng(44)
    xyz = np.array([[0.0, 0.0, 0.0], [1.3, -0.4, 0.7]])
    shell_atom, shell_l, shell_nprim, shell_prim0, exps, coefs = [], [], [], [], [], []
    for at in range(2):
        for l in (0, 1, 2):
            shell_atom.append(at)
            shell_l.append(l)
            shell_nprim.append(2)
            shell_prim0.append(len(exps))
            exps += list(rng.uniform(0.8, 3.0, 2))
            coefs += list(rng.uniform(0.3, 1.0, 2))
    i32 = lambda v: np.asarray(v, dtype=np.int32)  # noqa: E731
    return molgen.Molecule(xyz, i32([6, 6]), i32(shell_atom), i32(shell_l), i32(shell_nprim),
                           i32(shell_prim0), np.asarray(exps), np.asarray(coefs))


def _moment_1d(a, A, i, b, B, j):
    """int (x-A)^i (x-B)^j exp(-a(x-A)^2 - b(x-B)^2) dx, exact (Gauss-Hermite)."""
    p = a + b
    P = (a * A + b * B) / p
    x, w = np.polynomial.hermite.hermgauss(8)
    t = P + x / math.sqrt(p)
    return math.exp(-a * b / p * (A - B) ** 2) / math.sqrt(p) * float(w @ ((t - A) ** i * (t - B) ** j))


def _overlap(mol):
    funcs = []
    for s in range(len(mol.shell_l)):
        for pw in CART[int(mol.shell_l[s])]:
            funcs.append((s, pw))
    n = len(funcs)
    S = np.zeros((n, n))
    for u, (s, pu) in enumerate(funcs):
        for v, (t, pv) in enumerate(funcs):
            A, B = mol.xyz[mol.shell_atom[s]], mol.xyz[mol.shell_atom[t]]
            tot = 0.0
            for k in range(mol.shell_prim0[s], mol.shell_prim0[s] + mol.shell_nprim[s]):
                for m in range(mol.shell_prim0[t], mol.shell_prim0[t] + mol.shell_nprim[t]):
                    val = mol.coefs[k] * mol.coefs[m]
                    for ax in range(3):
                        val *= _moment_1d(mol.exps[k], A[ax], pu[ax], mol.exps[m], B[ax], pv[ax])
                    tot += val
            S[u, v] = tot
    return S


@pytest.fixture(scope="module")
def box():
    mol = _tight_molecule()
    h = 0.16
    axes = [np.arange(-9.0 + c, 9.0 + c + h / 2, h) for c in (0.65, -0.2, 0.35)]
    X, Y, Z = np.meshgrid(*axes, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    return mol, pts, h ** 3


def test_unit_weight_matrix_is_the_overlap(box):
    mol, pts, w = box
    V = xc_oracle.vmat(mol, pts, np.full(len(pts), w))
    S = _overlap(mol)
    np.testing.assert_allclose(V, S, rtol=1e-11, atol=1e-12 * np.abs(S).max())


def test_density_integrates_to_trace_DS(box):
    mol, pts, w = box
    rng = np.random.default_rng(3)
    X = rng.normal(size=(2, 20, 20))
    D = X + X.transpose(0, 2, 1)
    r = xc_oracle.rho(mol, pts, D)
    S = _overlap(mol)
    for m in range(2):
        assert float(r[m].sum() * w) == pytest.approx(float(np.sum(D[m] * S)), rel=1e-11)


def test_ao_component_order_and_centre():
    """A p_y function is odd in y about its centre and zero on the plane y = A_y;
    d_xy changes sign with x and with y."""
    mol = _tight_molecule()
    A = mol.xyz[0]
    pts = np.array([A + [0.3, 0.2, -0.1], A + [0.3, -0.2, -0.1], A + [0.3, 0.0, -0.1],
                    A + [-0.3, 0.2, -0.1]])
    phi = xc_oracle.ao(mol, pts)
    py, dxy = 1 + 1, 1 + 3 + 1         # s (1), p (x, y, z), d (xx, xy, ...)
    assert phi[py, 0] == pytest.approx(-phi[py, 1], rel=1e-15) and phi[py, 2] == 0.0
    assert phi[dxy, 0] == pytest.approx(-phi[dxy, 1], rel=1e-15)
    assert phi[dxy, 0] == pytest.approx(-phi[dxy, 3], rel=1e-15)


def test_ao_gradient_by_central_differences():
    mol = _tight_molecule()
    rng = np.random.default_rng(8)
    pts = rng.uniform(-1.5, 2.5, (40, 3))
    g = xc_oracle.ao_grad(mol, pts)
    h = 1e-5
    for ax in range(3):
        dp = np.zeros(3)
        dp[ax] = h
        fd = (xc_oracle.ao(mol, pts + dp) - xc_oracle.ao(mol, pts - dp)) / (2 * h)
        np.testing.assert_allclose(g[ax], fd, rtol=1e-7, atol=1e-8)


def test_density_gradient_integrates_to_zero_and_gga_matrix(box):
    """grad rho of a localised density integrates to zero; with wv = 0 and a
    constant wg the GGA matrix is the integral of grad_c(phi_mu phi_nu), also zero."""
    mol, pts, w = box
    rng = np.random.default_rng(6)
    X = rng.normal(size=(20, 20))
    D = X + X.T
    gr = xc_oracle.rho_grad(mol, pts, D)[0]
    scale = float(np.abs(xc_oracle.rho(mol, pts, D)).sum() * w)
    assert np.abs(gr.sum(axis=1) * w).max() <= 1e-10 * scale
    wg = np.zeros((3, len(pts)))
    wg[1] = w
    V = xc_oracle.vmat_gga(mol, pts, np.zeros(len(pts)), wg)
    assert np.abs(V).max() <= 1e-10 * np.abs(_overlap(mol)).max()
