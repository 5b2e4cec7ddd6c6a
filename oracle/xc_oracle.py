"""CPU FP64 oracle for the exchange-correlation integration's data-parallel part
(test infrastructure only: the tests, the smoke check and the benchmark's CPU
leg use it; the library never does).

What it computes (paper, "Key Components Redesign and Implementation", EXC
paragraph: the integral is evaluated on grid points; basis-function values form
the AO matrix, from which the density on the grid and the XC matrix follow by
matrix products):

  ao(mol, pts)          phi[mu][g] = value of basis function mu at grid point g:
                        c_k-weighted sum over the shell's primitives of
                        x^lx y^ly z^lz exp(-a_k r^2), r measured from the shell's
                        atom, Cartesian components in the library's order.
  rho(mol, pts, D)      rho_g = sum_{mu,nu} phi_mu(g) D_mu,nu phi_nu(g).
  vmat(mol, pts, wv)    V_mu,nu = sum_g wv_g phi_mu(g) phi_nu(g), wv_g = the grid
                        weight times the functional's potential at g.
  ao_grad, rho_grad, vmat_gga: the gradient terms of gradient-corrected
                        functionals (the analytic AO derivatives, grad rho, and V with
                        the terms of the density-gradient derivative).

The definitions are written out with dense arrays (no screening, no blocks):
the library's distance cut-off and block sparsity must reproduce them within
the threshold that defines the sparsity.

Parity status: pinned (tests/test_xc_oracle.py).
"""
from __future__ import annotations

import numpy as np


def cart_powers(l: int):
    return [(lx, ly, l - lx - ly) for lx in range(l, -1, -1) for ly in range(l - lx, -1, -1)]


def ao(mol, pts):
    pts = np.asarray(pts, dtype=np.float64)
    rows = []
    for s in range(len(mol.shell_l)):
        l = int(mol.shell_l[s])
        A = np.asarray(mol.xyz[int(mol.shell_atom[s])], dtype=np.float64)
        d = pts - A
        r2 = np.sum(d * d, axis=1)
        p0, npr = int(mol.shell_prim0[s]), int(mol.shell_nprim[s])
        radial = np.zeros(len(pts))
        for k in range(p0, p0 + npr):
            radial += mol.coefs[k] * np.exp(-mol.exps[k] * r2)
        for (lx, ly, lz) in cart_powers(l):
            rows.append(d[:, 0] ** lx * d[:, 1] ** ly * d[:, 2] ** lz * radial)
    return np.array(rows)


def ao_grad(mol, pts):
    """d phi_mu / d r_c at the points, [3][n_ao][n_grid]: the derivative of
    x^a y^b z^c exp(-a_k r^2) along x is (a x^(a-1) - 2 a_k x^(a+1)) y^b z^c
    exp(-a_k r^2), summed over the primitives with their coefficients."""
    pts = np.asarray(pts, dtype=np.float64)
    out = [[], [], []]
    for s in range(len(mol.shell_l)):
        l = int(mol.shell_l[s])
        A = np.asarray(mol.xyz[int(mol.shell_atom[s])], dtype=np.float64)
        d = pts - A
        r2 = np.sum(d * d, axis=1)
        p0, npr = int(mol.shell_prim0[s]), int(mol.shell_nprim[s])
        for pw in cart_powers(l):
            for ax in range(3):
                val = np.zeros(len(pts))
                for k in range(p0, p0 + npr):
                    e = np.exp(-mol.exps[k] * r2)
                    term = np.ones(len(pts))
                    for bx in range(3):
                        if bx != ax:
                            term = term * d[:, bx] ** pw[bx]
                    lo = pw[ax] * d[:, ax] ** (pw[ax] - 1) if pw[ax] > 0 else 0.0
                    val += mol.coefs[k] * term * (lo - 2.0 * mol.exps[k] * d[:, ax] ** (pw[ax] + 1)) * e
                out[ax].append(val)
    return np.array(out)


def rho_grad(mol, pts, D):
    """grad rho_g = 2 sum_{mu,nu} grad phi_mu(g) D_mu,nu phi_nu(g) (D symmetric),
    [n_dm][3][n_grid]."""
    phi, dphi = ao(mol, pts), ao_grad(mol, pts)
    D = np.asarray(D, dtype=np.float64)
    if D.ndim == 2:
        D = D[None]
    return 2.0 * np.einsum("cmg,dmn,ng->dcg", dphi, D, phi)


def vmat_gga(mol, pts, wv, wg):
    """V = sum_g [wv_g phi_mu phi_nu + sum_c wg[c][g] (d_c phi_mu phi_nu + phi_mu d_c phi_nu)],
    wg[c][g] = the grid weight times the functional's derivative with respect to the
    density gradient component c."""
    phi, dphi = ao(mol, pts), ao_grad(mol, pts)
    V = np.einsum("mg,g,ng->mn", phi, np.asarray(wv, dtype=np.float64), phi)
    W = np.einsum("cmg,cg,ng->mn", dphi, np.asarray(wg, dtype=np.float64), phi)
    return V + W + W.T


def rho(mol, pts, D):
    phi = ao(mol, pts)
    D = np.asarray(D, dtype=np.float64)
    if D.ndim == 2:
        D = D[None]
    return np.einsum("mg,dmn,ng->dg", phi, D, phi)


def vmat(mol, pts, wv):
    phi = ao(mol, pts)
    return np.einsum("mg,g,ng->mn", phi, np.asarray(wv, dtype=np.float64), phi)
