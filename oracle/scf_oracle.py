"""CPU FP64 oracle for the SCF steps on either side of the J/K build (test
infrastructure only: the tests, the smoke check and the benchmark's CPU leg use
it; the library never does).

What it computes (paper, "DFT Calculation Flow": the Kohn-Sham equations are
solved by diagonalising the Fock matrix, the density is rebuilt from the occupied
orbitals, and the iterations are accelerated by direct inversion in the iterative
subspace; "Key Components Redesign and Implementation", SCF-iteration paragraph:
both steps run on the GPU):

  roothaan(F, S, n_occ): F C = S C diag(eps) with C^T S C = I and eps ascending
      (one library routine, the generalised symmetric eigensolver), and the
      closed-shell density D = 2 sum_{i < n_occ} c_i c_i^T.
  diis(Fs, Ds, S): Pulay's extrapolation.  Error of each pair e_i = F_i D_i S -
      S D_i F_i (zero at self-consistency); coefficients c minimise
      |sum_i c_i e_i|^2 subject to sum_i c_i = 1, from the bordered system
      [B -1; -1^T 0] [c; lambda] = [0; -1] with B_ij = <e_i, e_j>; the result is
      sum_i c_i F_i.

Parity status: pinned (tests/test_scf_oracle.py).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


def roothaan(F, S, n_occ: int):
    """(eps [n], C [n][n] with orbital j in column j, D [n][n])."""
    F = np.asarray(F, dtype=np.float64)
    S = np.asarray(S, dtype=np.float64)
    eps, C = scipy.linalg.eigh(F, S)
    Cocc = C[:, :n_occ]
    D = 2.0 * Cocc @ Cocc.T
    return eps, C, D


def diis_error(F, D, S):
    F, D, S = (np.asarray(X, dtype=np.float64) for X in (F, D, S))
    return F @ D @ S - S @ D @ F


def diis(Fs, Ds, S):
    """(extrapolated F, coefficients c, max |e| of the last pair)."""
    es = [diis_error(F, D, S) for F, D in zip(Fs, Ds)]
    m = len(es)
    A = np.zeros((m + 1, m + 1))
    for i in range(m):
        for j in range(m):
            A[i, j] = float(np.sum(es[i] * es[j]))
    A[:m, m] = -1.0
    A[m, :m] = -1.0
    rhs = np.zeros(m + 1)
    rhs[m] = -1.0
    c = np.linalg.solve(A, rhs)[:m]
    Fx = sum(ci * np.asarray(Fi, dtype=np.float64) for ci, Fi in zip(c, Fs))
    return Fx, c, float(np.abs(es[-1]).max())
