"""Pins of the SCF-step oracle (oracle/scf_oracle.py) against what the mathematics
fixes: the generalised eigenproblem's residual, S-orthonormality and a 2x2 closed
form; the density as an S-projector; a zero DIIS error at self-consistency; DIIS
on one and two vectors in closed form."""
import math

import numpy as np
import pytest

from oracle import scf_oracle


def _spd(n, rng, spread=0.3):
    X = rng.normal(size=(n, n)) * spread / math.sqrt(n)
    return np.eye(n) + 0.5 * (X + X.T) + spread * np.eye(n)


def _sym(n, rng):
    X = rng.normal(size=(n, n))
    return 0.5 * (X + X.T)


@pytest.mark.parametrize("n,n_occ", [(2, 1), (7, 3), (40, 11)])
def test_roothaan_residual_orthonormality_and_projector(n, n_occ):
    rng = np.random.default_rng(n)
    S, F = _spd(n, rng), _sym(n, rng)
    eps, C, D = scf_oracle.roothaan(F, S, n_occ)
    scale = np.abs(F).max()
    assert np.abs(F @ C - S @ C @ np.diag(eps)).max() <= 1e-12 * scale * n
    np.testing.assert_allclose(C.T @ S @ C, np.eye(n), atol=1e-12)
    assert np.all(np.diff(eps) >= 0)
    P = 0.5 * D @ S                       # projector onto the occupied space
    np.testing.assert_allclose(P @ P, P, atol=1e-11)
    assert np.trace(P) == pytest.approx(n_occ, abs=1e-11)


def test_roothaan_two_by_two_closed_form():
    a, b, c = 0.7, -0.35, -1.2
    eps, C, D = scf_oracle.roothaan([[a, b], [b, c]], np.eye(2), 1)
    mid, rad = 0.5 * (a + c), math.hypot(0.5 * (a - c), b)
    assert eps[0] == pytest.approx(mid - rad, abs=1e-15)
    assert eps[1] == pytest.approx(mid + rad, abs=1e-15)
    # lower eigenvector of a 2x2 symmetric matrix: (b, lambda - a), normalised
    v = np.array([b, eps[0] - a])
    v /= np.linalg.norm(v)
    np.testing.assert_allclose(D, 2.0 * np.outer(v, v), atol=1e-14)


def test_diis_error_vanishes_at_self_consistency():
    """D built from F's own occupied orbitals commutes with F in the S metric."""
    rng = np.random.default_rng(5)
    S, F = _spd(30, rng), _sym(30, rng)
    _, _, D = scf_oracle.roothaan(F, S, 9)
    assert np.abs(scf_oracle.diis_error(F, D, S)).max() <= 1e-11 * np.abs(F).max()
    D2 = D + 1e-3 * _sym(30, rng)
    assert np.abs(scf_oracle.diis_error(F, D2, S)).max() > 1e-6


def test_diis_one_and_two_vectors_in_closed_form():
    rng = np.random.default_rng(9)
    n = 12
    S = _spd(n, rng)
    Fs = [_sym(n, rng) for _ in range(2)]
    Ds = [_sym(n, rng) for _ in range(2)]
    Fx, c, _ = scf_oracle.diis(Fs[:1], Ds[:1], S)
    np.testing.assert_allclose(Fx, Fs[0], atol=0)
    assert c[0] == pytest.approx(1.0, abs=1e-15)
    e1, e2 = (F @ D @ S - S @ D @ F for F, D in zip(Fs, Ds))
    # minimise |c e1 + (1 - c) e2|^2 over c
    d = e1 - e2
    c1 = -float(np.sum(d * e2)) / float(np.sum(d * d))
    Fx, c, emax = scf_oracle.diis(Fs, Ds, S)
    assert c[0] == pytest.approx(c1, rel=1e-12) and c[1] == pytest.approx(1 - c1, rel=1e-12)
    np.testing.assert_allclose(Fx, c1 * Fs[0] + (1 - c1) * Fs[1], atol=1e-13)
    assert emax == pytest.approx(np.abs(e2).max(), rel=1e-15)


def test_diis_opposite_errors_average():
    """Errors e and -e: the minimum-norm combination is the average."""
    rng = np.random.default_rng(2)
    n = 6
    S = np.eye(n)
    F1 = _sym(n, rng)
    D1 = _sym(n, rng)
    # F2 = -F1 with the same D gives e2 = -e1
    Fx, c, _ = scf_oracle.diis([F1, -F1], [D1, D1], S)
    np.testing.assert_allclose(c, [0.5, 0.5], atol=1e-14)
    np.testing.assert_allclose(Fx, 0.0, atol=1e-14)
