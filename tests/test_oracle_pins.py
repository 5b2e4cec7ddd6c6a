"""Pins of the CPU oracle against mathematics that does not go through it.

Every check here is independent of the oracle's own code path: mpmath special
functions, closed forms, numerical differentiation, brute-force quadrature,
symmetry and invariance properties, and finite differences.
"""
import math

import numpy as np
import pytest

import oracle
import pins
from paper_2406_11185_amd import molgen

rng_cases = np.random.default_rng(20240617)


# --- Boys function -------------------------------------------------------------

@pytest.mark.parametrize("T", [0.0, 1e-12, 1e-6, 0.05, 0.7, 2.5, 9.9, 17.3, 29.999, 30.0,
                               30.001, 45.0, 80.0, 200.0])
def test_boys_matches_incomplete_gamma(T):
    F = oracle.boys(12, T)
    for m in range(13):
        ref = float(pins.boys_mp(m, T))
        assert abs(F[m] - ref) <= 2e-15 * abs(ref) + 1e-300, (m, T, F[m], ref)


def test_boys_at_zero_and_asymptote():
    F = oracle.boys(10, 0.0)
    for m in range(11):
        assert F[m] == pytest.approx(1.0 / (2 * m + 1), rel=1e-15)
    T = 150.0
    F = oracle.boys(9, T)
    for m in range(10):
        dfac = math.prod(range(2 * m - 1, 0, -2)) if m > 0 else 1
        asym = dfac / 2 ** (m + 1) * math.sqrt(math.pi / T ** (2 * m + 1))
        assert F[m] == pytest.approx(asym, rel=1e-13)


def test_boys_recurrences_hold():
    for T in (0.3, 4.0, 29.0, 31.0, 60.0):
        F = oracle.boys(10, T)
        e = math.exp(-T)
        for m in range(10):
            assert (2 * m + 1) * F[m] == pytest.approx(2 * T * F[m + 1] + e, rel=1e-14)


# --- primitive integrals --------------------------------------------------------

def _rand_prims(rng, pows):
    ex = rng.uniform(0.1, 4.0, 4)
    C = [rng.uniform(-1.5, 1.5, 3) for _ in range(4)]
    args = []
    for k in range(4):
        args += [pows[k], ex[k], C[k]]
    return args


def test_ssss_closed_form():
    rng = np.random.default_rng(1)
    z = (0, 0, 0)
    for _ in range(20):
        args = _rand_prims(rng, [z, z, z, z])
        o = oracle.prim_eri(*args)
        ref = float(pins.ssss_closed(args[1], args[2], args[4], args[5], args[7], args[8],
                                     args[10], args[11]))
        assert o == pytest.approx(ref, rel=1e-14)
    # coincident centres: T = 0 branch
    A = np.zeros(3)
    o = oracle.prim_eri(z, 0.7, A, z, 0.3, A, z, 1.1, A, z, 0.2, A)
    ref = float(pins.ssss_closed(0.7, A, 0.3, A, 1.1, A, 0.2, A))
    assert o == pytest.approx(ref, rel=1e-14)


DERIV_CASES = [
    ((1, 0, 0), (0, 0, 0), (0, 0, 0), (0, 0, 0)),
    ((0, 0, 1), (0, 1, 0), (0, 0, 0), (0, 0, 0)),
    ((2, 0, 0), (0, 0, 0), (0, 0, 0), (0, 0, 0)),
    ((1, 1, 0), (0, 0, 0), (0, 0, 1), (0, 0, 0)),
    ((0, 1, 0), (0, 0, 0), (0, 1, 0), (1, 0, 0)),
    ((0, 0, 0), (0, 0, 2), (0, 0, 0), (0, 1, 0)),
]


@pytest.mark.parametrize("pows", DERIV_CASES)
def test_prim_eri_as_centre_derivatives(pows):
    rng = np.random.default_rng(hash(pows) % 2**32)
    args = _rand_prims(rng, list(pows))
    o = oracle.prim_eri(*args)
    ref = pins.eri_by_derivs(*args)
    assert abs(o - ref) <= 1e-12 * max(abs(ref), 1e-3), (o, ref)


QUAD_CASES = [
    ((0, 0, 0), (0, 0, 0), (0, 0, 0), (0, 0, 0)),
    ((1, 0, 0), (0, 1, 0), (0, 0, 0), (0, 0, 1)),
    ((2, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 0)),
    ((0, 1, 1), (1, 0, 1), (2, 0, 0), (0, 1, 1)),
    ((1, 0, 1), (0, 2, 0), (1, 1, 0), (0, 0, 2)),
    ((0, 0, 2), (0, 0, 2), (0, 0, 2), (0, 0, 2)),
    ((3, 0, 0), (0, 1, 1), (0, 2, 0), (1, 0, 0)),   # one centre at l+1 (gradient)
]


@pytest.mark.parametrize("pows", QUAD_CASES)
def test_prim_eri_by_quadrature(pows):
    rng = np.random.default_rng(sum(sum(p) * (i + 3) for i, p in enumerate(pows)))
    args = _rand_prims(rng, list(pows))
    o = oracle.prim_eri(*args)
    ref = pins.eri_quadrature(*args)
    assert abs(o - ref) <= 1e-11 * max(abs(ref), 1e-6), (o, ref)


def test_prim_eri_axis_permutation_and_inversion():
    rng = np.random.default_rng(3)
    perm = [1, 2, 0]
    for _ in range(10):
        pows = [tuple(int(x) for x in rng.integers(0, 2, 3)) for _ in range(4)]
        args = _rand_prims(rng, pows)
        o = oracle.prim_eri(*args)
        pa = list(args)
        for k in range(4):
            pa[3 * k] = tuple(args[3 * k][i] for i in perm)
            pa[3 * k + 2] = np.asarray(args[3 * k + 2])[perm]
        assert oracle.prim_eri(*pa) == pytest.approx(o, rel=1e-13, abs=1e-16)
        inv = list(args)
        for k in range(4):
            inv[3 * k + 2] = -np.asarray(args[3 * k + 2])
        ltot = sum(sum(p) for p in pows)
        assert oracle.prim_eri(*inv) == pytest.approx((-1) ** ltot * o, rel=1e-13, abs=1e-16)


# --- contracted shell quartets --------------------------------------------------

@pytest.fixture(scope="module")
def w4():
    return molgen.workload("w4")


def test_eightfold_symmetry(w4):
    b = oracle.Basis(w4)
    rng = np.random.default_rng(11)
    for _ in range(12):
        A, B, C, D = (int(x) for x in rng.integers(0, w4.n_shells, 4))
        ref = oracle.shell_quartet(b, A, B, C, D)
        perms = {
            (B, A, C, D): (1, 0, 2, 3), (A, B, D, C): (0, 1, 3, 2), (B, A, D, C): (1, 0, 3, 2),
            (C, D, A, B): (2, 3, 0, 1), (D, C, A, B): (3, 2, 0, 1), (C, D, B, A): (2, 3, 1, 0),
            (D, C, B, A): (3, 2, 1, 0),
        }
        for (a, bb, c, d), axes in perms.items():
            other = oracle.shell_quartet(b, a, bb, c, d)
            # other[i_a, i_b, i_c, i_d] with the roles permuted back to (A B | C D)
            back = np.transpose(other, np.argsort(axes))
            np.testing.assert_allclose(back, ref, rtol=1e-13, atol=1e-16)


def test_schwarz_inequality_and_positive_diagonal(w4):
    b = oracle.Basis(w4)
    Q = oracle.schwarz(b)
    rng = np.random.default_rng(12)
    for _ in range(200):
        A, B, C, D = (int(x) for x in rng.integers(0, w4.n_shells, 4))
        blk = oracle.shell_quartet(b, A, B, C, D)
        assert np.abs(blk).max() <= Q[A, B] * Q[C, D] * (1 + 1e-12) + 1e-18
    for A in range(w4.n_shells):
        blk = oracle.shell_quartet(b, A, A, A, A)
        n = blk.shape[0]
        M = blk.reshape(n * n, n * n)
        assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > -1e-12


def test_translation_invariance(w4):
    J0, K0, _ = oracle.jk(w4, 0.0)
    shifted = w4.with_xyz(w4.xyz + np.array([0.37, -1.2, 2.05]))
    J1, K1, _ = oracle.jk(shifted, 0.0)
    np.testing.assert_allclose(J1, J0, atol=1e-12)
    np.testing.assert_allclose(K1, K0, atol=1e-12)


# --- J and K --------------------------------------------------------------------

def test_unique_digestion_equals_definition_blocks(w4):
    """Symmetry-unique digestion against the plain sums for every shell pair."""
    J, K, kept = oracle.jk(w4, 0.0)
    assert kept == 171 * 172 // 2
    ns = w4.n_shells
    bf0 = w4.shell_bf0
    pairs = [(m, n) for m in range(ns) for n in range(ns) if (m * 7 + n) % 5 == 0]
    blocks = oracle.jk_blocks(w4, 0.0, pairs)
    for (m, n), (jb, kb) in zip(pairs, blocks):
        nm, nn = jb.shape[1:]
        np.testing.assert_allclose(J[0, bf0[m]:bf0[m] + nm, bf0[n]:bf0[n] + nn], jb[0],
                                   atol=1e-13, rtol=1e-12)
        np.testing.assert_allclose(K[0, bf0[m]:bf0[m] + nm, bf0[n]:bf0[n] + nn], kb[0],
                                   atol=1e-13, rtol=1e-12)


def test_full_tensor_brute_force():
    """Tiny molecule: full n^4 ERI tensor from ordered quartets, J/K by einsum."""
    mol = molgen.make_molecule(1, 1, seed=7)
    b = oracle.Basis(mol)
    n, ns = mol.n_bf, mol.n_shells
    bf0 = mol.shell_bf0
    nc = [molgen.ncart(int(l)) for l in mol.shell_l]
    eri = np.zeros((n, n, n, n))
    for A in range(ns):
        for B in range(ns):
            for C in range(ns):
                for D in range(ns):
                    eri[bf0[A]:bf0[A] + nc[A], bf0[B]:bf0[B] + nc[B], bf0[C]:bf0[C] + nc[C],
                        bf0[D]:bf0[D] + nc[D]] = oracle.shell_quartet(b, A, B, C, D)
    Dm = mol.D[0]
    Jref = np.einsum("ijkl,kl->ij", eri, Dm)
    Kref = np.einsum("ikjl,kl->ij", eri, Dm)
    J, K, _ = oracle.jk(mol, 0.0)
    np.testing.assert_allclose(J[0], Jref, atol=1e-13, rtol=1e-12)
    np.testing.assert_allclose(K[0], Kref, atol=1e-13, rtol=1e-12)


def test_rank_one_identity_and_positivity(w4):
    """D = c c^T: (Jc)_mu = (mu phi|phi phi) = (Kc)_mu; E_J, E_K >= 0 for D = C C^T."""
    rng = np.random.default_rng(2)
    c = rng.normal(size=w4.n_bf)
    D1 = np.outer(c, c)
    J, K, _ = oracle.jk(w4, 0.0, D=D1)
    np.testing.assert_allclose(J[0] @ c, K[0] @ c, rtol=1e-11, atol=1e-11)
    J, K, _ = oracle.jk(w4, 0.0)
    EJ, EK = oracle.energy(J, K, w4.D)
    assert EJ[0] > 0 and EK[0] > 0
    np.testing.assert_allclose(J, J.transpose(0, 2, 1), atol=1e-14)
    np.testing.assert_allclose(K, K.transpose(0, 2, 1), atol=1e-14)


def test_screening_error_is_bounded():
    mol = molgen.make_molecule(3, 3, seed=21)
    J0, K0, k0 = oracle.jk(mol, 0.0)
    tol = 1e-4  # small molecule: every pair bound is above 3e-3, so screen coarsely
    J1, K1, k1 = oracle.jk(mol, tol)
    assert k1 < k0
    dmax = np.abs(mol.D).max()
    bound = (k0 - k1) * tol * dmax * 2 * 36
    assert np.abs(J1 - J0).max() <= bound
    assert np.abs(K1 - K0).max() <= bound
    assert np.abs(J1 - J0).max() > 0


# --- gradient -------------------------------------------------------------------

def _energy(mol):
    J, K, _ = oracle.jk(mol, 0.0)
    EJ, EK = oracle.energy(J, K, mol.D)
    return EJ - EK


def test_gradient_central_differences():
    mol = molgen.make_molecule(1, 1, seed=7)
    G = oracle.grad(mol, 0.0)
    h = 1e-4
    for a in range(mol.n_atoms):
        for x in range(3):
            xp = mol.xyz.copy(); xp[a, x] += h
            xm = mol.xyz.copy(); xm[a, x] -= h
            fd = (_energy(mol.with_xyz(xp)) - _energy(mol.with_xyz(xm))) / (2 * h)
            assert abs(G[0, a, x] - fd[0]) <= 1e-7, (a, x, G[0, a, x], fd)


def test_gradient_translation_sum_and_s_only_rotation():
    mol = molgen.make_molecule(1, 2, seed=9)
    G = oracle.grad(mol, 0.0)
    np.testing.assert_allclose(G[0].sum(axis=0), 0.0, atol=1e-11)
    # s-only basis: E is rotation invariant, so the torque sum_A R_A x g_A vanishes
    s_only = [i for i, l in enumerate(mol.shell_l) if l == 0]
    sub = molgen.Molecule(mol.xyz, mol.Z, mol.shell_atom[s_only], mol.shell_l[s_only],
                          mol.shell_nprim[s_only], mol.shell_prim0[s_only], mol.exps,
                          mol.coefs)
    rng = np.random.default_rng(4)
    Cm = rng.normal(size=(sub.n_bf, 3))
    sub = sub.with_D(Cm @ Cm.T)
    Gs = oracle.grad(sub, 0.0)[0]
    torque = np.cross(sub.xyz, Gs).sum(axis=0)
    np.testing.assert_allclose(torque, 0.0, atol=1e-11)


# --- contracted shell quartets against brute-force quadrature --------------------

# Cartesian components in the order every interface here uses (descending powers
# of x, then y), written out by hand
CART = {0: [(0, 0, 0)],
        1: [(1, 0, 0), (0, 1, 0), (0, 0, 1)],
        2: [(2, 0, 0), (1, 1, 0), (1, 0, 1), (0, 2, 0), (0, 1, 1), (0, 0, 2)]}


def _four_centre_basis(nprim, seed):
    """Four atoms, each with one s, one p and one d shell of `nprim` primitives."""
    rng = np.random.default_rng(seed)
    xyz = rng.uniform(-1.2, 1.2, (4, 3))
    shell_atom, shell_l, shell_nprim, shell_prim0, exps, coefs = [], [], [], [], [], []
    for at in range(4):
        for l in (0, 1, 2):
            shell_atom.append(at)
            shell_l.append(l)
            shell_nprim.append(nprim)
            shell_prim0.append(len(exps))
            exps += list(rng.uniform(0.3, 1.6, nprim))
            coefs += list(rng.uniform(0.2, 1.0, nprim))
    i32 = lambda v: np.asarray(v, dtype=np.int32)  # noqa: E731
    return molgen.Molecule(xyz, i32([8, 8, 8, 8]), i32(shell_atom), i32(shell_l),
                           i32(shell_nprim), i32(shell_prim0), np.asarray(exps),
                           np.asarray(coefs))


def _contracted_by_quadrature(mol, shells, comps, omega=None):
    """sum over primitives of c c c c x (quadrature of the primitive integral)."""
    tot = 0.0
    ranges = [range(int(mol.shell_prim0[s]), int(mol.shell_prim0[s] + mol.shell_nprim[s]))
              for s in shells]
    cents = [mol.xyz[int(mol.shell_atom[s])] for s in shells]
    for i in ranges[0]:
        for j in ranges[1]:
            for k in ranges[2]:
                for m in ranges[3]:
                    cc = mol.coefs[i] * mol.coefs[j] * mol.coefs[k] * mol.coefs[m]
                    tot += cc * pins.eri_quadrature(comps[0], mol.exps[i], cents[0],
                                                    comps[1], mol.exps[j], cents[1],
                                                    comps[2], mol.exps[k], cents[2],
                                                    comps[3], mol.exps[m], cents[3],
                                                    omega=omega)
    return tot


@pytest.mark.parametrize("ls,ncomp", [((2, 0, 1, 0), 6), ((2, 2, 1, 1), 4), ((2, 2, 2, 2), 3)])
def test_contracted_quartet_components(ls, ncomp):
    """Contraction over primitives and the Cartesian component order of the
    oracle's shell quartets: selected components of (ds|ps), (dd|pp), (dd|dd)
    quartets of two-primitive shells on four centres."""
    mol = _four_centre_basis(2, seed=sum(ls) + 40)
    shells = [3 * at + l for at, l in enumerate(ls)]   # shell of angular momentum l on atom at
    blk = oracle.shell_quartet(oracle.Basis(mol), *shells)
    rng = np.random.default_rng(7 + sum(ls))
    picks = {tuple(len(CART[l]) - 1 for l in ls), (0, 0, 0, 0)}
    while len(picks) < ncomp:
        picks.add(tuple(int(rng.integers(len(CART[l]))) for l in ls))
    for idx in sorted(picks):
        comps = [CART[l][i] for l, i in zip(ls, idx)]
        ref = _contracted_by_quadrature(mol, shells, comps)
        assert abs(blk[idx] - ref) <= 1e-11 * max(abs(ref), 1e-6), (idx, blk[idx], ref)


@pytest.mark.parametrize("la,lb", [(2, 0), (1, 1)])
def test_schwarz_factor_is_max_of_diagonal(la, lb):
    """Q_AB^2 = max over components of (ab|ab), from quadrature values."""
    mol = _four_centre_basis(1, seed=60 + la + lb)
    A, B = 3 * 0 + la, 3 * 1 + lb
    diag = []
    for ca in CART[la]:
        for cb in CART[lb]:
            diag.append(_contracted_by_quadrature(mol, (A, B, A, B), (ca, cb, ca, cb)))
    Q = oracle.schwarz(oracle.Basis(mol))
    assert Q[A, B] ** 2 == pytest.approx(max(diag), rel=1e-11)
    assert max(diag) < sum(diag)   # the max, not the sum, is what is pinned


# --- timing-leg digestion and screening counts ---------------------------------------

def test_bra_sample_over_all_pairs_equals_jk(w4):
    """The timing leg over every unique bra pair gives orc_jk's accumulators:
    its J + J^T equals the full J (and the same for K), with the same count."""
    for tol in (0.0, 1e-6):
        J, K, kept = oracle.jk(w4, tol)
        npair = w4.n_shells * (w4.n_shells + 1) // 2
        Js, Ks, ks = oracle.jk_bra_sample(w4, tol, np.arange(npair))
        assert ks == kept
        np.testing.assert_allclose(Js + Js.transpose(0, 2, 1), J, atol=1e-13, rtol=1e-13)
        np.testing.assert_allclose(Ks + Ks.transpose(0, 2, 1), K, atol=1e-13, rtol=1e-13)
        # disjoint samples add up to the whole
        half = np.arange(0, npair, 2)
        Ja, _, ka = oracle.jk_bra_sample(w4, tol, half)
        Jb, _, kb = oracle.jk_bra_sample(w4, tol, np.arange(1, npair, 2))
        assert ka + kb == kept
        np.testing.assert_allclose(Ja + Jb, Js, atol=1e-14)


def _pair_class_counts(mol):
    ls = [int(x) for x in mol.shell_l]
    n = np.zeros(6, dtype=np.int64)
    for i in range(len(ls)):
        for j in range(i + 1):
            l1, l2 = max(ls[i], ls[j]), min(ls[i], ls[j])
            n[l1 * (l1 + 1) // 2 + l2] += 1
    return n


def test_screen_counts_without_screening_are_combinatorial(w4):
    counts, near = oracle.screen_counts(w4, 0.0, 0.0)
    n = _pair_class_counts(w4)
    for X in range(6):
        for Y in range(X + 1):
            q = X * (X + 1) // 2 + Y
            want = n[X] * (n[X] + 1) // 2 if X == Y else n[X] * n[Y]
            assert counts[q, 0] == want and counts[q, 1] == 0 and counts[q, 2] == 0
    assert near.sum() == 0


def test_screen_counts_match_a_direct_classification():
    """Kept / single / skipped per class from the oracle's C++ loop against the
    same rule applied in Python to its Schwarz matrix, and the kept total against
    the quartets orc_jk computes."""
    mol = molgen.make_molecule(3, 3, seed=21)
    tol, thr = 1e-4, 3e-2
    counts, _ = oracle.screen_counts(mol, tol, thr)
    Q = oracle.schwarz(oracle.Basis(mol))
    ls = [int(x) for x in mol.shell_l]
    pairs = [(i, j) for i in range(len(ls)) for j in range(i + 1)]
    pcls = [max(ls[i], ls[j]) * (max(ls[i], ls[j]) + 1) // 2 + min(ls[i], ls[j]) for i, j in pairs]
    ref = np.zeros((21, 3), dtype=np.int64)
    for a in range(len(pairs)):
        for b in range(a + 1):
            S = Q[pairs[a]] * Q[pairs[b]]
            X, Y = max(pcls[a], pcls[b]), min(pcls[a], pcls[b])
            ref[X * (X + 1) // 2 + Y, 2 if S < tol else (1 if S < thr else 0)] += 1
    assert np.array_equal(counts, ref)
    assert counts[:, 1].sum() > 0 and counts[:, 2].sum() > 0
    _, _, kept = oracle.jk(mol, tol)
    assert counts[:, 0].sum() + counts[:, 1].sum() == kept


def test_gradient_rows_of_selected_atoms():
    """The atom-restricted gradient gives exactly the selected rows of the full one."""
    mol = molgen.make_molecule(2, 2, seed=11)
    G = oracle.grad(mol, 1e-8)
    Gs = oracle.grad(mol, 1e-8, atoms=[1, 3])
    # same terms summed in another order (OpenMP partial sums): rounding only
    np.testing.assert_allclose(Gs[:, [1, 3]], G[:, [1, 3]], rtol=0, atol=1e-12)
    assert np.all(Gs[:, [0, 2]] == 0.0)


# --- erf-attenuated operator erf(omega r12)/r12 ----------------------------------

OMEGA_QUAD_CASES = [QUAD_CASES[0], QUAD_CASES[2], QUAD_CASES[4], QUAD_CASES[5]]


@pytest.mark.parametrize("omega", [0.15, 0.6, 2.5])
@pytest.mark.parametrize("pows", OMEGA_QUAD_CASES)
def test_prim_eri_omega_by_quadrature(pows, omega):
    """The long-range integral is the Coulomb u integral cut at u = omega."""
    rng = np.random.default_rng(sum(sum(p) * (i + 5) for i, p in enumerate(pows)))
    args = _rand_prims(rng, list(pows))
    o = oracle.prim_eri(*args, omega=omega)
    ref = pins.eri_quadrature(*args, omega=omega)
    assert abs(o - ref) <= 1e-11 * max(abs(ref), 1e-6), (o, ref)


def test_prim_eri_omega_limits():
    """omega -> infinity gives 1/r12; omega -> 0 gives (2 omega/sqrt(pi)) S_ab S_cd."""
    rng = np.random.default_rng(31)
    for pows in QUAD_CASES:
        args = _rand_prims(rng, list(pows))
        coul = oracle.prim_eri(*args)
        big = oracle.prim_eri(*args, omega=1e7)
        assert big == pytest.approx(coul, rel=1e-12, abs=1e-15)
        omega = 1e-5
        small = oracle.prim_eri(*args, omega=omega)
        (pa, a, A, pb, b, B, pc, c, C, pd, d, D) = args
        gh = pins._gh_2d(8)
        ovl = 1.0
        for k in range(3):   # u = 0: the bra and ket factors decouple into overlaps
            ovl *= pins._dim_integral(0.0, a, A[k], pa[k], b, B[k], pb[k], c, C[k], pc[k],
                                      d, D[k], pd[k], gh)
        ref = 2.0 * omega / math.sqrt(math.pi) * ovl
        assert small == pytest.approx(ref, rel=1e-8, abs=1e-14 * abs(coul))


def test_omega_quartets_bounded_by_coulomb_schwarz(w4):
    """erf(omega r)/r and erfc(omega r)/r are both positive definite kernels, so
    |(ab|cd)_omega| <= sqrt((ab|ab)_omega (cd|cd)_omega) <= Q_ab Q_cd (the 1/r12
    bounds used for screening), and (ab|ab)_omega grows with omega."""
    b0 = oracle.Basis(w4)
    b1 = oracle.Basis(w4, omega=0.4)
    b2 = oracle.Basis(w4, omega=1.3)
    Q = oracle.schwarz(b0)
    rng = np.random.default_rng(13)
    for _ in range(150):
        A, B, C, D = (int(x) for x in rng.integers(0, w4.n_shells, 4))
        blk = oracle.shell_quartet(b1, A, B, C, D)
        assert np.abs(blk).max() <= Q[A, B] * Q[C, D] * (1 + 1e-12) + 1e-18
    for A in range(0, w4.n_shells, 3):
        B = (A * 5 + 1) % w4.n_shells
        d1 = oracle.shell_quartet(b1, A, B, A, B)
        d2 = oracle.shell_quartet(b2, A, B, A, B)
        d0 = oracle.shell_quartet(b0, A, B, A, B)
        n = d1.shape[0] * d1.shape[1]
        M1, M2, M0 = (x.reshape(n, n) for x in (d1, d2, d0))
        assert np.linalg.eigvalsh(0.5 * (M1 + M1.T)).min() > -1e-12
        assert np.linalg.eigvalsh(0.5 * ((M2 - M1) + (M2 - M1).T)).min() > -1e-12
        assert np.linalg.eigvalsh(0.5 * ((M0 - M2) + (M0 - M2).T)).min() > -1e-12


def test_contracted_omega_quartet_components():
    """Contraction and component order at omega: (dd|pp) of two-primitive shells."""
    ls, omega = (2, 2, 1, 1), 0.45
    mol = _four_centre_basis(2, seed=61)
    shells = [3 * at + l for at, l in enumerate(ls)]
    blk = oracle.shell_quartet(oracle.Basis(mol, omega=omega), *shells)
    for idx in [(0, 0, 0, 0), (5, 3, 2, 1), (1, 4, 0, 2)]:
        comps = [CART[l][i] for l, i in zip(ls, idx)]
        ref = _contracted_by_quadrature(mol, shells, comps, omega=omega)
        assert abs(blk[idx] - ref) <= 1e-11 * max(abs(ref), 1e-6), (idx, blk[idx], ref)


def test_omega_jk_full_tensor_brute_force():
    """Tiny molecule at omega: n^4 tensor from ordered quartets, J/K by einsum,
    screening with the 1/r12 bounds removed by tol = 0."""
    mol = molgen.make_molecule(1, 1, seed=9)
    omega = 0.33
    b = oracle.Basis(mol, omega=omega)
    n, ns = mol.n_bf, mol.n_shells
    bf0 = mol.shell_bf0
    nc = [molgen.ncart(int(l)) for l in mol.shell_l]
    eri = np.zeros((n, n, n, n))
    for A in range(ns):
        for B in range(ns):
            for C in range(ns):
                for D in range(ns):
                    eri[bf0[A]:bf0[A] + nc[A], bf0[B]:bf0[B] + nc[B], bf0[C]:bf0[C] + nc[C],
                        bf0[D]:bf0[D] + nc[D]] = oracle.shell_quartet(b, A, B, C, D)
    Dm = mol.D[0]
    J, K, _ = oracle.jk(mol, 0.0, omega=omega)
    np.testing.assert_allclose(J[0], np.einsum("ijkl,kl->ij", eri, Dm), atol=1e-13, rtol=1e-12)
    np.testing.assert_allclose(K[0], np.einsum("ikjl,kl->ij", eri, Dm), atol=1e-13, rtol=1e-12)
    J0, _, _ = oracle.jk(mol, 0.0)
    assert np.abs(J[0]).max() < np.abs(J0[0]).max()


def test_omega_rejected_by_gradient():
    mol = molgen.make_molecule(1, 1, seed=7)
    with pytest.raises(ValueError, match="omega"):
        oracle.grad(mol, 0.0, omega=0.3)


# --- pure (spherical) d functions --------------------------------------------------

def _cart_overlap_same_centre(l, a):
    """S[c][c'] of x^p y^q z^r exp(-a r^2) components on one centre: products of 1-D
    moments int x^k exp(-2 a x^2) dx by Gauss-Hermite quadrature (exact)."""
    x, w = np.polynomial.hermite.hermgauss(8)
    t = x / math.sqrt(2 * a)
    mom = lambda k: float(w @ t ** k) / math.sqrt(2 * a)   # noqa: E731
    comps = CART[l]
    S = np.zeros((len(comps), len(comps)))
    for i, p in enumerate(comps):
        for j, q in enumerate(comps):
            S[i, j] = np.prod([mom(p[k] + q[k]) for k in range(3)])
    return S


def test_pure_d_functions_orthonormal_and_free_of_s():
    """The five pure d functions have the norm of the xx component, are mutually
    orthogonal and have no overlap with the s-type combination xx + yy + zz."""
    C = oracle.pure_d()
    for a in (0.3, 1.7):
        S = _cart_overlap_same_centre(2, a)
        np.testing.assert_allclose(C.T @ S @ C, S[0, 0] * np.eye(5), rtol=1e-13, atol=1e-14 * S[0, 0])
        r2 = np.array([1.0, 0, 0, 1.0, 0, 1.0])
        np.testing.assert_allclose(r2 @ S @ C, 0.0, atol=1e-14 * S[0, 0])


def test_pure_d_trace_is_rotation_invariant():
    """sum_m (d_m d_m|s s') is unchanged when the molecule is rotated (the five
    functions span a rotation-invariant space with equal norms); the Cartesian sum
    over the six components is not."""
    mol = molgen.make_molecule(2, 2, seed=17)
    rng = np.random.default_rng(4)
    Rm, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    rot = mol.with_xyz(mol.xyz @ Rm.T)
    ls = np.asarray(mol.shell_l)
    d_sh = int(np.where(ls == 2)[0][0])
    s_sh = [int(x) for x in np.where(ls == 0)[0] if mol.shell_atom[x] != mol.shell_atom[d_sh]][:2]
    vals = []
    for pure in (True, False):
        pair = []
        for m in (mol, rot):
            blk = oracle.shell_quartet(oracle.Basis(m, pure=pure), d_sh, d_sh, s_sh[0], s_sh[1])
            pair.append(sum(blk[i, i, 0, 0] for i in range(blk.shape[0])))
        vals.append(pair)
    assert vals[0][1] == pytest.approx(vals[0][0], rel=1e-12)
    assert abs(vals[1][1] - vals[1][0]) > 1e-6 * abs(vals[1][0])


def _pure_transform(mol):
    """Block-diagonal T ([n_cart][n_pure]) with the oracle's pure-d table in the d blocks."""
    C = oracle.pure_d()
    ls = [int(l) for l in mol.shell_l]
    nc = [ncart for ncart in (molgen.ncart(l) for l in ls)]
    npu = [5 if l == 2 else molgen.ncart(l) for l in ls]
    T = np.zeros((sum(nc), sum(npu)))
    r = c = 0
    for l, a, b in zip(ls, nc, npu):
        T[r:r + a, c:c + b] = C if l == 2 else np.eye(a)
        r, c = r + a, c + b
    return T


@pytest.mark.parametrize("tol", [0.0, 1e-6])
def test_pure_jk_equals_the_cartesian_build_transformed(tol):
    """J, K over pure functions (each quartet block transformed, then digested) equal
    T^T J_cart[T D T^T] T, K likewise, for the same screening decisions."""
    mol = molgen.make_molecule(2, 3, seed=19, n_dm=2)
    T = _pure_transform(mol)
    rng = np.random.default_rng(8)
    X = rng.normal(size=(2, T.shape[1], T.shape[1]))
    Dp = X + X.transpose(0, 2, 1)
    Jp, Kp, kept_p = oracle.jk(mol, tol, D=Dp, pure=True)
    Dc = np.einsum("ia,mab,jb->mij", T, Dp, T)
    Jc, Kc, kept_c = oracle.jk(mol, tol, D=Dc)
    assert kept_p == kept_c
    np.testing.assert_allclose(Jp, np.einsum("ia,mij,jb->mab", T, Jc, T), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(Kp, np.einsum("ia,mij,jb->mab", T, Kc, T), rtol=1e-12, atol=1e-12)
    pairs = [(0, 2), (3, 3), (5, 1), (2, 7)]
    bf0 = np.concatenate([[0], np.cumsum([5 if l == 2 else molgen.ncart(int(l)) for l in mol.shell_l])])
    for (m, n), (jb, kb) in zip(pairs, oracle.jk_blocks(mol, tol, pairs, D=Dp, pure=True)):
        np.testing.assert_allclose(jb, Jp[:, bf0[m]:bf0[m + 1], bf0[n]:bf0[n + 1]], rtol=1e-12,
                                   atol=1e-12)
        np.testing.assert_allclose(kb, Kp[:, bf0[m]:bf0[m + 1], bf0[n]:bf0[n + 1]], rtol=1e-12,
                                   atol=1e-12)


def test_pure_basis_rejected_by_gradient():
    mol = molgen.make_molecule(1, 1, seed=7)
    b = oracle.Basis(mol, pure=True)
    assert oracle._load().orc_grad(b.h, 1, oracle._pd(np.zeros((1, b.n_bf, b.n_bf))), 0.0,
                                   oracle._pd(np.zeros((1, b.n_atoms, 3))), 1, -1, None) == -1
