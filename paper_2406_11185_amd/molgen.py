"""Seeded synthetic molecules, basis sets and density matrices.

This module only draws inputs.  It holds none of the integral, digestion or
gradient arithmetic, so both the HIP path and the CPU oracle can consume what
it produces without sharing any of the method's code.

The workloads stand in for the paper's large-molecule scaling study (a protein
in a split-valence polarised basis, section "Benchmarks", scaling subsection):
heavy atoms carry 3 s + 2 p + 1 Cartesian d shell, hydrogens 2 s + 1 p, every
shell contracts 3 primitives.  Exponents and coefficients are synthetic.

Recipe (units: bohr, hartree):
  * rng = numpy.random.default_rng(seed)
  * heavy Z: the 4-atom case uses [8, 8]; otherwise rng.choice([6, 7, 8])
  * sites: m = ceil(N^(1/3)); the first N points of an m x m x m lattice with
    2.8 bohr spacing in lexicographic (i, j, k) order; atoms (heavy first,
    then H) take sites rng.permutation(N); jitter rng.uniform(-0.3, 0.3, (N, 3))
  * shells per atom, in order: heavy s s s p p d, H s s p; for each shell
    alpha0 = rng.uniform(0.1, 0.5), exponents alpha0 * 3**k (k = 0, 1, 2),
    coefficients rng.uniform(0.2, 1.0, 3), scaled so that the contracted
    x^l component has unit self-overlap
  * density: electrons = sum(Z) + n_H, n_occ = electrons // 2,
    C ~ N(0, 1/n_bf) of shape (n_bf, n_occ), D = C C^T
  * extra densities of one geometry: default_rng([seed, j]), j = 0, 1, ...

Cartesian components of a shell with angular momentum l are ordered with
descending powers of x, then y: p = x, y, z; d = xx, xy, xz, yy, yz, zz.
Contraction coefficients multiply unnormalised primitives
x^lx y^ly z^lz exp(-alpha r^2).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

LATTICE_BOHR = 2.8
JITTER_BOHR = 0.3
HEAVY_SHELLS = (0, 0, 0, 1, 1, 2)
H_SHELLS = (0, 0, 1)
NPRIM = 3


def ncart(l: int) -> int:
    return (l + 1) * (l + 2) // 2


@dataclass
class Molecule:
    """Atoms, a segmented Cartesian Gaussian basis and one or more densities."""

    xyz: np.ndarray            # (n_atoms, 3) float64, bohr
    Z: np.ndarray              # (n_atoms,) int32
    shell_atom: np.ndarray     # (n_shells,) int32
    shell_l: np.ndarray        # (n_shells,) int32
    shell_nprim: np.ndarray    # (n_shells,) int32
    shell_prim0: np.ndarray    # (n_shells,) int32
    exps: np.ndarray           # (n_prim_total,) float64
    coefs: np.ndarray          # (n_prim_total,) float64
    D: np.ndarray = field(default=None)  # (n_dm, n_bf, n_bf) float64
    name: str = ""

    @property
    def n_atoms(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def n_shells(self) -> int:
        return int(self.shell_l.shape[0])

    @property
    def n_bf(self) -> int:
        return int(sum(ncart(int(l)) for l in self.shell_l))

    @property
    def shell_bf0(self) -> np.ndarray:
        n = np.array([ncart(int(l)) for l in self.shell_l], dtype=np.int64)
        return np.concatenate([[0], np.cumsum(n)[:-1]]).astype(np.int32)

    def with_xyz(self, xyz: np.ndarray) -> "Molecule":
        """Same basis and densities with the atoms moved (shells follow atoms)."""
        return Molecule(np.ascontiguousarray(xyz, dtype=np.float64), self.Z, self.shell_atom,
                        self.shell_l, self.shell_nprim, self.shell_prim0, self.exps,
                        self.coefs, self.D, self.name)

    def with_D(self, D: np.ndarray) -> "Molecule":
        D = np.asarray(D, dtype=np.float64)
        if D.ndim == 2:
            D = D[None]
        return Molecule(self.xyz, self.Z, self.shell_atom, self.shell_l, self.shell_nprim,
                        self.shell_prim0, self.exps, self.coefs, np.ascontiguousarray(D),
                        self.name)


def _double_factorial(k: int) -> int:
    r = 1
    while k > 1:
        r *= k
        k -= 2
    return r


def normalise(l: int, exps: np.ndarray, coefs: np.ndarray) -> np.ndarray:
    """Scale coefs so that the contracted x^l component has unit self-overlap.

    The overlap of x^l e^{-a r^2} with x^l e^{-b r^2} over all space is
    (2l-1)!! / (2(a+b))^l * (pi/(a+b))^{3/2}.
    """
    s = exps[:, None] + exps[None, :]
    ov = _double_factorial(2 * l - 1) / (2.0 * s) ** l * (math.pi / s) ** 1.5
    norm2 = float(coefs @ ov @ coefs)
    return coefs / math.sqrt(norm2)


def lattice_sites(n: int) -> np.ndarray:
    m = int(math.ceil(round(n ** (1.0 / 3.0), 12)))
    while m ** 3 < n:
        m += 1
    pts = [(i, j, k) for i in range(m) for j in range(m) for k in range(m)]
    return LATTICE_BOHR * np.array(pts[:n], dtype=np.float64)


def make_molecule(n_heavy: int, n_h: int, seed: int, heavy_z=None, name: str = "",
                  n_dm: int = 1) -> Molecule:
    rng = np.random.default_rng(seed)
    if heavy_z is None:
        heavy_z = rng.choice([6, 7, 8], n_heavy)
    Z = np.concatenate([np.asarray(heavy_z, dtype=np.int32), np.ones(n_h, np.int32)])
    n = n_heavy + n_h
    sites = lattice_sites(n)
    perm = rng.permutation(n)
    xyz = sites[perm] + rng.uniform(-JITTER_BOHR, JITTER_BOHR, (n, 3))

    shell_atom, shell_l, exps, coefs = [], [], [], []
    for a in range(n):
        for l in (HEAVY_SHELLS if Z[a] > 1 else H_SHELLS):
            a0 = rng.uniform(0.1, 0.5)
            e = a0 * 3.0 ** np.arange(NPRIM)
            c = normalise(l, e, rng.uniform(0.2, 1.0, NPRIM))
            shell_atom.append(a)
            shell_l.append(l)
            exps.append(e)
            coefs.append(c)
    ns = len(shell_l)
    mol = Molecule(
        xyz=np.ascontiguousarray(xyz),
        Z=Z,
        shell_atom=np.array(shell_atom, np.int32),
        shell_l=np.array(shell_l, np.int32),
        shell_nprim=np.full(ns, NPRIM, np.int32),
        shell_prim0=(NPRIM * np.arange(ns)).astype(np.int32),
        exps=np.concatenate(exps).astype(np.float64),
        coefs=np.concatenate(coefs).astype(np.float64),
        name=name,
    )
    nbf = mol.n_bf
    n_occ = int(Z.sum()) // 2
    Cm = rng.normal(0.0, math.sqrt(1.0 / nbf), (nbf, n_occ))
    Ds = [Cm @ Cm.T]
    if n_dm > 1:
        Ds = [density(nbf, n_occ, np.random.default_rng([seed, j])) for j in range(n_dm)]
    return mol.with_D(np.stack(Ds))


def density(nbf: int, n_occ: int, rng) -> np.ndarray:
    Cm = rng.normal(0.0, math.sqrt(1.0 / nbf), (nbf, n_occ))
    return Cm @ Cm.T


# The five benchmark workloads: (heavy, H, seed, fixed heavy Z, tol, precision, n_dm)
WORKLOADS = {
    "w4": dict(n_heavy=2, n_h=2, seed=0, heavy_z=[8, 8], tol=0.0, precision="fp64", n_dm=1,
               desc="4 atoms, 40 functions, no screening"),
    "w30": dict(n_heavy=12, n_h=18, seed=1, heavy_z=None, tol=1e-10, precision="fp64", n_dm=1,
                desc="30 atoms, 270 functions, tol 1e-10"),
    "w120": dict(n_heavy=48, n_h=72, seed=2, heavy_z=None, tol=1e-10, precision="mixed", n_dm=1,
                 desc="120 atoms, 1080 functions, mixed precision, tol 1e-10"),
    "w30grad": dict(n_heavy=12, n_h=18, seed=1, heavy_z=None, tol=1e-10, precision="fp64",
                    n_dm=1, desc="30-atom gradient"),
    "w200": dict(n_heavy=80, n_h=120, seed=4, heavy_z=None, tol=1e-10, precision="mixed",
                 n_dm=10, desc="200 atoms, 1800 functions, 10 densities, mixed + gradient"),
}


def workload(name: str) -> Molecule:
    w = WORKLOADS[name]
    return make_molecule(w["n_heavy"], w["n_h"], w["seed"], w["heavy_z"], name=name,
                         n_dm=w["n_dm"])


def ragged_molecule(n_heavy: int, n_h: int, seed: int, counts=(1, 2, 4, 8)) -> Molecule:
    """Edge case for the contraction loops: the geometry and density of
    make_molecule, but every shell redrawn with a primitive count taken from
    `counts` (up to the library's maximum of 8), exponents a0 * 3^k."""
    base = make_molecule(n_heavy, n_h, seed)
    rng = np.random.default_rng([seed, 77])
    nps, exps, coefs = [], [], []
    for l in base.shell_l:
        k = int(rng.choice(counts))
        e = rng.uniform(0.1, 0.5) * 3.0 ** np.arange(k)
        nps.append(k)
        exps.append(e)
        coefs.append(normalise(int(l), e, rng.uniform(0.2, 1.0, k)))
    nps = np.array(nps, np.int32)
    return Molecule(xyz=base.xyz, Z=base.Z, shell_atom=base.shell_atom, shell_l=base.shell_l,
                    shell_nprim=nps,
                    shell_prim0=np.concatenate([[0], np.cumsum(nps)[:-1]]).astype(np.int32),
                    exps=np.concatenate(exps).astype(np.float64),
                    coefs=np.concatenate(coefs).astype(np.float64),
                    name=f"r{n_heavy}_{n_h}_{seed}").with_D(base.D)


def small_molecule(n_heavy: int, n_h: int, seed: int, n_dm: int = 1) -> Molecule:
    """Extra parity cases between the named workloads (same recipe)."""
    return make_molecule(n_heavy, n_h, seed, None, name=f"m{n_heavy}_{n_h}_{seed}", n_dm=n_dm)


def single_bin_molecule(n_h: int, seed: int) -> Molecule:
    """Edge case for the launch schedule: the H atoms of make_molecule with only
    their first s shell each, so that every shell pair has the same class and
    primitive count and a build makes exactly one class launch.  The density
    follows the same recipe (one occupied orbital per two functions)."""
    base = make_molecule(0, n_h, seed, heavy_z=[])
    keep = [s for s in range(base.n_shells)
            if base.shell_l[s] == 0 and (s == 0 or base.shell_atom[s - 1] != base.shell_atom[s])]
    keep = np.array(keep, dtype=np.int64)
    rng = np.random.default_rng([seed, 91])
    nbf = len(keep)
    mol = Molecule(xyz=base.xyz, Z=base.Z, shell_atom=base.shell_atom[keep].astype(np.int32),
                   shell_l=base.shell_l[keep].astype(np.int32),
                   shell_nprim=base.shell_nprim[keep].astype(np.int32),
                   shell_prim0=base.shell_prim0[keep].astype(np.int32),
                   exps=base.exps, coefs=base.coefs, name=f"s{n_h}_{seed}")
    return mol.with_D(density(nbf, max(1, nbf // 2), rng))


def atom_grid(mol: Molecule, n_rad: int = 40, n_ang: int = 110, r_scale: float = 1.0):
    """Synthetic integration grid: around each atom, n_rad radial shells at
    r = r_scale x / (1 - x), x = (i + 1/2) / n_rad, times n_ang directions spread
    over the sphere (golden-angle spiral); weight = the shell's volume element
    times 4 pi / n_ang.  Returns (points [n][3], weights [n]).  Input data only:
    no partition of the molecular volume between atoms."""
    x = (np.arange(n_rad) + 0.5) / n_rad
    r = r_scale * x / (1.0 - x)
    dr = r_scale / (1.0 - x) ** 2 / n_rad
    k = np.arange(n_ang) + 0.5
    cos_t = 1.0 - 2.0 * k / n_ang
    sin_t = np.sqrt(1.0 - cos_t ** 2)
    phi = np.pi * (1.0 + 5 ** 0.5) * k
    dirs = np.stack([sin_t * np.cos(phi), sin_t * np.sin(phi), cos_t], axis=1)
    shell_pts = (r[:, None, None] * dirs[None, :, :]).reshape(-1, 3)
    shell_w = np.repeat(4.0 * np.pi * r ** 2 * dr / n_ang, n_ang)
    pts = np.concatenate([shell_pts + a for a in np.asarray(mol.xyz)])
    w = np.tile(shell_w, len(mol.xyz))
    return np.ascontiguousarray(pts), np.ascontiguousarray(w)
