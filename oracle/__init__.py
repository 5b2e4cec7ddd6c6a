"""CPU FP64 oracle for the J/K build and its nuclear gradient (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this package; the library under paper_2406_11185_amd never imports it.  The
arithmetic lives in md_oracle.cpp (McMurchie-Davidson integrals, own Boys
function, plain digestion); this module only marshals numpy arrays.

Parity status of each entry point (what pins it is listed in the tests):
  boys, prim_eri, shell_quartet, schwarz, jk, jk_blocks, jk_bra_sample, grad,
  screen_counts  -- pinned (the erf(omega r12)/r12 form of prim_eri, shell_quartet,
  jk and jk_blocks as well, and their pure-d form: pure_d, shell_quartet, jk,
  jk_blocks)
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.orc_basis_new.restype = ctypes.c_void_p
    lib.orc_basis_new.argtypes = [ctypes.c_int, _dp, ctypes.c_int, _ip, _ip, _ip, _ip, _dp, _dp]
    lib.orc_basis_free.argtypes = [ctypes.c_void_p]
    lib.orc_boys.argtypes = [ctypes.c_int, ctypes.c_double, _dp]
    lib.orc_prim_eri.restype = ctypes.c_double
    lib.orc_prim_eri.argtypes = [_ip, ctypes.c_double, _dp] * 4
    lib.orc_prim_eri_omega.restype = ctypes.c_double
    lib.orc_prim_eri_omega.argtypes = [_ip, ctypes.c_double, _dp] * 4 + [ctypes.c_double]
    lib.orc_basis_set_omega.argtypes = [ctypes.c_void_p, ctypes.c_double]
    lib.orc_basis_set_pure.argtypes = [ctypes.c_void_p, ctypes.c_int]
    lib.orc_n_bf.argtypes = [ctypes.c_void_p]
    lib.orc_pure_d.argtypes = [_dp]
    lib.orc_shell_quartet.argtypes = [ctypes.c_void_p] + [ctypes.c_int] * 4 + [_dp]
    lib.orc_schwarz.argtypes = [ctypes.c_void_p, _dp]
    lib.orc_jk.restype = ctypes.c_longlong
    lib.orc_jk.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp, ctypes.c_double, _dp, _dp,
                           ctypes.c_int]
    lib.orc_jk_blocks.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp, ctypes.c_double,
                                  ctypes.c_int, _ip, _ip, _dp, _dp, ctypes.c_int]
    lib.orc_grad.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp, ctypes.c_double, _dp,
                             ctypes.c_int, ctypes.c_longlong, _ip]
    _llp = ctypes.POINTER(ctypes.c_longlong)
    lib.orc_screen_counts.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double, _llp,
                                      _llp]
    lib.orc_jk_bra_sample.restype = ctypes.c_longlong
    lib.orc_jk_bra_sample.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp, ctypes.c_double,
                                      ctypes.c_int, _ip, _dp, _dp, ctypes.c_int]
    _lib = lib
    return lib


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _pd(a):
    return a.ctypes.data_as(_dp)


def _pi(a):
    return a.ctypes.data_as(_ip)


def ncart(l):
    return (l + 1) * (l + 2) // 2


class Basis:
    """Oracle-side copy of a basis (any object with the molgen.Molecule fields).
    omega > 0: its integrals are those of erf(omega r12)/r12.  pure: d shells carry
    the five pure functions of pure_d() (basis functions renumbered)."""

    def __init__(self, mol, omega: float = 0.0, pure: bool = False):
        lib = _load()
        self._keep = [_d(mol.xyz), _i(mol.shell_atom), _i(mol.shell_l), _i(mol.shell_nprim),
                      _i(mol.shell_prim0), _d(mol.exps), _d(mol.coefs)]
        x, sa, sl, sn, sp, e, c = self._keep
        self.n_atoms = x.shape[0]
        self.shell_l = sl
        self.n_bf = int(sum(ncart(int(l)) for l in sl))
        self.h = lib.orc_basis_new(self.n_atoms, _pd(x), sl.shape[0], _pi(sa), _pi(sl), _pi(sn),
                                   _pi(sp), _pd(e), _pd(c))
        if omega and lib.orc_basis_set_omega(self.h, float(omega)) != 0:
            raise ValueError("omega must be finite and >= 0")
        self.pure = bool(pure)
        if self.pure:
            lib.orc_basis_set_pure(self.h, 1)
            self.n_bf = int(lib.orc_n_bf(self.h))

    def nfun(self, s: int) -> int:
        l = int(self.shell_l[s])
        return 5 if self.pure and l == 2 else ncart(l)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.orc_basis_free(self.h)
            self.h = None


def boys(nmax: int, T: float) -> np.ndarray:
    F = np.zeros(nmax + 1)
    if _load().orc_boys(nmax, float(T), _pd(F)) != 0:
        raise ValueError("bad Boys arguments")
    return F


def prim_eri(pa, a, A, pb, b, B, pc, c, C, pd, d, D, omega: float = 0.0) -> float:
    """Primitive integral with unit coefficients for Cartesian powers pa..pd
    (omega > 0: of erf(omega r12)/r12)."""
    keep = []
    args = []
    for p, e, X in ((pa, a, A), (pb, b, B), (pc, c, C), (pd, d, D)):
        pp, XX = _i(p), _d(X)
        keep += [pp, XX]
        args += [_pi(pp), float(e), _pd(XX)]
    if omega:
        return float(_load().orc_prim_eri_omega(*args, float(omega)))
    return float(_load().orc_prim_eri(*args))


def pure_d() -> np.ndarray:
    """C[c][m]: coefficient of Cartesian component c (xx, xy, xz, yy, yz, zz) in the
    pure d function m (m = -2..2)."""
    C = np.zeros((6, 5))
    _load().orc_pure_d(_pd(C))
    return C


def shell_quartet(basis: Basis, A: int, B: int, C: int, D: int) -> np.ndarray:
    """Contracted block over the shells' functions (pure d where the basis has them)."""
    shape = (basis.nfun(A), basis.nfun(B), basis.nfun(C), basis.nfun(D))
    out = np.zeros(shape)
    _load().orc_shell_quartet(basis.h, A, B, C, D, _pd(out))
    return out


def schwarz(basis: Basis) -> np.ndarray:
    ns = basis.shell_l.shape[0]
    Q = np.zeros((ns, ns))
    _load().orc_schwarz(basis.h, _pd(Q))
    return Q


def _dm(D):
    D = _d(D)
    if D.ndim == 2:
        D = D[None]
    return np.ascontiguousarray(D)


def _dm_for(b: Basis, mol, D):
    D = _dm(mol.D if D is None else D)
    if D.shape[1:] != (b.n_bf, b.n_bf):
        raise ValueError(f"D must be [n_dm][{b.n_bf}][{b.n_bf}] for this basis")
    return D


def jk(mol, tol: float, D=None, nthreads: int = 0, omega: float = 0.0, pure: bool = False):
    """Full J, K ([n_dm][n][n]) and the number of quartets kept by screening
    (omega > 0: of erf(omega r12)/r12, screened with the 1/r12 bounds; pure: over
    the pure-d basis, D given in it)."""
    b = Basis(mol, omega, pure)
    D = _dm_for(b, mol, D)
    J = np.zeros_like(D)
    K = np.zeros_like(D)
    kept = _load().orc_jk(b.h, D.shape[0], _pd(D), float(tol), _pd(J), _pd(K), nthreads)
    return J, K, int(kept)


def jk_blocks(mol, tol: float, pairs, D=None, nthreads: int = 0, omega: float = 0.0,
              pure: bool = False):
    """J and K blocks of the shell pairs (M, N) by the plain definitions."""
    b = Basis(mol, omega, pure)
    D = _dm_for(b, mol, D)
    sM = _i([p[0] for p in pairs])
    sN = _i([p[1] for p in pairs])
    sizes = [D.shape[0] * b.nfun(m) * b.nfun(n) for m, n in pairs]
    Jo = np.zeros(sum(sizes))
    Ko = np.zeros(sum(sizes))
    _load().orc_jk_blocks(b.h, D.shape[0], _pd(D), float(tol), len(pairs), _pi(sM), _pi(sN),
                          _pd(Jo), _pd(Ko), nthreads)
    out, o = [], 0
    for (m, n), s in zip(pairs, sizes):
        shp = (D.shape[0], b.nfun(m), b.nfun(n))
        out.append((Jo[o:o + s].reshape(shp), Ko[o:o + s].reshape(shp)))
        o += s
    return out


def grad(mol, tol: float, D=None, nthreads: int = 0, bra_pairs: int = -1, atoms=None,
         omega: float = 0.0):
    """dE/dR ([n_dm][n_atoms][3]) of E = 1/2 tr(DJ) - 1/4 tr(DK) at fixed D.

    atoms: optional list of atom indices; only their rows are computed (exactly),
    the other rows are left zero.  Only the 1/r12 operator (omega = 0) has a
    gradient here; omega > 0 raises ValueError."""
    b = Basis(mol, omega)
    D = _dm(mol.D if D is None else D)
    G = np.zeros((D.shape[0], b.n_atoms, 3))
    sel = None
    if atoms is not None:
        sel = np.zeros(b.n_atoms, dtype=np.int32)
        sel[np.asarray(atoms, dtype=np.int64)] = 1
    rc = _load().orc_grad(b.h, D.shape[0], _pd(D), float(tol), _pd(G), nthreads, bra_pairs,
                          _pi(sel) if sel is not None else None)
    if rc != 0:
        raise ValueError("oracle gradient: unsupported number of densities or omega")
    return G


def jk_bra_sample(mol, tol: float, bra_idx, D=None, nthreads: int = 0):
    """Unsymmetrised J/K contributions of the listed unique bra pairs (timing leg)."""
    b = Basis(mol)
    D = _dm(mol.D if D is None else D)
    J = np.zeros_like(D)
    K = np.zeros_like(D)
    idx = _i(bra_idx)
    kept = _load().orc_jk_bra_sample(b.h, D.shape[0], _pd(D), float(tol), idx.shape[0],
                                     _pi(idx), _pd(J), _pd(K), nthreads)
    return J, K, int(kept)


def screen_counts(mol, tol: float, thr: float = 0.0):
    """Per quartet class (index X(X+1)/2 + Y over pair classes ss, ps, pp, ds, dp, dd):
    counts [21][3] of double-precision (S >= thr), single-precision (tol <= S < thr)
    and skipped (S < tol) unique quartets, and near [21], the quartets whose bound S
    is within a relative 1e-12 of tol or thr.  thr = 0: every kept quartet counts
    as double precision."""
    b = Basis(mol)
    counts = np.zeros((21, 3), dtype=np.int64)
    near = np.zeros(21, dtype=np.int64)
    llp = ctypes.POINTER(ctypes.c_longlong)
    _load().orc_screen_counts(b.h, float(tol), float(thr), counts.ctypes.data_as(llp),
                              near.ctypes.data_as(llp))
    return counts, near


def energy(J, K, D):
    """E_J = 1/2 tr(DJ), E_K = 1/4 tr(DK) per density."""
    D = _dm(D)
    EJ = 0.5 * np.einsum("mij,mij->m", D, J)
    EK = 0.25 * np.einsum("mij,mij->m", D, K)
    return EJ, EK
