"""ctypes binding of libjk.so (argument marshalling only).

The names mirror the C ABI in include/jk.h: jk_opts_default, jk_ctx_create,
jk_ctx_destroy, jk_validate_basis, jk_build, jk_build_noalloc, jk_grad,
jk_get_stats, jk_last_error.  All arithmetic runs in the library's HIP kernels; PyTorch only
supplies device memory and the current stream.  If libjk.so is missing the
import fails loudly -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libjk.so")

JK_OK, JK_EINVAL, JK_EUNSUPPORTED, JK_ENOMEM, JK_EHIP = 0, 1, 2, 3, 4
JK_FP64, JK_MIXED = 0, 1
JK_NCLASS = 21
JK_MAX_NDM = 16
ERR_NAMES = {1: "JK_EINVAL", 2: "JK_EUNSUPPORTED", 3: "JK_ENOMEM", 4: "JK_EHIP"}

EXPORTS = ["jk_opts_default", "jk_ctx_create", "jk_ctx_destroy", "jk_validate_basis", "jk_build",
           "jk_build_noalloc", "jk_grad", "jk_get_stats", "jk_last_error", "jk_pure_count",
           "jk_pure_to_cart", "jk_cart_to_pure", "jk_scf_create", "jk_scf_destroy", "jk_scf_diag",
           "jk_scf_diis", "jk_scf_diis_reset", "jk_xc_rho", "jk_xc_vmat", "jk_xc_rho_gga",
           "jk_xc_vmat_gga"]


class JkError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERR_NAMES.get(code, code)}: {msg}")
        self.code = code


class jk_basis(ctypes.Structure):
    _fields_ = [("n_atoms", ctypes.c_int32), ("xyz", ctypes.POINTER(ctypes.c_double)),
                ("n_shells", ctypes.c_int32), ("shell_atom", ctypes.POINTER(ctypes.c_int32)),
                ("shell_l", ctypes.POINTER(ctypes.c_int32)),
                ("shell_nprim", ctypes.POINTER(ctypes.c_int32)),
                ("shell_prim0", ctypes.POINTER(ctypes.c_int32)),
                ("exps", ctypes.POINTER(ctypes.c_double)),
                ("coefs", ctypes.POINTER(ctypes.c_double))]


class jk_opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("fp32_below", ctypes.c_double),
                ("boys_fp64_T", ctypes.c_double), ("n_dm", ctypes.c_int32),
                ("deterministic", ctypes.c_int32), ("timing", ctypes.c_int32),
                ("max_scratch_bytes", ctypes.c_uint64), ("acc_copies", ctypes.c_int32),
                ("serial", ctypes.c_int32), ("reuse_setup", ctypes.c_int32),
                ("energy", ctypes.c_void_p),
                ("dEdD", ctypes.c_void_p), ("omega", ctypes.c_double)]


class jk_stats(ctypes.Structure):
    _fields_ = [("quartets_fp64", ctypes.c_int64 * JK_NCLASS),
                ("quartets_fp32", ctypes.c_int64 * JK_NCLASS),
                ("quartets_skipped", ctypes.c_int64), ("n_pairs", ctypes.c_int64),
                ("work_items", ctypes.c_int64),
                ("ms_kernel_fp64", ctypes.c_double * JK_NCLASS),
                ("ms_kernel_fp32", ctypes.c_double * JK_NCLASS),
                ("ms_setup", ctypes.c_double), ("ms_total", ctypes.c_double),
                ("launches_fp64", ctypes.c_int32 * JK_NCLASS),
                ("launches_fp32", ctypes.c_int32 * JK_NCLASS),
                ("class_l", (ctypes.c_int32 * 4) * JK_NCLASS), ("setup_reused", ctypes.c_int32)]


_lib = None


def load():
    """Load libjk.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run python -m paper_2406_11185_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    lib.jk_opts_default.argtypes = [ctypes.POINTER(jk_opts)]
    lib.jk_ctx_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int]
    lib.jk_ctx_destroy.argtypes = [vp]
    lib.jk_validate_basis.argtypes = [ctypes.POINTER(jk_basis), ctypes.POINTER(ctypes.c_int32)]
    lib.jk_build.argtypes = [vp, ctypes.POINTER(jk_basis), vp, vp, vp, ctypes.c_double,
                             ctypes.POINTER(jk_opts), vp]
    lib.jk_build_noalloc.argtypes = lib.jk_build.argtypes
    lib.jk_grad.argtypes = [vp, ctypes.POINTER(jk_basis), vp, vp, ctypes.c_double,
                            ctypes.POINTER(jk_opts), vp]
    lib.jk_get_stats.argtypes = [vp, ctypes.POINTER(jk_stats)]
    lib.jk_last_error.argtypes = [vp]
    lib.jk_last_error.restype = ctypes.c_char_p
    lib.jk_pure_count.argtypes = [ctypes.POINTER(jk_basis), ctypes.POINTER(ctypes.c_int32)]
    lib.jk_pure_to_cart.argtypes = [ctypes.POINTER(jk_basis), ctypes.c_int32, vp, vp, vp]
    lib.jk_cart_to_pure.argtypes = lib.jk_pure_to_cart.argtypes
    lib.jk_scf_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.c_int32, ctypes.c_int32]
    lib.jk_scf_destroy.argtypes = [vp]
    lib.jk_scf_diag.argtypes = [vp, vp, vp, ctypes.c_int32, vp, vp, vp, vp]
    lib.jk_scf_diis.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    lib.jk_scf_diis_reset.argtypes = [vp]
    lib.jk_xc_rho.argtypes = [ctypes.POINTER(jk_basis), vp, ctypes.c_int32, vp, ctypes.c_int32,
                              ctypes.c_double, vp, vp, vp]
    lib.jk_xc_vmat.argtypes = [ctypes.POINTER(jk_basis), vp, ctypes.c_int32, vp, ctypes.c_double,
                               vp, vp, vp]
    lib.jk_xc_rho_gga.argtypes = [ctypes.POINTER(jk_basis), vp, ctypes.c_int32, vp, ctypes.c_int32,
                                  ctypes.c_double, vp, vp, vp]
    lib.jk_xc_vmat_gga.argtypes = [ctypes.POINTER(jk_basis), vp, ctypes.c_int32, vp, vp,
                                   ctypes.c_double, vp, vp]
    _lib = lib
    return lib


class Basis:
    """Host arrays of a molecule's basis (fields as in molgen.Molecule) and the C struct."""

    def __init__(self, mol):
        self.xyz = np.ascontiguousarray(mol.xyz, dtype=np.float64)
        self.shell_atom = np.ascontiguousarray(mol.shell_atom, dtype=np.int32)
        self.shell_l = np.ascontiguousarray(mol.shell_l, dtype=np.int32)
        self.shell_nprim = np.ascontiguousarray(mol.shell_nprim, dtype=np.int32)
        self.shell_prim0 = np.ascontiguousarray(mol.shell_prim0, dtype=np.int32)
        self.exps = np.ascontiguousarray(mol.exps, dtype=np.float64)
        self.coefs = np.ascontiguousarray(mol.coefs, dtype=np.float64)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        self.c = jk_basis(self.xyz.shape[0], self.xyz.ctypes.data_as(dp),
                          self.shell_l.shape[0], self.shell_atom.ctypes.data_as(ip),
                          self.shell_l.ctypes.data_as(ip), self.shell_nprim.ctypes.data_as(ip),
                          self.shell_prim0.ctypes.data_as(ip), self.exps.ctypes.data_as(dp),
                          self.coefs.ctypes.data_as(dp))

    @property
    def n_atoms(self):
        return int(self.xyz.shape[0])


def jk_opts_default() -> jk_opts:
    o = jk_opts()
    load().jk_opts_default(ctypes.byref(o))
    return o


def make_opts(precision="fp64", fp32_below=1e-4, n_dm=1, timing=False, boys_fp64_T=30.0,
              max_scratch_bytes=0, deterministic=0, acc_copies=0, serial=False, energy=None,
              dEdD=None, reuse_setup=False, omega=0.0) -> jk_opts:
    """jk_opts from keywords; energy / dEdD are float64 device tensors (or None);
    omega > 0 selects the erf(omega r12)/r12 integrals."""
    o = jk_opts_default()
    o.precision = {"fp64": JK_FP64, "mixed": JK_MIXED}[precision] if isinstance(precision, str) \
        else int(precision)
    o.fp32_below = float(fp32_below)
    o.n_dm = int(n_dm)
    o.timing = 1 if timing else 0
    o.boys_fp64_T = float(boys_fp64_T)
    o.max_scratch_bytes = int(max_scratch_bytes)
    o.deterministic = int(deterministic)
    o.acc_copies = int(acc_copies)
    o.serial = 1 if serial else 0
    o.reuse_setup = 1 if reuse_setup else 0
    o.energy = energy.data_ptr() if energy is not None else None
    o.dEdD = dEdD.data_ptr() if dEdD is not None else None
    o.omega = float(omega)
    return o


def jk_validate_basis(basis: Basis) -> int:
    n = ctypes.c_int32(0)
    rc = load().jk_validate_basis(ctypes.byref(basis.c), ctypes.byref(n))
    if rc != JK_OK:
        raise JkError(rc, "invalid basis")
    return int(n.value)


def jk_last_error(ctx) -> str:
    h = ctx.h if isinstance(ctx, Context) else ctx
    return load().jk_last_error(h).decode()


class Context:
    """Owns a jk_ctx on one device."""

    def __init__(self, device: int = 0):
        lib = load()
        h = ctypes.c_void_p()
        rc = lib.jk_ctx_create(ctypes.byref(h), int(device))
        if rc != JK_OK:
            raise JkError(rc, lib.jk_last_error(None).decode())
        self.h = h
        self.device = device

    def close(self):
        if getattr(self, "h", None):
            load().jk_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != JK_OK:
            raise JkError(rc, jk_last_error(self))

    def stats(self) -> jk_stats:
        st = jk_stats()
        self._check(load().jk_get_stats(self.h, ctypes.byref(st)))
        return st


_default_ctx = {}


def default_context(device: int = 0) -> Context:
    if device not in _default_ctx:
        _default_ctx[device] = Context(device)
    return _default_ctx[device]


def _stream_ptr(torch, device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _check_dev(t, shape, name):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
            and t.is_contiguous() and tuple(t.shape) == tuple(shape)):
        raise ValueError(f"{name}: expected a contiguous float64 CUDA tensor of shape {shape}")


def jk_build(ctx: Context, basis: Basis, D, J, K, tol: float, opts: jk_opts | None = None,
             stream=None) -> None:
    """Direct binding: D, J, K are float64 device tensors [n_dm][n][n]."""
    import torch
    s = stream if stream is not None else _stream_ptr(torch, D.device)
    rc = load().jk_build(ctx.h, ctypes.byref(basis.c), ctypes.c_void_p(D.data_ptr()),
                         ctypes.c_void_p(J.data_ptr()), ctypes.c_void_p(K.data_ptr()),
                         float(tol), ctypes.byref(opts) if opts is not None else None, s)
    ctx._check(rc)


def jk_build_noalloc(ctx: Context, basis: Basis, D, J, K, tol: float,
                     opts: jk_opts | None = None, stream=None) -> None:
    """jk_build without any allocation in the call (static device scratch)."""
    import torch
    s = stream if stream is not None else _stream_ptr(torch, D.device)
    rc = load().jk_build_noalloc(ctx.h, ctypes.byref(basis.c), ctypes.c_void_p(D.data_ptr()),
                                 ctypes.c_void_p(J.data_ptr()), ctypes.c_void_p(K.data_ptr()),
                                 float(tol), ctypes.byref(opts) if opts is not None else None, s)
    ctx._check(rc)


def jk_pure_count(basis: Basis) -> int:
    n = ctypes.c_int32(0)
    rc = load().jk_pure_count(ctypes.byref(basis.c), ctypes.byref(n))
    if rc != JK_OK:
        raise JkError(rc, "invalid basis")
    return int(n.value)


def _change_basis(fn, basis: Basis, X, Y, stream):
    import torch
    s = stream if stream is not None else _stream_ptr(torch, X.device)
    rc = fn(ctypes.byref(basis.c), int(X.shape[0]), ctypes.c_void_p(X.data_ptr()),
            ctypes.c_void_p(Y.data_ptr()), s)
    if rc != JK_OK:
        raise JkError(rc, "change of basis between pure and Cartesian functions")


def jk_pure_to_cart(basis: Basis, X_pure, X_cart, stream=None) -> None:
    """X_cart = T X_pure T^T (device tensors [n_dm][n_pure][n_pure] -> [n_dm][n][n])."""
    n, npu = jk_validate_basis(basis), jk_pure_count(basis)
    _check_dev(X_pure, (X_pure.shape[0], npu, npu), "X_pure")
    _check_dev(X_cart, (X_pure.shape[0], n, n), "X_cart")
    _change_basis(load().jk_pure_to_cart, basis, X_pure, X_cart, stream)


def jk_cart_to_pure(basis: Basis, X_cart, X_pure, stream=None) -> None:
    """X_pure = T^T X_cart T (device tensors [n_dm][n][n] -> [n_dm][n_pure][n_pure])."""
    n, npu = jk_validate_basis(basis), jk_pure_count(basis)
    _check_dev(X_cart, (X_cart.shape[0], n, n), "X_cart")
    _check_dev(X_pure, (X_cart.shape[0], npu, npu), "X_pure")
    _change_basis(load().jk_cart_to_pure, basis, X_cart, X_pure, stream)


class ScfSteps:
    """A jk_scf handle: Roothaan diagonalisation and DIIS on the GPU for [n][n]
    float64 CUDA tensors (jk_scf_diag, jk_scf_diis)."""

    def __init__(self, n: int, depth: int = 8, device: int = 0):
        h = ctypes.c_void_p()
        rc = load().jk_scf_create(ctypes.byref(h), int(device), int(n), int(depth))
        if rc != JK_OK:
            raise JkError(rc, "jk_scf_create")
        self.h, self.n, self.device = h, int(n), int(device)

    def close(self):
        if getattr(self, "h", None):
            load().jk_scf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def diag(self, F, S, n_occ: int, vectors: bool = True, density: bool = True):
        """(eps [n], C [n][n] with row j = orbital j or None, D or None)."""
        import torch
        n = self.n
        _check_dev(F, (n, n), "F")
        _check_dev(S, (n, n), "S")
        eps = torch.empty(n, dtype=torch.float64, device=F.device)
        C = torch.empty_like(F) if vectors else None
        D = torch.empty_like(F) if density else None
        ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None  # noqa: E731
        rc = load().jk_scf_diag(self.h, ptr(F), ptr(S), int(n_occ), ptr(C), ptr(eps), ptr(D),
                                _stream_ptr(torch, F.device))
        if rc != JK_OK:
            raise JkError(rc, "jk_scf_diag")
        return eps, C, D

    def diis(self, F, D, S):
        """(extrapolated F, max |F D S - S D F| as a 1-element device tensor)."""
        import torch
        n = self.n
        for t, name in ((F, "F"), (D, "D"), (S, "S")):
            _check_dev(t, (n, n), name)
        Fo = torch.empty_like(F)
        err = torch.empty(1, dtype=torch.float64, device=F.device)
        rc = load().jk_scf_diis(self.h, ctypes.c_void_p(F.data_ptr()), ctypes.c_void_p(D.data_ptr()),
                                ctypes.c_void_p(S.data_ptr()), ctypes.c_void_p(Fo.data_ptr()),
                                ctypes.c_void_p(err.data_ptr()), _stream_ptr(torch, F.device))
        if rc != JK_OK:
            raise JkError(rc, "jk_scf_diis")
        return Fo, err

    def reset(self):
        load().jk_scf_diis_reset(self.h)


def xc_rho(mol, grid, D, eps: float = 1e-12, tiles=None):
    """Density on the grid points (jk_xc_rho): grid [n_grid][3], D [n][n] or
    [n_dm][n][n] float64 CUDA tensors; returns [n_grid] or [n_dm][n_grid].
    tiles: optional int64 CUDA tensor of one element, incremented by the block
    products run."""
    import torch
    basis = mol if isinstance(mol, Basis) else Basis(mol)
    n = jk_validate_basis(basis)
    squeeze = D.dim() == 2
    Dd = (D.unsqueeze(0) if squeeze else D).contiguous()
    _check_dev(grid, (grid.shape[0], 3), "grid")
    _check_dev(Dd, (Dd.shape[0], n, n), "D")
    rho = torch.empty((Dd.shape[0], grid.shape[0]), dtype=torch.float64, device=grid.device)
    rc = load().jk_xc_rho(ctypes.byref(basis.c), ctypes.c_void_p(grid.data_ptr()),
                          int(grid.shape[0]), ctypes.c_void_p(Dd.data_ptr()), int(Dd.shape[0]),
                          float(eps), ctypes.c_void_p(rho.data_ptr()),
                          ctypes.c_void_p(tiles.data_ptr()) if tiles is not None else None,
                          _stream_ptr(torch, grid.device))
    if rc != JK_OK:
        raise JkError(rc, "jk_xc_rho")
    return rho[0] if squeeze else rho


def xc_vmat(mol, grid, wv, eps: float = 1e-12, tiles=None):
    """V[mu][nu] = sum_g wv[g] phi_mu(g) phi_nu(g) (jk_xc_vmat); float64 CUDA tensors."""
    import torch
    basis = mol if isinstance(mol, Basis) else Basis(mol)
    n = jk_validate_basis(basis)
    _check_dev(grid, (grid.shape[0], 3), "grid")
    _check_dev(wv, (grid.shape[0],), "wv")
    V = torch.empty((n, n), dtype=torch.float64, device=grid.device)
    rc = load().jk_xc_vmat(ctypes.byref(basis.c), ctypes.c_void_p(grid.data_ptr()),
                           int(grid.shape[0]), ctypes.c_void_p(wv.data_ptr()), float(eps),
                           ctypes.c_void_p(V.data_ptr()),
                           ctypes.c_void_p(tiles.data_ptr()) if tiles is not None else None,
                           _stream_ptr(torch, grid.device))
    if rc != JK_OK:
        raise JkError(rc, "jk_xc_vmat")
    return V


def xc_rho_gga(mol, grid, D, eps: float = 1e-12):
    """(rho [n_dm][n_grid], grad rho [n_dm][3][n_grid]) (jk_xc_rho_gga); D [n][n]
    gives [n_grid] and [3][n_grid]."""
    import torch
    basis = mol if isinstance(mol, Basis) else Basis(mol)
    n = jk_validate_basis(basis)
    squeeze = D.dim() == 2
    Dd = (D.unsqueeze(0) if squeeze else D).contiguous()
    _check_dev(grid, (grid.shape[0], 3), "grid")
    _check_dev(Dd, (Dd.shape[0], n, n), "D")
    ng = grid.shape[0]
    rho = torch.empty((Dd.shape[0], ng), dtype=torch.float64, device=grid.device)
    grad = torch.empty((Dd.shape[0], 3, ng), dtype=torch.float64, device=grid.device)
    rc = load().jk_xc_rho_gga(ctypes.byref(basis.c), ctypes.c_void_p(grid.data_ptr()), int(ng),
                              ctypes.c_void_p(Dd.data_ptr()), int(Dd.shape[0]), float(eps),
                              ctypes.c_void_p(rho.data_ptr()), ctypes.c_void_p(grad.data_ptr()),
                              _stream_ptr(torch, grid.device))
    if rc != JK_OK:
        raise JkError(rc, "jk_xc_rho_gga")
    return (rho[0], grad[0]) if squeeze else (rho, grad)


def xc_vmat_gga(mol, grid, wv, wg, eps: float = 1e-12):
    """V with the density-gradient terms (jk_xc_vmat_gga); wv [n_grid], wg [3][n_grid]."""
    import torch
    basis = mol if isinstance(mol, Basis) else Basis(mol)
    n = jk_validate_basis(basis)
    ng = grid.shape[0]
    _check_dev(grid, (ng, 3), "grid")
    _check_dev(wv, (ng,), "wv")
    _check_dev(wg, (3, ng), "wg")
    V = torch.empty((n, n), dtype=torch.float64, device=grid.device)
    rc = load().jk_xc_vmat_gga(ctypes.byref(basis.c), ctypes.c_void_p(grid.data_ptr()), int(ng),
                               ctypes.c_void_p(wv.data_ptr()), ctypes.c_void_p(wg.data_ptr()),
                               float(eps), ctypes.c_void_p(V.data_ptr()),
                               _stream_ptr(torch, grid.device))
    if rc != JK_OK:
        raise JkError(rc, "jk_xc_vmat_gga")
    return V


def jk_grad(ctx: Context, basis: Basis, D, dEdR, tol: float, opts: jk_opts | None = None,
            stream=None) -> None:
    import torch
    s = stream if stream is not None else _stream_ptr(torch, D.device)
    rc = load().jk_grad(ctx.h, ctypes.byref(basis.c), ctypes.c_void_p(D.data_ptr()),
                        ctypes.c_void_p(dEdR.data_ptr()), float(tol),
                        ctypes.byref(opts) if opts is not None else None, s)
    ctx._check(rc)


def jk(mol, D, tol: float, precision: str = "fp64", fp32_below: float = 1e-4,
       timing: bool = False, ctx: Context | None = None, energies: bool = False,
       dEdD: bool = False, pure: bool = False, **opt):
    """J, K for the densities D ([n][n] or [n_dm][n][n] float64 CUDA tensor).

    energies=True adds E ([n_dm][3]: E_J, E_K, E_J - E_K, from the library's
    finalize step); dEdD=True adds dE/dD = J - K/2 (same shape as J).  pure=True:
    D, J, K and dE/dD are over pure d functions (jk_pure_to_cart, jk_build,
    jk_cart_to_pure in turn).  Extra keywords go to make_opts (deterministic,
    acc_copies, serial, omega, ...)."""
    import torch
    basis = mol if isinstance(mol, Basis) else Basis(mol)
    squeeze = D.dim() == 2
    Dd = D.unsqueeze(0) if squeeze else D
    Dd = Dd.contiguous()
    if pure:
        Dp = Dd
        n = jk_validate_basis(basis)
        Dd = torch.empty((Dp.shape[0], n, n), dtype=torch.float64, device=Dp.device)
        jk_pure_to_cart(basis, Dp, Dd)
    n_dm, n = Dd.shape[0], Dd.shape[1]
    _check_dev(Dd, (n_dm, n, n), "D")
    ctx = ctx or default_context(Dd.device.index or 0)
    J = torch.empty_like(Dd)
    K = torch.empty_like(Dd)
    E = torch.empty((n_dm, 3), dtype=torch.float64, device=Dd.device) if energies else None
    G = torch.empty_like(Dd) if dEdD else None
    opts = make_opts(precision, fp32_below, n_dm, timing, energy=E, dEdD=G, **opt)
    jk_build(ctx, basis, Dd, J, K, tol, opts)
    if pure:
        mats = [J, K] + ([G] if dEdD else [])
        for i, X in enumerate(mats):
            Y = torch.empty_like(Dp)
            jk_cart_to_pure(basis, X, Y)
            mats[i] = Y
        J, K = mats[0], mats[1]
        if dEdD:
            G = mats[2]
    out = [J[0], K[0]] if squeeze else [J, K]
    if energies:
        out.append(E[0] if squeeze else E)
    if dEdD:
        out.append(G[0] if squeeze else G)
    return tuple(out)


def grad(mol, D, tol: float, precision: str = "fp64", fp32_below: float = 1e-4,
         ctx: Context | None = None, **opt):
    """dE/dR ([n_atoms][3] or [n_dm][n_atoms][3]) of E = 1/2 tr(DJ) - 1/4 tr(DK)."""
    import torch
    basis = mol if isinstance(mol, Basis) else Basis(mol)
    squeeze = D.dim() == 2
    Dd = (D.unsqueeze(0) if squeeze else D).contiguous()
    n_dm, n = Dd.shape[0], Dd.shape[1]
    _check_dev(Dd, (n_dm, n, n), "D")
    ctx = ctx or default_context(Dd.device.index or 0)
    G = torch.empty((n_dm, basis.n_atoms, 3), dtype=torch.float64, device=Dd.device)
    opts = make_opts(precision, fp32_below, n_dm, **opt)
    jk_grad(ctx, basis, Dd, G, tol, opts)
    return G[0] if squeeze else G


class JKEnergy:
    """E = 1/2 tr(DJ) - 1/4 tr(DK) as a torch.autograd.Function.

    JKEnergy.apply(xyz, D, mol, tol, precision) -> E (0-d tensor, or [n_dm]).
    The forward pass takes E and dE/dD = J - K/2 from jk_build's finalize step;
    the backward pass calls jk_grad (derivative-integral kernels) for dE/dxyz.
    Only the upstream gradient's chain-rule scaling happens here.
    """

    _fn = None

    @classmethod
    def apply(cls, xyz, D, mol, tol: float, precision: str = "fp64"):
        if cls._fn is None:
            cls._fn = _make_jk_energy()
        return cls._fn.apply(xyz, D, mol, tol, precision)


def _make_jk_energy():
    import torch

    class _JKEnergy(torch.autograd.Function):
        @staticmethod
        def forward(ctx, xyz, D, mol, tol, precision):
            moved = mol.with_xyz(xyz.detach().cpu().double().numpy())
            basis = Basis(moved)
            _, _, E, dEdD = jk(basis, D, tol, precision=precision, energies=True, dEdD=True)
            ctx.save_for_backward(D, dEdD)
            ctx.basis = basis
            ctx.tol = tol
            ctx.precision = precision
            ctx.xyz_dev = xyz.device
            return E[..., 2].clone()

        @staticmethod
        def backward(ctx, gE):
            D, dEdD = ctx.saved_tensors
            g_xyz = g_D = None
            scale = gE.reshape(gE.shape + (1, 1)) if gE.dim() else gE
            if ctx.needs_input_grad[0]:
                G = grad(ctx.basis, D, ctx.tol, precision=ctx.precision)
                g_xyz = (G * scale).sum(dim=0) if G.dim() == 3 else G * scale
                g_xyz = g_xyz.to(ctx.xyz_dev)
            if ctx.needs_input_grad[1]:
                g_D = dEdD * scale
            return g_xyz, g_D, None, None, None

    return _JKEnergy
