/* jk.h -- C ABI of the MI355X (gfx950) direct-SCF Coulomb/exchange build.
 *
 * The library evaluates, on one GPU, the Coulomb and exchange matrices of the
 * paper's Kohn-Sham Fock build (arXiv 2406.11185, section "DFT Calculation
 * Flow", Fock-matrix equation):
 *
 *     J[mu][nu] = sum_{lam,sig} D[lam][sig] (mu nu|lam sig)
 *     K[mu][nu] = sum_{lam,sig} D[lam][sig] (mu lam|nu sig)
 *
 * with the electron-repulsion integrals of the "Electron Repulsion Integrals"
 * paragraph ("Key Components Redesign and Implementation"),
 *
 *     (mu nu|lam sig) = double integral phi_mu(r) phi_nu(r) phi_lam(r') phi_sig(r') / |r - r'|,
 *
 * over contracted Cartesian Gaussian shells, Cauchy-Schwarz screening of shell
 * quartets against a tolerance, and the paper's single/double precision
 * dispatch (same paragraph, third item).  K is returned without the hybrid
 * exchange factor c_x (c_x = 1); the energy convention used for the gradient
 * is E = 1/2 tr(D J) - 1/4 tr(D K).
 *
 * Conventions shared by every entry point
 *   - Units: bohr and hartree; exponents in bohr^-2.
 *   - A shell is a segmented contraction of unnormalised primitives
 *     x^lx y^ly z^lz exp(-a r^2) centred on its atom; coefficients multiply
 *     these primitives as given (the library normalises nothing).
 *   - Basis functions are numbered shell by shell, in the order of the shells;
 *     inside a shell the Cartesian components run over descending powers of x,
 *     then y: p = x, y, z; d = xx, xy, xz, yy, yz, zz.
 *   - Matrices are dense, row-major, FP64, [n_dm][n_bf][n_bf].  D must be
 *     symmetric (only the symmetric part enters the results).
 *   - Ownership: the caller owns every pointer.  The basis is host memory and
 *     is read during the call only.  D, J, K and dEdR are DEVICE pointers on the
 *     context's device.  J, K and dEdR are overwritten, never accumulated into.
 *   - Streams: all device work is enqueued on `hip_stream` (a hipStream_t; NULL
 *     means the legacy default stream).  The call returns after the work is
 *     enqueued; results are valid once that stream reaches this point.  The
 *     call itself synchronises the stream once, after the screening step, to
 *     size the integral launches.
 *   - Errors: every function returns JK_OK (0) or a JK_E* code.  All argument
 *     checks run before any device work, so on an argument error the outputs
 *     are untouched.  jk_last_error() returns a message for the last failure on
 *     that context.  No C++ exception crosses this interface.
 *   - Calls on one context must not overlap (the context owns scratch memory).
 */
#ifndef JK_H_
#define JK_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define JK_OK 0
#define JK_EINVAL 1        /* bad argument or basis                                  */
#define JK_EUNSUPPORTED 2  /* valid request outside what the library implements      */
#define JK_ENOMEM 3        /* device memory exhausted or over opts.max_scratch_bytes */
#define JK_EHIP 4          /* a HIP runtime call failed                              */

#define JK_FP64 0   /* every kept quartet in FP64                                         */
#define JK_MIXED 1  /* FP32 integrals where the Schwarz bound is below opts.fp32_below  */

#define JK_MAX_L 2        /* s, p and Cartesian d shells                  */
#define JK_MAX_NPRIM 8    /* primitives per shell                          */
#define JK_MAX_NDM 16     /* densities sharing one pass over the integrals */
#define JK_NCLASS 21      /* canonical shell-quartet classes over s, p, d  */

typedef struct jk_ctx jk_ctx;

/* Molecule and basis (host memory). */
typedef struct {
  int32_t n_atoms;
  const double* xyz;          /* [n_atoms][3] atom positions, bohr                      */
  int32_t n_shells;
  const int32_t* shell_atom;  /* [n_shells] atom carrying the shell, 0..n_atoms-1        */
  const int32_t* shell_l;     /* [n_shells] angular momentum 0..2 (3+ -> JK_EUNSUPPORTED) */
  const int32_t* shell_nprim; /* [n_shells] primitives, 1..JK_MAX_NPRIM                  */
  const int32_t* shell_prim0; /* [n_shells] first primitive in exps/coefs                */
  const double* exps;         /* primitive exponents, > 0                                */
  const double* coefs;        /* contraction coefficients (of unnormalised primitives)   */
} jk_basis;

/* Options.  jk_opts_default() fills the defaults noted here. */
typedef struct {
  int32_t precision;          /* JK_FP64 (default) or JK_MIXED                           */
  double fp32_below;          /* JK_MIXED: quartets with tol <= Q_AB*Q_CD < fp32_below use
                                 FP32 integrals (default 1e-4); FP64 at or above it      */
  double boys_fp64_T;         /* FP32 kernels evaluate F_m(T) in FP64 for T > this value;
                                 0 < value <= 30 (default 30)                            */
  int32_t n_dm;               /* densities in D/J/K (or dEdR), 1..JK_MAX_NDM (default 1) */
  int32_t deterministic;      /* 0 (default): J, K and dE/dR are summed with FP64 device
                                 atomics, so the last bits can differ between runs.
                                 1: every contribution is added as a two-word fixed-point
                                 integer (order-independent sums); results are bitwise
                                 reproducible and agree with mode 0 to ~1e-13 relative.
                                 Every accumulated element and every single contribution
                                 must stay below 2^31 in magnitude.                     */
  int32_t timing;             /* 1: time each integral kernel with HIP events (stats)    */
  uint64_t max_scratch_bytes; /* 0 = no limit; else JK_ENOMEM if more scratch is needed */
  int32_t acc_copies;         /* jk_build: accumulator copies of J and K that the
                                 integral kernels spread their atomic adds over; 0
                                 (default) = the library's choice (up to 8 within 256 MB),
                                 1..8 = exactly that many (1: J and K themselves)        */
  int32_t serial;             /* 1: every class launch goes to the caller's stream in turn,
                                 so each kernel runs alone (default 0: after the largest
                                 launch, the rest are spread over three internal streams) */
  int32_t reuse_setup;        /* 1: reuse the pair data, Schwarz factors, screening ranges
                                 and work items of the previous call on this context when
                                 the basis (every array element), tol, precision and
                                 fp32_below are unchanged (D may change, as between SCF
                                 iterations); any call that sets them up again replaces
                                 the kept ones.  They are written on the stream of the
                                 call that made them: a call on another stream must be
                                 ordered after that call by the caller.  0 (default):
                                 set up on every call.                                   */
  double* energy;             /* jk_build, optional (NULL = not written): DEVICE pointer to
                                 [n_dm][3] receiving E_J = 1/2 tr(D J), E_K = 1/4 tr(D K)
                                 and E = E_J - E_K, summed in a fixed order             */
  double* dEdD;               /* jk_build, optional (NULL = not written): DEVICE pointer to
                                 [n_dm][n_bf][n_bf] receiving dE/dD = J - K/2            */
  double omega;               /* jk_build: 0 (default) = the 1/r12 integrals; omega > 0 =
                                 those of erf(omega r12)/r12 (bohr^-1, finite), the
                                 long-range exchange of range-separated hybrids such as
                                 the paper's omegaB97x runs (section "Benchmarks").
                                 Screening keeps the 1/r12 bounds Q_AB (valid, as
                                 |(ab|cd)_omega| <= Q_AB Q_CD); the setup does not
                                 depend on omega.  jk_grad: JK_EUNSUPPORTED if != 0.  */
} jk_opts;

/* Counters of the last jk_build / jk_grad on a context. */
typedef struct {
  int64_t quartets_fp64[JK_NCLASS];   /* kept quartets computed in FP64, per class        */
  int64_t quartets_fp32[JK_NCLASS];   /* kept quartets computed in FP32, per class        */
  int64_t quartets_skipped;           /* unique quartets dropped by the Schwarz screen    */
  int64_t n_pairs;                    /* unique shell pairs                               */
  int64_t work_items;                 /* (bra pair, ket range) launches units             */
  double ms_kernel_fp64[JK_NCLASS];   /* timing=1: summed kernel time per class (ms)      */
  double ms_kernel_fp32[JK_NCLASS];
  double ms_setup;                    /* timing=1: pair data, bounds, sort, work lists    */
  double ms_total;                    /* timing=1: whole call on the stream               */
  int32_t launches_fp64[JK_NCLASS];   /* integral kernel launches per class               */
  int32_t launches_fp32[JK_NCLASS];
  int32_t class_l[JK_NCLASS][4];      /* (la, lb, lc, ld) of each class index             */
  int32_t setup_reused;               /* 1 if the call reused the kept setup (reuse_setup) */
} jk_stats;

/* Fill `opts` with the defaults.  Returns JK_EINVAL if opts is NULL. */
int jk_opts_default(jk_opts* opts);

/* Create a context on HIP device `device` (allocates the Boys-function tables).
 * On success *out receives the context; on failure *out is set to NULL. */
int jk_ctx_create(jk_ctx** out, int device);

/* Release a context and all device memory it holds.  NULL is accepted. */
int jk_ctx_destroy(jk_ctx* ctx);

/* Check a basis on the host only (no HIP call).  On success, *n_bf_out (if not
 * NULL) receives the number of basis functions.  JK_EUNSUPPORTED for l > 2 or
 * more than JK_MAX_NPRIM primitives; JK_EINVAL for anything malformed. */
int jk_validate_basis(const jk_basis* basis, int32_t* n_bf_out);

/* Coulomb and exchange build ("Electron Repulsion Integrals" paragraph and the
 * Fock-matrix equation of the paper).  For each of the opts->n_dm densities in
 * D ([n_dm][n_bf][n_bf], device), writes J and K (same shape, device).
 * A shell quartet (AB|CD) is computed iff Q_AB * Q_CD >= tol, where
 * Q_AB = sqrt(max over components of (ab|ab)); tol = 0 keeps every quartet.
 * opts may be NULL (defaults). */
int jk_build(jk_ctx* ctx, const jk_basis* basis, const double* D, double* J, double* K,
             double tol, const jk_opts* opts, void* hip_stream);

/* jk_build for callers that cannot allocate memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * arguments, results and kernels as jk_build, but every device buffer of the
 * call is carved from one static device array of 64 MiB that the library holds
 * on each GPU it runs on (until the process ends), and the two small
 * device-to-host copies go through host memory allocated with the context.
 * The call makes no hipMalloc, hipFree or other allocating call.  Returns
 * JK_ENOMEM with a message when the molecule needs more than the 64 MiB (about
 * 300 basis functions with the default options), JK_EUNSUPPORTED for
 * opts->timing = 1.  Every call on a GPU shares that GPU's array and leaves its
 * contents behind; calls that overlap on one GPU (other streams, other
 * contexts, other threads) race and must not be made. */
int jk_build_noalloc(jk_ctx* ctx, const jk_basis* basis, const double* D, double* J, double* K,
                     double tol, const jk_opts* opts, void* hip_stream);

/* Nuclear gradient of E = 1/2 tr(D J) - 1/4 tr(D K) at fixed D (basis functions
 * move with their atoms), under the same screening rule as jk_build: the
 * two-electron part of the single-point force, one of the core tasks in the
 * paper's "Tasks" section.  Writes dEdR ([n_dm][n_atoms][3], device,
 * hartree/bohr).  opts->acc_copies, opts->energy and opts->dEdD are ignored. */
int jk_grad(jk_ctx* ctx, const jk_basis* basis, const double* D, double* dEdR, double tol,
            const jk_opts* opts, void* hip_stream);

/* Pure (spherical) d functions.  The paper's workloads use bases of pure
 * functions ("Benchmarks"); the builds above work on Cartesian shells, and these
 * calls carry matrices between the two bases so that a pure-basis caller can use
 * them: a d shell's five pure functions are the real solid harmonics of degree 2
 * over its Cartesian components (xx, xy, xz, yy, yz, zz), in the order
 *   m = -2: sqrt(3) xy,  m = -1: sqrt(3) yz,  m = 0: zz - (xx + yy)/2,
 *   m = 1: sqrt(3) xz,   m = 2: sqrt(3)/2 (xx - yy),
 * each with the norm of the xx component; s and p shells are the same in both
 * bases.  Pure functions are numbered shell by shell like the Cartesian ones.
 * With T the block-diagonal [n_cart][n_pure] matrix of these coefficients:
 *   jk_pure_to_cart: X_cart = T X_pure T^T  (a pure density -> the D of jk_build)
 *   jk_cart_to_pure: X_pure = T^T X_cart T  (J, K, dE/dD of jk_build -> pure)
 * for each of n_dm (1..JK_MAX_NDM) matrices; energies need no change
 * (tr(P T^T J T) = tr(T P T^T J)).  Input and output are DEVICE pointers
 * ([n_dm][n_pure][n_pure] and [n_dm][n_cart][n_cart], row-major FP64) on the
 * current HIP device and must not overlap; the work is enqueued on hip_stream
 * (NULL = legacy default stream), which the call synchronises once (after a
 * small table is copied to the device).  No method arithmetic beyond this
 * change of basis.  JK_EINVAL for a bad basis, NULL pointers or n_dm out of
 * range; JK_EUNSUPPORTED above 65535 output functions; JK_ENOMEM / JK_EHIP if
 * the table cannot be allocated or a HIP call fails. */
int jk_pure_count(const jk_basis* basis, int32_t* n_pure_out);
int jk_pure_to_cart(const jk_basis* basis, int32_t n_dm, const double* X_pure, double* X_cart,
                    void* hip_stream);
int jk_cart_to_pure(const jk_basis* basis, int32_t n_dm, const double* X_cart, double* X_pure,
                    void* hip_stream);

/* The SCF steps beside the build, on the GPU (paper, "Key Components Redesign and
 * Implementation", SCF-iteration paragraph; "DFT Calculation Flow"): the
 * Roothaan diagonalisation with the closed-shell density, and Pulay's DIIS
 * extrapolation.  A jk_scf handle (one device, one size n, a DIIS history of
 * `depth` pairs) owns a rocBLAS handle and workspace for ~(2 depth + 3) n^2
 * doubles.  All matrices are DEVICE pointers, [n][n] row-major FP64, symmetric
 * where stated; calls on one handle must not overlap; the work is enqueued on
 * hip_stream (NULL = legacy default), and each call synchronises that stream
 * once (to read the solver's status).
 *
 * jk_scf_create: JK_EINVAL unless 1 <= n <= 46340 and 1 <= depth <= 32.
 * jk_scf_diag: solves F C = S C diag(eps) for symmetric F and symmetric
 *   positive-definite S.  eps [n] ascending (required); C [n][n] (optional):
 *   row j = orbital j, S-orthonormal (C S C^T = I); D [n][n] (optional) =
 *   2 sum_{j < n_occ} c_j c_j^T.  JK_EINVAL if S is not positive definite.
 * jk_scf_diis: stores (F, D) with its error e = F D S - S D F (replacing the
 *   oldest pair once depth are stored) and writes F_out = sum_i c_i F_i over the
 *   stored pairs, c minimising |sum_i c_i e_i| with sum_i c_i = 1; if that
 *   system is singular, F_out = F.  err_out (optional, DEVICE, 1 double) =
 *   max |e| of the new pair.  jk_scf_diis_reset empties the history. */
typedef struct jk_scf jk_scf;
int jk_scf_create(jk_scf** out, int device, int32_t n, int32_t depth);
int jk_scf_destroy(jk_scf* scf);
int jk_scf_diag(jk_scf* scf, const double* F, const double* S, int32_t n_occ, double* C,
                double* eps, double* D, void* hip_stream);
int jk_scf_diis(jk_scf* scf, const double* F, const double* D, const double* S, double* F_out,
                double* err_out, void* hip_stream);
int jk_scf_diis_reset(jk_scf* scf);

/* Grid part of the exchange-correlation integration (paper, "Key Components
 * Redesign and Implementation", EXC paragraph): basis-function values on the grid
 * points with distance-based sparsity (a shell is skipped beyond the radius where
 * r^l sum_k |c_k| exp(-a_k r^2) falls below eps), stored in 32 x 32 blocks of
 * functions x points, a block left out when all its values are below eps, and
 * block-sparse matrix products:
 *   jk_xc_rho:  rho[m][g] = sum_{mu,nu} phi_mu(g) D[m][mu][nu] phi_nu(g)
 *   jk_xc_vmat: V[mu][nu] = sum_g wv[g] phi_mu(g) phi_nu(g)   (symmetric)
 * with wv = grid weight times the functional's potential (the functional is the
 * caller's).  grid: DEVICE [n_grid][3] points (bohr); D: DEVICE [n_dm][n_bf][n_bf]
 * (symmetric), rho: DEVICE [n_dm][n_grid]; wv: DEVICE [n_grid]; V: DEVICE
 * [n_bf][n_bf]; Cartesian functions as in jk_build.  eps in (0, 1) (the paper's
 * default 1e-12).  tiles (optional, DEVICE int64, NULL = not written): the number
 * of 32 x 32 x 32 block products the call ran is ADDED to *tiles (2 * 32^3 flops
 * each; zero it first).  Points are processed in batches of 16384; the call allocates its
 * workspace (about n_bf x 16384 doubles, and 8 n_bf^2 more for jk_xc_vmat)
 * stream-ordered on the current device, and
 * synchronises hip_stream once (after copying the shell table).  JK_EINVAL for a bad
 * basis, pointer, count or eps; JK_ENOMEM / JK_EHIP on allocation or HIP failure. */
int jk_xc_rho(const jk_basis* basis, const double* grid, int32_t n_grid, const double* D,
              int32_t n_dm, double eps, double* rho, int64_t* tiles, void* hip_stream);
int jk_xc_vmat(const jk_basis* basis, const double* grid, int32_t n_grid, const double* wv,
               double eps, double* V, int64_t* tiles, void* hip_stream);

/* The same for gradient-corrected functionals (the paper's hybrids are GGA and
 * meta-GGA): with the first derivatives of every basis function (the distance
 * cut-off then also bounds them, and a block is zero when the values and the
 * three derivatives are all below eps),
 *   jk_xc_rho_gga:  rho as above, grad_rho[m][c][g] = 2 sum_{mu,nu} d_c phi_mu(g)
 *                   D[m][mu][nu] phi_nu(g)   (DEVICE [n_dm][3][n_grid])
 *   jk_xc_vmat_gga: V[mu][nu] = sum_g wv[g] phi_mu phi_nu + sum_c wg[c][g]
 *                   (d_c phi_mu phi_nu + phi_mu d_c phi_nu)   (wg DEVICE [3][n_grid]:
 *                   the grid weight times the functional's derivative with respect to
 *                   the density-gradient component c)
 * Workspace four times that of the calls above. */
int jk_xc_rho_gga(const jk_basis* basis, const double* grid, int32_t n_grid, const double* D,
                  int32_t n_dm, double eps, double* rho, double* grad_rho, void* hip_stream);
int jk_xc_vmat_gga(const jk_basis* basis, const double* grid, int32_t n_grid, const double* wv,
                   const double* wg, double eps, double* V, void* hip_stream);

/* Counters of the last successful jk_build / jk_grad.  With opts.timing = 1
 * this waits for the recorded events. */
int jk_get_stats(jk_ctx* ctx, jk_stats* out);

/* Message of the last failure on ctx ("" if none); ctx NULL -> last failure of
 * jk_ctx_create in this thread. */
const char* jk_last_error(const jk_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* JK_H_ */
