// CPU FP64 oracle for the Coulomb/exchange build (test infrastructure only).
//
// This file is the checker, not the product: only the test-suite, the smoke
// check and the benchmark's CPU-baseline leg load it.  It shares no code,
// header, table or constant generator with the HIP library.
//
// What it computes (paper, "Key Components Redesign and Implementation",
// "Electron Repulsion Integrals" paragraph, and the Fock-matrix equation of
// "DFT Calculation Flow"):
//   (mu nu|lam sig) = double integral of phi_mu phi_nu(r) phi_lam phi_sig(r') / |r - r'|
//   J_mu,nu = sum_{lam,sig} D_lam,sig (mu nu|lam sig)
//   K_mu,nu = sum_{lam,sig} D_lam,sig (mu lam|nu sig)        (c_x = 1, sign in E)
//   E = 1/2 tr(D J) - 1/4 tr(D K), and dE/dR at fixed D.
// Shell quartets are skipped when their Cauchy-Schwarz bound Q_AB * Q_CD is
// below the tolerance (same paragraph, mixed-precision item).
//
// The integrals use the McMurchie-Davidson scheme (Hermite expansion
// coefficients E_t^{ij} and Hermite Coulomb integrals R_tuv), a different
// algorithm from the recurrences the GPU path uses.  The Boys function is
// evaluated from its power series (T < 30) or from erf (T >= 30).
//
// Basis convention: a shell is a contraction of unnormalised primitives
// x^lx y^ly z^lz exp(-a r^2) centred on its atom; Cartesian components are
// ordered with descending powers of x then y (xx, xy, xz, yy, yz, zz).
// Optionally (orc_basis_set_pure) a d shell carries the five pure functions of
// pure_d below instead, and D, J, K are over those functions.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <algorithm>
#include <omp.h>

namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;

int ncart(int l) { return (l + 1) * (l + 2) / 2; }

void cart_powers(int l, int idx, int p[3]) {
  int k = 0;
  for (int lx = l; lx >= 0; --lx)
    for (int ly = l - lx; ly >= 0; --ly) {
      if (k == idx) { p[0] = lx; p[1] = ly; p[2] = l - lx - ly; return; }
      ++k;
    }
}

// Boys function F_n(T) for n = 0..nmax.
//   T < 30 : F_nmax from the series e^{-T} sum_i (2T)^i / ((2n+1)(2n+3)...(2n+2i+1)),
//            then downward recursion F_n = (2T F_{n+1} + e^{-T}) / (2n+1).
//   T >= 30: F_0 = (1/2) sqrt(pi/T) erf(sqrt(T)), then upward recursion
//            F_{n+1} = ((2n+1) F_n - e^{-T}) / (2T).
void boys(int nmax, double T, double* F) {
  const double eT = std::exp(-T);
  if (T < 30.0) {
    double term = 1.0 / (2 * nmax + 1), sum = term;
    for (int i = 1; i < 2000; ++i) {
      term *= 2.0 * T / (2 * nmax + 2 * i + 1);
      sum += term;
      if (term < 1e-18 * sum) break;
    }
    F[nmax] = eT * sum;
    for (int n = nmax - 1; n >= 0; --n) F[n] = (2.0 * T * F[n + 1] + eT) / (2 * n + 1);
  } else {
    F[0] = 0.5 * std::sqrt(kPi / T) * std::erf(std::sqrt(T));
    for (int n = 0; n < nmax; ++n) F[n + 1] = ((2 * n + 1) * F[n] - eT) / (2.0 * T);
  }
}

// Hermite expansion coefficients of one Cartesian direction of a Gaussian
// product:  x_A^i x_B^j exp(-a x_A^2 - b x_B^2) = sum_t E[i][j][t] Lambda_t.
struct Herm1D {
  static constexpr int kI = 5;          // powers 0..4 on either centre
  static constexpr int kT = 2 * kI - 1;  // t = 0..8
  int imax = 0, jmax = 0;
  double e[kI][kI][kT];
  double get(int i, int j, int t) const {
    if (t < 0 || t > i + j || i < 0 || j < 0) return 0.0;
    return e[i][j][t];
  }
  void build(int imax_, int jmax_, double a, double b, double Ax, double Bx) {
    imax = imax_; jmax = jmax_;
    const double p = a + b, mu = a * b / p;
    const double Px = (a * Ax + b * Bx) / p;
    const double XPA = Px - Ax, XPB = Px - Bx, XAB = Ax - Bx;
    const double o2p = 1.0 / (2.0 * p);
    e[0][0][0] = std::exp(-mu * XAB * XAB);
    for (int i = 0; i <= imax; ++i) {
      if (i > 0)
        for (int t = 0; t <= i; ++t)
          e[i][0][t] = o2p * get(i - 1, 0, t - 1) + XPA * get(i - 1, 0, t) +
                       (t + 1) * get(i - 1, 0, t + 1);
      for (int j = 1; j <= jmax; ++j)
        for (int t = 0; t <= i + j; ++t)
          e[i][j][t] = o2p * get(i, j - 1, t - 1) + XPB * get(i, j - 1, t) +
                       (t + 1) * get(i, j - 1, t + 1);
    }
  }
};

// Hermite Coulomb integrals R^0_tuv(rho, R_PQ) for t+u+v <= L, built from
// R^n_000 = (-2 rho)^n F_n(rho |PQ|^2) by the Hermite recursion.
struct HermR {
  static constexpr int kD = 13;  // t, u, v, n = 0..12
  int L = 0;
  std::vector<double> r = std::vector<double>((size_t)kD * kD * kD * kD);
  double r0[kD][kD][kD];  // R^0_tuv, the only order the integrals read
  double& at(int n, int t, int u, int v) { return r[((n * kD + t) * kD + u) * kD + v]; }
  double get(int n, int t, int u, int v) {
    if (t < 0 || u < 0 || v < 0) return 0.0;
    return at(n, t, u, v);
  }
  void build(int L_, double rho, double X, double Y, double Z) {
    L = L_;
    double F[32];
    boys(L, rho * (X * X + Y * Y + Z * Z), F);
    double f = 1.0;
    for (int n = 0; n <= L; ++n) { at(n, 0, 0, 0) = f * F[n]; f *= -2.0 * rho; }
    for (int s = 1; s <= L; ++s)
      for (int n = 0; n <= L - s; ++n)
        for (int t = 0; t <= s; ++t)
          for (int u = 0; u <= s - t; ++u) {
            const int v = s - t - u;
            double val;
            if (t > 0)      val = (t - 1) * get(n + 1, t - 2, u, v) + X * get(n + 1, t - 1, u, v);
            else if (u > 0) val = (u - 1) * get(n + 1, t, u - 2, v) + Y * get(n + 1, t, u - 1, v);
            else            val = (v - 1) * get(n + 1, t, u, v - 2) + Z * get(n + 1, t, u, v - 1);
            at(n, t, u, v) = val;
          }
    for (int t = 0; t <= L; ++t)
      for (int u = 0; u <= L - t; ++u)
        for (int v = 0; v <= L - t - u; ++v) r0[t][u][v] = at(0, t, u, v);
  }
};

// One primitive quartet: expansion tables for bra and ket and the R table,
// so that any Cartesian integral with powers within the table limits follows.
struct PrimQuartet {
  Herm1D Eb[3], Ek[3];
  HermR R;
  double pref;
  // omega > 0: the long-range operator erf(omega r12)/r12 instead of 1/r12.  Its
  // Hermite integrals are those of 1/r12 with rho replaced by
  // rho_w = rho omega^2/(omega^2 + rho), times sqrt(rho_w/rho) (the Fourier
  // transform of erf(omega r)/r is that of 1/r times exp(-k^2/(4 omega^2))).
  void build(const int lmax[4], double a, const double* A, double b, const double* B,
             double c, const double* C, double d, const double* D, double omega = 0.0) {
    const double p = a + b, q = c + d;
    double P[3], Q[3];
    for (int k = 0; k < 3; ++k) {
      P[k] = (a * A[k] + b * B[k]) / p;
      Q[k] = (c * C[k] + d * D[k]) / q;
      Eb[k].build(lmax[0], lmax[1], a, b, A[k], B[k]);
      Ek[k].build(lmax[2], lmax[3], c, d, C[k], D[k]);
    }
    const double rho = p * q / (p + q);
    const double s = omega > 0.0 ? omega * omega / (omega * omega + rho) : 1.0;
    R.build(lmax[0] + lmax[1] + lmax[2] + lmax[3], rho * s, P[0] - Q[0], P[1] - Q[1],
            P[2] - Q[2]);
    pref = 2.0 * std::pow(kPi, 2.5) / (p * q * std::sqrt(p + q)) * std::sqrt(s);
  }
  // (a b | c d) for Cartesian powers pa..pd (each [3]); negative power -> 0.
  double eri(const int* pa, const int* pb, const int* pc, const int* pd) {
    for (int k = 0; k < 3; ++k)
      if (pa[k] < 0 || pb[k] < 0 || pc[k] < 0 || pd[k] < 0) return 0.0;
    double s = 0.0;
    for (int t = 0; t <= pa[0] + pb[0]; ++t) {
      const double ex = Eb[0].get(pa[0], pb[0], t);
      for (int u = 0; u <= pa[1] + pb[1]; ++u) {
        const double ey = Eb[1].get(pa[1], pb[1], u);
        for (int v = 0; v <= pa[2] + pb[2]; ++v) {
          const double ez = Eb[2].get(pa[2], pb[2], v);
          double inner = 0.0;
          for (int tt = 0; tt <= pc[0] + pd[0]; ++tt) {
            const double fx = Ek[0].get(pc[0], pd[0], tt);
            for (int uu = 0; uu <= pc[1] + pd[1]; ++uu) {
              const double fy = Ek[1].get(pc[1], pd[1], uu);
              for (int vv = 0; vv <= pc[2] + pd[2]; ++vv) {
                const double fz = Ek[2].get(pc[2], pd[2], vv);
                const double sign = ((tt + uu + vv) & 1) ? -1.0 : 1.0;
                inner += sign * fx * fy * fz * R.r0[t + tt][u + uu][v + vv];
              }
            }
          }
          s += ex * ey * ez * inner;
        }
      }
    }
    return pref * s;
  }
};

// The five pure d functions, real solid harmonics of degree 2 times the shell's
// radial part, written over the Cartesian components (xx, xy, xz, yy, yz, zz), in
// the order m = -2, -1, 0, 1, 2:
//   S(2,-2) = sqrt(3) xy            S(2,-1) = sqrt(3) yz
//   S(2, 0) = zz - (xx + yy)/2      S(2, 1) = sqrt(3) xz
//   S(2, 2) = sqrt(3)/2 (xx - yy)
// Each has the norm of the xx component and they are mutually orthogonal and
// free of the s-type combination xx + yy + zz.  C[c][m] = coefficient of
// Cartesian component c in function m.
void pure_d(double C[6][5]) {
  const double r3 = std::sqrt(3.0);
  for (int c = 0; c < 6; ++c)
    for (int m = 0; m < 5; ++m) C[c][m] = 0.0;
  C[1][0] = r3;                           // xy
  C[4][1] = r3;                           // yz
  C[5][2] = 1.0; C[0][2] = -0.5; C[3][2] = -0.5;
  C[2][3] = r3;                           // xz
  C[0][4] = 0.5 * r3; C[3][4] = -0.5 * r3;
}

struct Basis {
  int n_atoms = 0, n_shells = 0, n_bf = 0;
  double omega = 0.0;   // > 0: integrals of erf(omega r12)/r12 (screening stays Coulomb)
  int pure = 0;         // 1: d shells carry the five pure functions of pure_d
  std::vector<double> xyz;
  std::vector<int> atom, l, nprim, prim0, bf0;
  std::vector<double> exps, coefs;
  const double* center(int s) const { return &xyz[3 * atom[s]]; }
};

int nfun(const Basis& bs, int s) { return bs.pure && bs.l[s] == 2 ? 5 : ncart(bs.l[s]); }

// Coefficient of Cartesian component c in function f of shell s.
double fun_coef(const Basis& bs, int s, int c, int f) {
  if (!(bs.pure && bs.l[s] == 2)) return c == f ? 1.0 : 0.0;
  double C[6][5];
  pure_d(C);
  return C[c][f];
}

// The Cartesian block of shells sh[0..3] over their functions:
//   out[al be ga de] = sum_{abcd} C_A[a][al] C_B[b][be] C_C[c][ga] C_D[d][de] cart[abcd]
// (a copy when no shell has pure functions).
void to_functions(const Basis& bs, const int sh[4], const double* cart, double* out) {
  int nc[4], nf[4];
  for (int k = 0; k < 4; ++k) { nc[k] = ncart(bs.l[sh[k]]); nf[k] = nfun(bs, sh[k]); }
  int o = 0;
  for (int al = 0; al < nf[0]; ++al)
    for (int be = 0; be < nf[1]; ++be)
      for (int ga = 0; ga < nf[2]; ++ga)
        for (int de = 0; de < nf[3]; ++de) {
          double v = 0.0;
          for (int a = 0; a < nc[0]; ++a) {
            const double ca = fun_coef(bs, sh[0], a, al);
            if (ca == 0.0) continue;
            for (int b = 0; b < nc[1]; ++b) {
              const double cb = fun_coef(bs, sh[1], b, be);
              if (cb == 0.0) continue;
              for (int c = 0; c < nc[2]; ++c) {
                const double cc = fun_coef(bs, sh[2], c, ga);
                if (cc == 0.0) continue;
                for (int d = 0; d < nc[3]; ++d) {
                  const double cd = fun_coef(bs, sh[3], d, de);
                  if (cd == 0.0) continue;
                  v += ca * cb * cc * cd * cart[((a * nc[1] + b) * nc[2] + c) * nc[3] + d];
                }
              }
            }
          }
          out[o++] = v;
        }
}

// Contracted Cartesian block (AB|CD), out[((a*nb+b)*nc+c)*nd+d].
void shell_quartet(const Basis& bs, int sA, int sB, int sC, int sD, double* out,
                   PrimQuartet& pq, double omega) {
  const int sh[4] = {sA, sB, sC, sD};
  int n[4], lmax[4];
  for (int k = 0; k < 4; ++k) { lmax[k] = bs.l[sh[k]]; n[k] = ncart(lmax[k]); }
  const int ntot = n[0] * n[1] * n[2] * n[3];
  std::fill(out, out + ntot, 0.0);
  std::vector<int> pw(4 * 6 * 3);
  for (int k = 0; k < 4; ++k)
    for (int i = 0; i < n[k]; ++i) cart_powers(lmax[k], i, &pw[(k * 6 + i) * 3]);
  for (int i = 0; i < bs.nprim[sA]; ++i)
    for (int j = 0; j < bs.nprim[sB]; ++j)
      for (int k = 0; k < bs.nprim[sC]; ++k)
        for (int m = 0; m < bs.nprim[sD]; ++m) {
          const int ia = bs.prim0[sA] + i, ib = bs.prim0[sB] + j;
          const int ic = bs.prim0[sC] + k, id = bs.prim0[sD] + m;
          pq.build(lmax, bs.exps[ia], bs.center(sA), bs.exps[ib], bs.center(sB),
                   bs.exps[ic], bs.center(sC), bs.exps[id], bs.center(sD), omega);
          const double cc = bs.coefs[ia] * bs.coefs[ib] * bs.coefs[ic] * bs.coefs[id];
          int idx = 0;
          for (int a = 0; a < n[0]; ++a)
            for (int b = 0; b < n[1]; ++b)
              for (int c = 0; c < n[2]; ++c)
                for (int d = 0; d < n[3]; ++d)
                  out[idx++] += cc * pq.eri(&pw[(0 * 6 + a) * 3], &pw[(6 + b) * 3],
                                            &pw[(12 + c) * 3], &pw[(18 + d) * 3]);
        }
}

// Q_AB = sqrt(max over components of the diagonal (ab|ab)).
std::vector<double> schwarz(const Basis& bs) {
  const int ns = bs.n_shells;
  std::vector<double> Q((size_t)ns * ns, 0.0);
#pragma omp parallel
  {
    PrimQuartet pq;
    std::vector<double> blk(6 * 6 * 6 * 6);
#pragma omp for schedule(dynamic)
    for (int A = 0; A < ns; ++A)
      for (int B = 0; B <= A; ++B) {
        shell_quartet(bs, A, B, A, B, blk.data(), pq, 0.0);   // Coulomb bound
        const int na = ncart(bs.l[A]), nb = ncart(bs.l[B]);
        double mx = 0.0;
        for (int a = 0; a < na; ++a)
          for (int b = 0; b < nb; ++b) {
            const double v = blk[((a * nb + b) * na + a) * nb + b];
            mx = std::max(mx, v);
          }
        Q[(size_t)A * ns + B] = Q[(size_t)B * ns + A] = std::sqrt(mx);
      }
  }
  return Q;
}

struct PairIdx { int A, B; };

std::vector<PairIdx> unique_pairs(int ns) {
  std::vector<PairIdx> v;
  for (int A = 0; A < ns; ++A)
    for (int B = 0; B <= A; ++B) v.push_back({A, B});
  return v;
}

thread_local char g_err[256] = "";

}  // namespace

extern "C" {

struct orc_basis;  // opaque handle == Basis

void* orc_basis_new(int n_atoms, const double* xyz, int n_shells, const int* shell_atom,
                    const int* shell_l, const int* shell_nprim, const int* shell_prim0,
                    const double* exps, const double* coefs) {
  Basis* b = new Basis;
  b->n_atoms = n_atoms;
  b->n_shells = n_shells;
  b->xyz.assign(xyz, xyz + 3 * n_atoms);
  b->atom.assign(shell_atom, shell_atom + n_shells);
  b->l.assign(shell_l, shell_l + n_shells);
  b->nprim.assign(shell_nprim, shell_nprim + n_shells);
  b->prim0.assign(shell_prim0, shell_prim0 + n_shells);
  int np = 0;
  for (int s = 0; s < n_shells; ++s) np = std::max(np, shell_prim0[s] + shell_nprim[s]);
  b->exps.assign(exps, exps + np);
  b->coefs.assign(coefs, coefs + np);
  b->bf0.resize(n_shells);
  int nbf = 0;
  for (int s = 0; s < n_shells; ++s) { b->bf0[s] = nbf; nbf += ncart(b->l[s]); }
  b->n_bf = nbf;
  return b;
}

void orc_basis_free(void* h) { delete static_cast<Basis*>(h); }

int orc_boys(int nmax, double T, double* F) {
  if (nmax < 0 || nmax > 30 || !(T >= 0.0)) return -1;
  boys(nmax, T, F);
  return 0;
}

// Primitive (unnormalised, unit-coefficient) integral for arbitrary powers.
double orc_prim_eri(const int* pa, double a, const double* A, const int* pb, double b,
                    const double* B, const int* pc, double c, const double* C, const int* pd,
                    double d, const double* D) {
  const int lmax[4] = {pa[0] + pa[1] + pa[2], pb[0] + pb[1] + pb[2], pc[0] + pc[1] + pc[2],
                       pd[0] + pd[1] + pd[2]};
  PrimQuartet pq;
  pq.build(lmax, a, A, b, B, c, C, d, D);
  return pq.eri(pa, pb, pc, pd);
}

// The same for erf(omega r12)/r12 (omega > 0).
double orc_prim_eri_omega(const int* pa, double a, const double* A, const int* pb, double b,
                          const double* B, const int* pc, double c, const double* C,
                          const int* pd, double d, const double* D, double omega) {
  const int lmax[4] = {pa[0] + pa[1] + pa[2], pb[0] + pb[1] + pb[2], pc[0] + pc[1] + pc[2],
                       pd[0] + pd[1] + pd[2]};
  PrimQuartet pq;
  pq.build(lmax, a, A, b, B, c, C, d, D, omega);
  return pq.eri(pa, pb, pc, pd);
}

// Integrals of this basis handle use erf(omega r12)/r12 from here on (omega > 0), or
// 1/r12 (omega = 0); the Schwarz bounds stay those of 1/r12, which bound both.
// d shells with the five pure functions (pure = 1) or the six Cartesian ones
// (pure = 0); renumbers the basis functions.  The gradient and the timing leg
// take Cartesian bases only.
int orc_basis_set_pure(void* h, int pure) {
  if (pure != 0 && pure != 1) return -1;
  Basis& b = *static_cast<Basis*>(h);
  b.pure = pure;
  int nbf = 0;
  for (int s = 0; s < b.n_shells; ++s) { b.bf0[s] = nbf; nbf += nfun(b, s); }
  b.n_bf = nbf;
  return 0;
}

int orc_n_bf(void* h) { return static_cast<Basis*>(h)->n_bf; }

// The pure-d coefficient table, C[c][m] row-major [6][5].
void orc_pure_d(double* out) {
  double C[6][5];
  pure_d(C);
  for (int c = 0; c < 6; ++c)
    for (int m = 0; m < 5; ++m) out[c * 5 + m] = C[c][m];
}

int orc_basis_set_omega(void* h, double omega) {
  if (!(omega >= 0.0) || !std::isfinite(omega)) return -1;
  static_cast<Basis*>(h)->omega = omega;
  return 0;
}

int orc_shell_quartet(void* h, int A, int B, int C, int D, double* out) {
  const Basis& bs = *static_cast<Basis*>(h);
  PrimQuartet pq;
  std::vector<double> cart(6 * 6 * 6 * 6);
  shell_quartet(bs, A, B, C, D, cart.data(), pq, bs.omega);
  const int sh[4] = {A, B, C, D};
  to_functions(bs, sh, cart.data(), out);   // over the shells' functions
  return 0;
}

int orc_schwarz(void* h, double* Q) {
  const Basis& bs = *static_cast<Basis*>(h);
  std::vector<double> q = schwarz(bs);
  std::copy(q.begin(), q.end(), Q);
  return 0;
}

// J, K over symmetry-unique shell quartets (AB|CD), A>=B, C>=D, pair AB >= pair CD,
// each quartet weighted by 1/(number of times it stands for itself) and digested
// into half-matrices that are symmetrised at the end.  D, J, K: [n_dm][n][n].
// Returns the number of quartets that passed the screening.
long long orc_jk(void* h, int n_dm, const double* D, double tol, double* J, double* K,
                 int nthreads) {
  const Basis& bs = *static_cast<Basis*>(h);
  const int n = bs.n_bf, ns = bs.n_shells;
  const std::vector<double> Q = schwarz(bs);
  const std::vector<PairIdx> pairs = unique_pairs(ns);
  const long long npair = (long long)pairs.size();
  const size_t nn = (size_t)n * n;
  std::vector<double> AJ((size_t)n_dm * nn, 0.0), AK((size_t)n_dm * nn, 0.0);
  long long kept = 0;
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel reduction(+ : kept)
  {
    std::vector<double> aj((size_t)n_dm * nn, 0.0), ak((size_t)n_dm * nn, 0.0);
    std::vector<double> cart(6 * 6 * 6 * 6), blk(6 * 6 * 6 * 6);
    PrimQuartet pq;
#pragma omp for schedule(dynamic, 1)
    for (long long pi = 0; pi < npair; ++pi) {
      const int A = pairs[pi].A, B = pairs[pi].B;
      for (long long qi = 0; qi <= pi; ++qi) {
        const int C = pairs[qi].A, Dd = pairs[qi].B;
        if (Q[(size_t)A * ns + B] * Q[(size_t)C * ns + Dd] < tol) continue;
        ++kept;
        shell_quartet(bs, A, B, C, Dd, cart.data(), pq, bs.omega);
        const int sh[4] = {A, B, C, Dd};
        to_functions(bs, sh, cart.data(), blk.data());
        double f = 1.0;
        if (A == B) f *= 0.5;
        if (C == Dd) f *= 0.5;
        if (pi == qi) f *= 0.5;
        const int na = nfun(bs, A), nb = nfun(bs, B), nc = nfun(bs, C), nd = nfun(bs, Dd);
        const int a0 = bs.bf0[A], b0 = bs.bf0[B], c0 = bs.bf0[C], d0 = bs.bf0[Dd];
        for (int m = 0; m < n_dm; ++m) {
          const double* Dm = D + (size_t)m * nn;
          double* jm = &aj[(size_t)m * nn];
          double* km = &ak[(size_t)m * nn];
          int idx = 0;
          for (int a = a0; a < a0 + na; ++a)
            for (int b = b0; b < b0 + nb; ++b)
              for (int c = c0; c < c0 + nc; ++c)
                for (int d = d0; d < d0 + nd; ++d) {
                  const double v = f * blk[idx++];
                  jm[(size_t)a * n + b] += 2.0 * Dm[(size_t)c * n + d] * v;
                  jm[(size_t)c * n + d] += 2.0 * Dm[(size_t)a * n + b] * v;
                  km[(size_t)a * n + c] += Dm[(size_t)b * n + d] * v;
                  km[(size_t)a * n + d] += Dm[(size_t)b * n + c] * v;
                  km[(size_t)b * n + c] += Dm[(size_t)a * n + d] * v;
                  km[(size_t)b * n + d] += Dm[(size_t)a * n + c] * v;
                }
        }
      }
    }
#pragma omp critical
    {
      for (size_t i = 0; i < aj.size(); ++i) { AJ[i] += aj[i]; AK[i] += ak[i]; }
    }
  }
  for (int m = 0; m < n_dm; ++m)
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        const size_t o = (size_t)m * nn;
        J[o + (size_t)i * n + j] = AJ[o + (size_t)i * n + j] + AJ[o + (size_t)j * n + i];
        K[o + (size_t)i * n + j] = AK[o + (size_t)i * n + j] + AK[o + (size_t)j * n + i];
      }
  return kept;
}

// J and K blocks of shell pairs (M_i, N_i) straight from the definitions,
// summing over every ordered pair of shells (no permutational symmetry):
//   J[mu][nu] = sum_{L,S} [Q_MN Q_LS >= tol] sum D[lam][sig] (mu nu|lam sig)
//   K[mu][nu] = sum_{L,S} [Q_ML Q_NS >= tol] sum D[lam][sig] (mu lam|nu sig)
// Blocks are packed one after another, each [n_dm][nM][nN].
int orc_jk_blocks(void* h, int n_dm, const double* D, double tol, int nblk, const int* sM,
                  const int* sN, double* Jout, double* Kout, int nthreads) {
  const Basis& bs = *static_cast<Basis*>(h);
  const int n = bs.n_bf, ns = bs.n_shells;
  const size_t nn = (size_t)n * n;
  const std::vector<double> Q = schwarz(bs);
  std::vector<size_t> off(nblk + 1, 0);
  for (int i = 0; i < nblk; ++i)
    off[i + 1] = off[i] + (size_t)n_dm * nfun(bs, sM[i]) * nfun(bs, sN[i]);
  if (nthreads > 0) omp_set_num_threads(nthreads);
  for (int ib = 0; ib < nblk; ++ib) {
    const int M = sM[ib], N = sN[ib];
    const int nm = nfun(bs, M), nnb = nfun(bs, N);
    std::vector<double> jb((size_t)n_dm * nm * nnb, 0.0), kb((size_t)n_dm * nm * nnb, 0.0);
#pragma omp parallel
    {
      std::vector<double> jl(jb.size(), 0.0), kl(kb.size(), 0.0);
      std::vector<double> cart(6 * 6 * 6 * 6), blk(6 * 6 * 6 * 6);
      PrimQuartet pq;
#pragma omp for schedule(dynamic, 1)
      for (int L = 0; L < ns; ++L)
        for (int S = 0; S < ns; ++S) {
          const int nl = nfun(bs, L), nsg = nfun(bs, S);
          const int l0 = bs.bf0[L], s0 = bs.bf0[S];
          if (Q[(size_t)M * ns + N] * Q[(size_t)L * ns + S] >= tol) {
            shell_quartet(bs, M, N, L, S, cart.data(), pq, bs.omega);
            const int sh[4] = {M, N, L, S};
            to_functions(bs, sh, cart.data(), blk.data());
            for (int m = 0; m < n_dm; ++m)
              for (int a = 0; a < nm; ++a)
                for (int b = 0; b < nnb; ++b) {
                  double s = 0.0;
                  for (int c = 0; c < nl; ++c)
                    for (int d = 0; d < nsg; ++d)
                      s += D[m * nn + (size_t)(l0 + c) * n + s0 + d] *
                           blk[((a * nnb + b) * nl + c) * nsg + d];
                  jl[((size_t)m * nm + a) * nnb + b] += s;
                }
          }
          if (Q[(size_t)M * ns + L] * Q[(size_t)N * ns + S] >= tol) {
            shell_quartet(bs, M, L, N, S, cart.data(), pq, bs.omega);
            const int sh[4] = {M, L, N, S};
            to_functions(bs, sh, cart.data(), blk.data());
            for (int m = 0; m < n_dm; ++m)
              for (int a = 0; a < nm; ++a)
                for (int b = 0; b < nnb; ++b) {
                  double s = 0.0;
                  for (int c = 0; c < nl; ++c)
                    for (int d = 0; d < nsg; ++d)
                      s += D[m * nn + (size_t)(l0 + c) * n + s0 + d] *
                           blk[((a * nl + c) * nnb + b) * nsg + d];
                  kl[((size_t)m * nm + a) * nnb + b] += s;
                }
          }
        }
#pragma omp critical
      for (size_t i = 0; i < jb.size(); ++i) { jb[i] += jl[i]; kb[i] += kl[i]; }
    }
    std::copy(jb.begin(), jb.end(), Jout + off[ib]);
    std::copy(kb.begin(), kb.end(), Kout + off[ib]);
  }
  return 0;
}

// dE/dR_atom of E = 1/2 tr(DJ) - 1/4 tr(DK) at fixed D, for each density.
// E = sum_{abcd} Gamma_abcd (ab|cd) with
//   Gamma_abcd = 1/2 D_ab D_cd - 1/8 (D_ac D_bd + D_ad D_bc),
// and a primitive derivative d/dA_x [x_A^i e^{-a x_A^2}] = 2a x_A^{i+1} e - i x_A^{i-1} e.
// All four centres are differentiated explicitly.  dEdR: [n_dm][n_atoms][3].
// If bra_pairs >= 0, only the first bra_pairs unique bra pairs are visited
// (a bounded sample used for timing).  If atom_sel is not NULL ([n_atoms]
// flags), only the derivatives with respect to the selected atoms are formed:
// a quartet enters only if one of its shells sits on a selected atom, and only
// the centres on selected atoms are differentiated (the other entries of dEdR
// stay zero).  dE/dR_X only depends on the quartets with a shell on X, so the
// selected entries equal those of the full gradient.
int orc_grad(void* h, int n_dm, const double* D, double tol, double* dEdR, int nthreads,
             long long bra_pairs, const int* atom_sel) {
  const Basis& bs = *static_cast<Basis*>(h);
  if (n_dm < 1 || n_dm > 16 || bs.omega != 0.0 || bs.pure) return -1;
  const int n = bs.n_bf, ns = bs.n_shells, na_ = bs.n_atoms;
  const size_t nn = (size_t)n * n;
  const std::vector<double> Q = schwarz(bs);
  const std::vector<PairIdx> pairs = unique_pairs(ns);
  long long npair = (long long)pairs.size();
  if (bra_pairs >= 0 && bra_pairs < npair) npair = bra_pairs;
  std::vector<double> G((size_t)n_dm * na_ * 3, 0.0);
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
  {
    std::vector<double> g((size_t)n_dm * na_ * 3, 0.0);
    PrimQuartet pq;
    std::vector<int> pw(4 * 6 * 3);
#pragma omp for schedule(dynamic, 1)
    for (long long pi = 0; pi < npair; ++pi) {
      const int A = pairs[pi].A, B = pairs[pi].B;
      for (long long qi = 0; qi <= pi; ++qi) {
        const int C = pairs[qi].A, Dd = pairs[qi].B;
        if (Q[(size_t)A * ns + B] * Q[(size_t)C * ns + Dd] < tol) continue;
        if (atom_sel && !atom_sel[bs.atom[A]] && !atom_sel[bs.atom[B]] && !atom_sel[bs.atom[C]] &&
            !atom_sel[bs.atom[Dd]])
          continue;
        double f = 8.0;
        if (A == B) f *= 0.5;
        if (C == Dd) f *= 0.5;
        if (pi == qi) f *= 0.5;
        const int sh[4] = {A, B, C, Dd};
        int lmax[4], nc[4], bf[4];
        for (int k = 0; k < 4; ++k) {
          lmax[k] = bs.l[sh[k]] + 1;
          nc[k] = ncart(bs.l[sh[k]]);
          bf[k] = bs.bf0[sh[k]];
          for (int i = 0; i < nc[k]; ++i) cart_powers(bs.l[sh[k]], i, &pw[(k * 6 + i) * 3]);
        }
        for (int i = 0; i < bs.nprim[A]; ++i)
          for (int j = 0; j < bs.nprim[B]; ++j)
            for (int k = 0; k < bs.nprim[C]; ++k)
              for (int m = 0; m < bs.nprim[Dd]; ++m) {
                const int ip[4] = {bs.prim0[A] + i, bs.prim0[B] + j, bs.prim0[C] + k,
                                   bs.prim0[Dd] + m};
                pq.build(lmax, bs.exps[ip[0]], bs.center(A), bs.exps[ip[1]], bs.center(B),
                         bs.exps[ip[2]], bs.center(C), bs.exps[ip[3]], bs.center(Dd));
                const double cc =
                    bs.coefs[ip[0]] * bs.coefs[ip[1]] * bs.coefs[ip[2]] * bs.coefs[ip[3]];
                for (int a = 0; a < nc[0]; ++a)
                  for (int b = 0; b < nc[1]; ++b)
                    for (int c = 0; c < nc[2]; ++c)
                      for (int d = 0; d < nc[3]; ++d) {
                        const int* p0[4] = {&pw[(0 + a) * 3], &pw[(6 + b) * 3],
                                            &pw[(12 + c) * 3], &pw[(18 + d) * 3]};
                        const int ia = bf[0] + a, ib = bf[1] + b, ic = bf[2] + c,
                                  id = bf[3] + d;
                        double gam[16];
                        for (int mm = 0; mm < n_dm; ++mm) {
                          const double* Dm = D + (size_t)mm * nn;
                          gam[mm] = 0.5 * Dm[(size_t)ia * n + ib] * Dm[(size_t)ic * n + id] -
                                    0.125 * (Dm[(size_t)ia * n + ic] * Dm[(size_t)ib * n + id] +
                                             Dm[(size_t)ia * n + id] * Dm[(size_t)ib * n + ic]);
                        }
                        for (int cen = 0; cen < 4; ++cen) {
                          const double ex = bs.exps[ip[cen]];
                          const int atom = bs.atom[sh[cen]];
                          if (atom_sel && !atom_sel[atom]) continue;
                          for (int x = 0; x < 3; ++x) {
                            int sp[4][3];
                            for (int k = 0; k < 4; ++k)
                              for (int y = 0; y < 3; ++y) sp[k][y] = p0[k][y];
                            sp[cen][x] += 1;
                            double dv = 2.0 * ex * pq.eri(sp[0], sp[1], sp[2], sp[3]);
                            if (p0[cen][x] > 0) {
                              sp[cen][x] -= 2;
                              dv -= p0[cen][x] * pq.eri(sp[0], sp[1], sp[2], sp[3]);
                            }
                            for (int mm = 0; mm < n_dm; ++mm)
                              g[((size_t)mm * na_ + atom) * 3 + x] += f * cc * gam[mm] * dv;
                          }
                        }
                      }
              }
      }
    }
#pragma omp critical
    for (size_t i = 0; i < G.size(); ++i) G[i] += g[i];
  }
  std::copy(G.begin(), G.end(), dEdR);
  return 0;
}

// Timing leg: J/K digestion restricted to the bra pairs listed (each with every
// ket pair that is unique with respect to it).  Returns the quartets computed.
long long orc_jk_bra_sample(void* h, int n_dm, const double* D, double tol, int nbra,
                            const int* bra_idx, double* J, double* K, int nthreads) {
  const Basis& bs = *static_cast<Basis*>(h);
  if (bs.pure) return -1;
  const int n = bs.n_bf, ns = bs.n_shells;
  const std::vector<double> Q = schwarz(bs);
  const std::vector<PairIdx> pairs = unique_pairs(ns);
  const size_t nn = (size_t)n * n;
  std::fill(J, J + n_dm * nn, 0.0);
  std::fill(K, K + n_dm * nn, 0.0);
  long long kept = 0;
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel reduction(+ : kept)
  {
    std::vector<double> blk(6 * 6 * 6 * 6);
    PrimQuartet pq;
    std::vector<double> aj((size_t)n_dm * nn, 0.0), ak((size_t)n_dm * nn, 0.0);
#pragma omp for schedule(dynamic, 1)
    for (int ii = 0; ii < nbra; ++ii) {
      const long long pi = bra_idx[ii];
      const int A = pairs[pi].A, B = pairs[pi].B;
      for (long long qi = 0; qi <= pi; ++qi) {
        const int C = pairs[qi].A, Dd = pairs[qi].B;
        if (Q[(size_t)A * ns + B] * Q[(size_t)C * ns + Dd] < tol) continue;
        ++kept;
        shell_quartet(bs, A, B, C, Dd, blk.data(), pq, bs.omega);
        double f = 1.0;
        if (A == B) f *= 0.5;
        if (C == Dd) f *= 0.5;
        if (pi == qi) f *= 0.5;
        const int na = ncart(bs.l[A]), nb = ncart(bs.l[B]), nc = ncart(bs.l[C]),
                  nd = ncart(bs.l[Dd]);
        const int a0 = bs.bf0[A], b0 = bs.bf0[B], c0 = bs.bf0[C], d0 = bs.bf0[Dd];
        for (int m = 0; m < n_dm; ++m) {
          const double* Dm = D + (size_t)m * nn;
          double* jm = &aj[(size_t)m * nn];
          double* km = &ak[(size_t)m * nn];
          int idx = 0;
          for (int a = a0; a < a0 + na; ++a)
            for (int b = b0; b < b0 + nb; ++b)
              for (int c = c0; c < c0 + nc; ++c)
                for (int d = d0; d < d0 + nd; ++d) {
                  const double v = f * blk[idx++];
                  jm[(size_t)a * n + b] += 2.0 * Dm[(size_t)c * n + d] * v;
                  jm[(size_t)c * n + d] += 2.0 * Dm[(size_t)a * n + b] * v;
                  km[(size_t)a * n + c] += Dm[(size_t)b * n + d] * v;
                  km[(size_t)a * n + d] += Dm[(size_t)b * n + c] * v;
                  km[(size_t)b * n + c] += Dm[(size_t)a * n + d] * v;
                  km[(size_t)b * n + d] += Dm[(size_t)a * n + c] * v;
                }
        }
      }
    }
#pragma omp critical
    for (size_t i = 0; i < aj.size(); ++i) { J[i] += aj[i]; K[i] += ak[i]; }
  }
  return kept;
}

// Screening and precision decisions of every symmetry-unique shell quartet
// (pair AB >= pair CD, the pairs numbered as in orc_jk), from S = Q_AB Q_CD:
// skipped if S < tol, single precision if tol <= S < thr, double precision if
// S >= thr (paper, "Electron Repulsion Integrals" paragraph, third item).  The
// counts are kept per quartet class: each pair has a class by its two angular
// momenta (l1 >= l2 ordered as ss, ps, pp, ds, dp, dd = 0..5); a quartet's class
// index is X (X+1)/2 + Y for its larger pair class X and smaller Y.
// counts[21][3] = {double, single, skipped}; near[21] counts the quartets
// whose S lies within a relative 1e-12 of tol or thr (where a different
// rounding of Q could flip the decision).
int orc_screen_counts(void* h, double tol, double thr, long long* counts, long long* near) {
  const Basis& bs = *static_cast<Basis*>(h);
  const int ns = bs.n_shells;
  const std::vector<double> Q = schwarz(bs);
  const std::vector<PairIdx> pairs = unique_pairs(ns);
  const long long npair = (long long)pairs.size();
  std::vector<int> pcls(npair);
  std::vector<double> pq(npair);
  for (long long i = 0; i < npair; ++i) {
    const int l1 = std::max(bs.l[pairs[i].A], bs.l[pairs[i].B]);
    const int l2 = std::min(bs.l[pairs[i].A], bs.l[pairs[i].B]);
    pcls[i] = l1 * (l1 + 1) / 2 + l2;
    pq[i] = Q[(size_t)pairs[i].A * ns + pairs[i].B];
  }
  std::fill(counts, counts + 21 * 3, 0LL);
  std::fill(near, near + 21, 0LL);
#pragma omp parallel
  {
    std::vector<long long> c(21 * 3, 0), nr(21, 0);
#pragma omp for schedule(dynamic, 64)
    for (long long i = 0; i < npair; ++i)
      for (long long j = 0; j <= i; ++j) {
        const int X = std::max(pcls[i], pcls[j]), Y = std::min(pcls[i], pcls[j]);
        const int q = X * (X + 1) / 2 + Y;
        const double S = pq[i] * pq[j];
        const int k = S < tol ? 2 : (S < thr ? 1 : 0);
        ++c[3 * q + k];
        if (std::fabs(S - tol) <= 1e-12 * tol || std::fabs(S - thr) <= 1e-12 * thr) ++nr[q];
      }
#pragma omp critical
    {
      for (int t = 0; t < 63; ++t) counts[t] += c[t];
      for (int t = 0; t < 21; ++t) near[t] += nr[t];
    }
  }
  return 0;
}

const char* orc_last_error(void) { return g_err; }

}  // extern "C"
