// Drives every entry point of the CPU oracle once on a three-atom s/p/d basis,
// for a build with AddressSanitizer and UndefinedBehaviorSanitizer
// (tests/test_sanitizers.py).  Exit status 0 when every call succeeds and the
// results pass the cheap consistency checks below; the sanitizers abort on the
// first memory or undefined-behaviour error.
#include <cmath>
#include <cstdio>
#include <vector>

extern "C" {
void* orc_basis_new(int, const double*, int, const int*, const int*, const int*, const int*,
                    const double*, const double*);
void orc_basis_free(void*);
int orc_boys(int, double, double*);
double orc_prim_eri(const int*, double, const double*, const int*, double, const double*,
                    const int*, double, const double*, const int*, double, const double*);
int orc_shell_quartet(void*, int, int, int, int, double*);
int orc_schwarz(void*, double*);
long long orc_jk(void*, int, const double*, double, double*, double*, int);
int orc_jk_blocks(void*, int, const double*, double, int, const int*, const int*, double*, double*,
                  int);
int orc_grad(void*, int, const double*, double, double*, int, long long, const int*);
long long orc_jk_bra_sample(void*, int, const double*, double, int, const int*, double*, double*,
                            int);
int orc_screen_counts(void*, double, double, long long*, long long*);
double orc_prim_eri_omega(const int*, double, const double*, const int*, double, const double*,
                          const int*, double, const double*, const int*, double, const double*,
                          double);
int orc_basis_set_omega(void*, double);
int orc_basis_set_pure(void*, int);
int orc_n_bf(void*);
void orc_pure_d(double*);
}

static int fail(const char* what) {
  std::fprintf(stderr, "oracle driver: %s\n", what);
  return 1;
}

int main() {
  // atoms 0, 1: s, p, d shells; atom 2: s, p (ragged contraction lengths)
  const double xyz[9] = {0.0, 0.0, 0.0, 1.4, 0.3, -0.2, -0.5, 1.7, 0.6};
  const int atom[8] = {0, 0, 0, 1, 1, 1, 2, 2};
  const int l[8] = {0, 1, 2, 0, 1, 2, 0, 1};
  const int nprim[8] = {3, 2, 1, 3, 2, 1, 2, 1};
  std::vector<int> prim0(8);
  int np = 0;
  for (int s = 0; s < 8; ++s) { prim0[s] = np; np += nprim[s]; }
  std::vector<double> ex(np), co(np);
  for (int p = 0; p < np; ++p) {
    ex[p] = 0.2 * std::pow(3.0, p % 3) + 0.05 * p;
    co[p] = 0.3 + 0.1 * (p % 4);
  }
  void* b = orc_basis_new(3, xyz, 8, atom, l, nprim, prim0.data(), ex.data(), co.data());
  int n = 0;
  for (int s = 0; s < 8; ++s) n += (l[s] + 1) * (l[s] + 2) / 2;
  const int n_dm = 2;
  std::vector<double> D(static_cast<size_t>(n_dm) * n * n);
  for (int m = 0; m < n_dm; ++m)
    for (int i = 0; i < n; ++i)
      for (int j = 0; j <= i; ++j) {
        const double v = std::sin(0.37 * (i + 1) * (j + 2) + m) / (1.0 + std::abs(i - j));
        D[(static_cast<size_t>(m) * n + i) * n + j] = D[(static_cast<size_t>(m) * n + j) * n + i] = v;
      }

  double F[31];
  for (double T : {0.0, 1e-9, 0.7, 12.0, 31.0, 80.0})
    if (orc_boys(30, T, F) != 0 || !std::isfinite(F[30])) return fail("boys");
  const int pa[3] = {2, 0, 0}, pb[3] = {0, 1, 0}, pc[3] = {0, 0, 1}, pd[3] = {1, 1, 0};
  if (!std::isfinite(orc_prim_eri(pa, 0.5, xyz, pb, 0.9, xyz + 3, pc, 1.3, xyz + 6, pd, 0.4, xyz)))
    return fail("prim_eri");
  std::vector<double> blk(6 * 6 * 6 * 6);
  if (orc_shell_quartet(b, 2, 5, 4, 7, blk.data()) != 0) return fail("shell_quartet");
  std::vector<double> Q(8 * 8);
  if (orc_schwarz(b, Q.data()) != 0) return fail("schwarz");

  std::vector<double> J(D.size()), K(D.size());
  const long long kept = orc_jk(b, n_dm, D.data(), 1e-10, J.data(), K.data(), 2);
  if (kept <= 0) return fail("jk");
  for (int m = 0; m < n_dm; ++m)
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        const size_t ij = (static_cast<size_t>(m) * n + i) * n + j, ji = (static_cast<size_t>(m) * n + j) * n + i;
        if (std::abs(J[ij] - J[ji]) > 1e-12 || std::abs(K[ij] - K[ji]) > 1e-12) return fail("J or K not symmetric");
      }
  // blocks of shell pairs (M, N) must reproduce the full build
  const int sM[3] = {5, 2, 7}, sN[3] = {1, 2, 3};
  std::vector<double> Jb(static_cast<size_t>(n_dm) * 3 * 36), Kb(Jb.size());
  if (orc_jk_blocks(b, n_dm, D.data(), 1e-10, 3, sM, sN, Jb.data(), Kb.data(), 2) != 0)
    return fail("jk_blocks");
  std::vector<int> bf0(8, 0);
  for (int s = 1; s < 8; ++s) bf0[s] = bf0[s - 1] + (l[s - 1] + 1) * (l[s - 1] + 2) / 2;
  size_t at = 0;
  for (int ib = 0; ib < 3; ++ib) {
    const int nm = (l[sM[ib]] + 1) * (l[sM[ib]] + 2) / 2, nn = (l[sN[ib]] + 1) * (l[sN[ib]] + 2) / 2;
    for (int m = 0; m < n_dm; ++m)
      for (int x = 0; x < nm; ++x)
        for (int y = 0; y < nn; ++y, ++at) {
          const size_t e = (static_cast<size_t>(m) * n + bf0[sM[ib]] + x) * n + bf0[sN[ib]] + y;
          if (std::abs(Jb[at] - J[e]) > 1e-12 || std::abs(Kb[at] - K[e]) > 1e-12)
            return fail("jk_blocks differs from jk");
        }
  }
  const int bra[2] = {0, 11};
  std::vector<double> Js(D.size()), Ks(D.size());
  if (orc_jk_bra_sample(b, n_dm, D.data(), 1e-10, 2, bra, Js.data(), Ks.data(), 2) <= 0)
    return fail("jk_bra_sample");
  std::vector<double> g(static_cast<size_t>(n_dm) * 3 * 3);
  if (orc_grad(b, n_dm, D.data(), 1e-10, g.data(), 2, -1, nullptr) != 0) return fail("grad");
  // translation invariance: the forces on the three atoms sum to zero
  for (int m = 0; m < n_dm; ++m)
    for (int x = 0; x < 3; ++x) {
      double s = 0.0;
      for (int a = 0; a < 3; ++a) s += g[(m * 3 + a) * 3 + x];
      if (std::abs(s) > 1e-9) return fail("gradient not translation invariant");
    }
  const int sel[3] = {0, 1, 0};   // atom 1 only
  if (orc_grad(b, 1, D.data(), 1e-10, g.data(), 1, -1, sel) != 0) return fail("grad (one atom)");
  // erf(omega r12)/r12: a build at omega and the gradient's refusal of it
  if (!std::isfinite(orc_prim_eri_omega(pa, 0.5, xyz, pb, 0.9, xyz + 3, pc, 1.3, xyz + 6, pd, 0.4,
                                        xyz, 0.3)))
    return fail("prim_eri_omega");
  if (orc_basis_set_omega(b, -1.0) == 0 || orc_basis_set_omega(b, 0.3) != 0)
    return fail("basis_set_omega");
  if (orc_jk(b, n_dm, D.data(), 1e-10, J.data(), K.data(), 2) <= 0) return fail("jk at omega");
  if (orc_grad(b, n_dm, D.data(), 1e-10, g.data(), 2, -1, nullptr) == 0)
    return fail("grad must refuse omega > 0");
  if (orc_basis_set_omega(b, 0.0) != 0) return fail("basis_set_omega");
  // pure d functions: renumbered basis, J/K over it, a quartet block, the table
  if (orc_basis_set_pure(b, 2) == 0 || orc_basis_set_pure(b, 1) != 0) return fail("basis_set_pure");
  const int np_ = orc_n_bf(b);
  if (np_ != n - 2) return fail("pure basis size");
  std::vector<double> Dp(static_cast<size_t>(np_) * np_, 0.1), Jp(Dp.size()), Kp(Dp.size());
  if (orc_jk(b, 1, Dp.data(), 1e-10, Jp.data(), Kp.data(), 2) <= 0) return fail("pure jk");
  std::vector<double> pblk(5 * 5 * 5 * 5), tab(30);
  if (orc_shell_quartet(b, 2, 5, 2, 5, pblk.data()) != 0) return fail("pure shell_quartet");
  orc_pure_d(tab.data());
  if (orc_grad(b, 1, Dp.data(), 1e-10, g.data(), 1, -1, nullptr) == 0)
    return fail("grad must refuse a pure basis");
  if (orc_basis_set_pure(b, 0) != 0 || orc_n_bf(b) != n) return fail("back to Cartesian");
  long long counts[63], near[21];
  if (orc_screen_counts(b, 1e-10, 1e-4, counts, near) != 0) return fail("screen_counts");
  long long tot = 0;
  for (long long c : counts) tot += c;
  if (tot != 36LL * 37 / 2) return fail("screen_counts total");
  orc_basis_free(b);
  std::printf("oracle driver ok: %lld quartets kept\n", kept);
  return 0;
}
