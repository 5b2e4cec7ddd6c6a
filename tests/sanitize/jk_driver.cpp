// Runs libjk's C entry points on a real device from a host program whose
// library host code is built with AddressSanitizer and UndefinedBehaviorSanitizer
// (tests/sanitize/build_jk_asan.py; the device code is built as usual).
//
//   jk_asan_driver INPUT OUTPUT
//
// INPUT (little-endian): int32 n_atoms, n_shells, n_prim, n_dm, n_bf; double
// xyz[3 n_atoms]; int32 shell_atom, shell_l, shell_nprim, shell_prim0 [n_shells];
// double exps[n_prim], coefs[n_prim]; double D[n_dm n_bf n_bf]; double tol.
// OUTPUT: for each of the cases below in order, J then K ([n_dm][n][n] doubles).
// Cases: FP64; mixed; deterministic with reuse_setup (second call, which must
// reuse the setup); jk_build_noalloc; one accumulator copy with energies and
// dE/dD (checked against J and K here); FP64 at omega = 0.3 (erf(omega r12)/r12);
// FP64 again; timing and jk_get_stats.  Between the last two, the pure-function
// transforms are checked in the driver by a trace identity.  Exit status 0
// when every call succeeds and every in-driver check holds.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "jk.h"

namespace {

int fail(const char* what, const jk_ctx* c = nullptr) {
  std::fprintf(stderr, "jk driver: %s (%s)\n", what, jk_last_error(c));
  return 1;
}

template <typename T>
bool get(FILE* f, std::vector<T>& v, size_t n) {
  v.resize(n);
  return n == 0 || std::fread(v.data(), sizeof(T), n, f) == n;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc != 3) return fail("usage: jk_asan_driver INPUT OUTPUT");
  FILE* in = std::fopen(argv[1], "rb");
  if (!in) return fail("cannot open input");
  std::vector<int32_t> head, atom, l, nprim, prim0;
  std::vector<double> xyz, exps, coefs, Dh, tolv;
  if (!get(in, head, 5)) return fail("short input");
  const int na = head[0], ns = head[1], np = head[2], n_dm = head[3], n = head[4];
  if (!get(in, xyz, 3 * static_cast<size_t>(na)) || !get(in, atom, ns) || !get(in, l, ns) ||
      !get(in, nprim, ns) || !get(in, prim0, ns) || !get(in, exps, np) || !get(in, coefs, np) ||
      !get(in, Dh, static_cast<size_t>(n_dm) * n * n) || !get(in, tolv, 1))
    return fail("short input");
  std::fclose(in);
  const double tol = tolv[0];
  jk_basis b{};
  b.n_atoms = na;
  b.xyz = xyz.data();
  b.n_shells = ns;
  b.shell_atom = atom.data();
  b.shell_l = l.data();
  b.shell_nprim = nprim.data();
  b.shell_prim0 = prim0.data();
  b.exps = exps.data();
  b.coefs = coefs.data();
  int32_t nbf = 0;
  if (jk_validate_basis(&b, &nbf) != JK_OK || nbf != n) return fail("basis");

  const size_t mat = static_cast<size_t>(n_dm) * n * n;
  double *D = nullptr, *J = nullptr, *K = nullptr, *E = nullptr, *G = nullptr;
  if (hipMalloc(&D, mat * 8) != hipSuccess || hipMalloc(&J, mat * 8) != hipSuccess ||
      hipMalloc(&K, mat * 8) != hipSuccess || hipMalloc(&E, 3 * n_dm * 8) != hipSuccess ||
      hipMalloc(&G, mat * 8) != hipSuccess)
    return fail("hipMalloc");
  if (hipMemcpy(D, Dh.data(), mat * 8, hipMemcpyHostToDevice) != hipSuccess) return fail("copy D");
  jk_ctx* c = nullptr;
  if (jk_ctx_create(&c, 0) != JK_OK) return fail("jk_ctx_create");
  FILE* out = std::fopen(argv[2], "wb");
  if (!out) return fail("cannot open output");
  std::vector<double> hj(mat), hk(mat);
  auto emit = [&]() -> bool {
    if (hipDeviceSynchronize() != hipSuccess) return false;
    if (hipMemcpy(hj.data(), J, mat * 8, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(hk.data(), K, mat * 8, hipMemcpyDeviceToHost) != hipSuccess)
      return false;
    return std::fwrite(hj.data(), 8, mat, out) == mat && std::fwrite(hk.data(), 8, mat, out) == mat;
  };
  jk_opts o;
  jk_opts_default(&o);
  o.n_dm = n_dm;

  // FP64
  if (jk_build(c, &b, D, J, K, tol, &o, nullptr) != JK_OK || !emit()) return fail("fp64", c);
  // mixed
  jk_opts om = o;
  om.precision = JK_MIXED;
  if (jk_build(c, &b, D, J, K, tol, &om, nullptr) != JK_OK || !emit()) return fail("mixed", c);
  // deterministic, setup kept and reused
  jk_opts od = o;
  od.deterministic = 1;
  od.reuse_setup = 1;
  jk_stats st;
  if (jk_build(c, &b, D, J, K, tol, &od, nullptr) != JK_OK) return fail("deterministic", c);
  if (jk_build(c, &b, D, J, K, tol, &od, nullptr) != JK_OK || jk_get_stats(c, &st) != JK_OK ||
      st.setup_reused != 1 || !emit())
    return fail("deterministic, reused setup", c);
  // allocation-free entry
  if (jk_build_noalloc(c, &b, D, J, K, tol, &o, nullptr) != JK_OK || !emit())
    return fail("jk_build_noalloc", c);
  // one accumulator copy, energies and dE/dD
  jk_opts oe = o;
  oe.acc_copies = 1;
  oe.energy = E;
  oe.dEdD = G;
  if (jk_build(c, &b, D, J, K, tol, &oe, nullptr) != JK_OK || !emit())
    return fail("single copy with energies", c);
  std::vector<double> he(3 * n_dm), hg(mat);
  if (hipMemcpy(he.data(), E, 3 * n_dm * 8, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(hg.data(), G, mat * 8, hipMemcpyDeviceToHost) != hipSuccess)
    return fail("copy energies");
  for (int m = 0; m < n_dm; ++m) {
    double ej = 0.0, ek = 0.0, scale = 1.0;
    for (size_t t = 0; t < static_cast<size_t>(n) * n; ++t) {
      const size_t u = m * static_cast<size_t>(n) * n + t;
      ej += 0.5 * Dh[u] * hj[u];
      ek += 0.25 * Dh[u] * hk[u];
      scale = std::fmax(scale, std::fabs(hj[u]) + std::fabs(hk[u]));
      if (std::fabs(hg[u] - (hj[u] - 0.5 * hk[u])) > 1e-12 * scale) return fail("dE/dD");
    }
    if (std::fabs(he[3 * m] - ej) > 1e-9 * std::fmax(1.0, std::fabs(ej)) ||
        std::fabs(he[3 * m + 1] - ek) > 1e-9 * std::fmax(1.0, std::fabs(ek)) ||
        std::fabs(he[3 * m + 2] - (he[3 * m] - he[3 * m + 1])) > 1e-12 * std::fmax(1.0, std::fabs(ej)))
      return fail("energies");
  }
  // erf(omega r12)/r12 at omega = 0.3, and the gradient's refusal of omega > 0
  jk_opts ow = o;
  ow.omega = 0.3;
  if (jk_build(c, &b, D, J, K, tol, &ow, nullptr) != JK_OK || !emit()) return fail("omega", c);
  if (jk_grad(c, &b, D, G, tol, &ow, nullptr) != JK_EUNSUPPORTED) return fail("grad at omega", c);
  // pure d functions: with P the leading pure-sized block of D (symmetric),
  // tr(P T^T J T) = tr(T P T^T J) for the FP64 J of the last build
  int32_t npu = 0;
  if (jk_pure_count(&b, &npu) != JK_OK || npu > n) return fail("jk_pure_count");
  if (jk_build(c, &b, D, J, K, tol, &o, nullptr) != JK_OK || !emit()) return fail("fp64 again", c);
  {
    const size_t pm = static_cast<size_t>(n_dm) * npu * npu;
    std::vector<double> Ph(pm), Jp(pm), Xc(mat);
    for (int m = 0; m < n_dm; ++m)
      for (int i = 0; i < npu; ++i)
        for (int j = 0; j < npu; ++j)
          Ph[(static_cast<size_t>(m) * npu + i) * npu + j] = Dh[(static_cast<size_t>(m) * n + i) * n + j];
    double *P = nullptr, *Pj = nullptr;
    if (hipMalloc(&P, pm * 8) != hipSuccess || hipMalloc(&Pj, pm * 8) != hipSuccess) return fail("hipMalloc");
    if (hipMemcpy(P, Ph.data(), pm * 8, hipMemcpyHostToDevice) != hipSuccess) return fail("copy P");
    if (jk_pure_to_cart(&b, n_dm, P, G, nullptr) != JK_OK ||
        jk_cart_to_pure(&b, n_dm, J, Pj, nullptr) != JK_OK || hipDeviceSynchronize() != hipSuccess)
      return fail("pure transforms");
    if (hipMemcpy(Xc.data(), G, mat * 8, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(Jp.data(), Pj, pm * 8, hipMemcpyDeviceToHost) != hipSuccess)
      return fail("copy pure results");
    for (int m = 0; m < n_dm; ++m) {
      double a = 0.0, bsum = 0.0, scale = 0.0;
      for (size_t t = 0; t < static_cast<size_t>(npu) * npu; ++t) {
        a += Ph[m * static_cast<size_t>(npu) * npu + t] * Jp[m * static_cast<size_t>(npu) * npu + t];
        scale += std::fabs(Ph[m * static_cast<size_t>(npu) * npu + t] * Jp[m * static_cast<size_t>(npu) * npu + t]);
      }
      for (size_t t = 0; t < static_cast<size_t>(n) * n; ++t)
        bsum += Xc[m * static_cast<size_t>(n) * n + t] * hj[m * static_cast<size_t>(n) * n + t];
      if (std::fabs(a - bsum) > 1e-12 * std::fmax(1.0, scale)) return fail("pure trace identity");
    }
    if (jk_pure_to_cart(&b, 0, P, G, nullptr) != JK_EINVAL) return fail("pure n_dm check");
    (void)hipFree(P);
    (void)hipFree(Pj);
  }
  // timing and statistics
  jk_opts ot = o;
  ot.timing = 1;
  if (jk_build(c, &b, D, J, K, tol, &ot, nullptr) != JK_OK || jk_get_stats(c, &st) != JK_OK)
    return fail("timing", c);
  if (!(st.ms_total > 0.0) || st.n_pairs != static_cast<int64_t>(ns) * (ns + 1) / 2)
    return fail("stats");
  // an invalid tol is rejected before any output is written
  if (jk_build(c, &b, D, J, K, -1.0, &o, nullptr) != JK_EINVAL) return fail("tol check");
  std::fclose(out);
  jk_ctx_destroy(c);
  for (double* p : {D, J, K, E, G}) (void)hipFree(p);
  std::printf("jk driver ok\n");
  return 0;
}
