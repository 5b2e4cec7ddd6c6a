// Host build of the generated energy-class code: contracted shell quartets with an
// exact Boys function, for comparison with the oracle (test harness, CPU only).
#include <type_traits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <algorithm>
#define __device__
#define __forceinline__ inline
namespace jk {
template <typename T> struct VrrCoef {
  T PAx, PAy, PAz, WPx, WPy, WPz, QCx, QCy, QCz, WQx, WQy, WQz;
  T oo2p, oo2p_rp, oo2q, oo2q_rq, oo2pq;
};
using std::fmax;
#include "cls_ssss.inc"
#include "cls_psss.inc"
#include "cls_psps.inc"
#include "cls_ppss.inc"
#include "cls_ppps.inc"
#include "cls_pppp.inc"
#include "cls_dsss.inc"
#include "cls_dsps.inc"
#include "cls_dspp.inc"
#include "cls_dsds.inc"
#include "cls_dpss.inc"
#include "cls_dpps.inc"
#include "cls_dppp.inc"
#include "cls_dpds.inc"
#include "cls_dpdp.inc"
#include "cls_ddss.inc"
#include "cls_ddps.inc"
#include "cls_ddpp.inc"
#include "cls_ddds.inc"
#include "cls_dddp.inc"
#include "cls_dddd.inc"
}
using namespace jk;

static double boys_exact(int m, double T) {
  long double term = 1.0L / (2 * m + 1), sum = term;
  for (int k = 1; k < 100000; ++k) { term *= 2.0L * T / (2 * m + 2 * k + 1); sum += term; if (term < sum * 1e-21L) break; }
  return (double)(std::exp(-(long double)T) * sum);
}

struct Sh { int l, np; double A[3]; double e[8], c[8]; };

template <class C, class V>
static void contract(const Sh& a, const Sh& b, const Sh& c, const Sh& d, V&& vrr) {
  const double PI = 3.14159265358979323846;
  for (int i = 0; i < a.np; ++i) for (int j = 0; j < b.np; ++j)
  for (int k = 0; k < c.np; ++k) for (int l = 0; l < d.np; ++l) {
    double p = a.e[i] + b.e[j], q = c.e[k] + d.e[l];
    double P[3], Q[3], AB2 = 0, CD2 = 0;
    for (int x = 0; x < 3; ++x) {
      P[x] = (a.e[i] * a.A[x] + b.e[j] * b.A[x]) / p;
      Q[x] = (c.e[k] * c.A[x] + d.e[l] * d.A[x]) / q;
      AB2 += (a.A[x] - b.A[x]) * (a.A[x] - b.A[x]);
      CD2 += (c.A[x] - d.A[x]) * (c.A[x] - d.A[x]);
    }
    double W[3], PQ2 = 0;
    for (int x = 0; x < 3; ++x) { W[x] = (p * P[x] + q * Q[x]) / (p + q); PQ2 += (P[x] - Q[x]) * (P[x] - Q[x]); }
    double rho = p * q / (p + q), T = rho * PQ2;
    double pref = 2 * std::pow(PI, 2.5) / (p * q * std::sqrt(p + q)) *
                  a.c[i] * b.c[j] * c.c[k] * d.c[l] * std::exp(-a.e[i] * b.e[j] / p * AB2) *
                  std::exp(-c.e[k] * d.e[l] / q * CD2);
    double F[16];
    for (int m = 0; m <= C::L; ++m) F[m] = pref * boys_exact(m, T);
    VrrCoef<double> cf;
    cf.PAx = P[0] - a.A[0]; cf.PAy = P[1] - a.A[1]; cf.PAz = P[2] - a.A[2];
    cf.WPx = W[0] - P[0]; cf.WPy = W[1] - P[1]; cf.WPz = W[2] - P[2];
    cf.QCx = Q[0] - c.A[0]; cf.QCy = Q[1] - c.A[1]; cf.QCz = Q[2] - c.A[2];
    cf.WQx = W[0] - Q[0]; cf.WQy = W[1] - Q[1]; cf.WQz = W[2] - Q[2];
    cf.oo2p = 0.5 / p; cf.oo2p_rp = 0.5 / p * rho / p; cf.oo2q = 0.5 / q; cf.oo2q_rq = 0.5 / q * rho / q;
    cf.oo2pq = 0.5 / (p + q);
    vrr(F, cf);
  }
}

// raw (ab|cd) via the digestion function with a one-hot D_cd
template <class C>
static void block_single(const Sh& a, const Sh& b, const Sh& c, const Sh& d, double* out) {
  double acc[C::NACC] = {0};
  contract<C>(a, b, c, d, [&](const double* F, const VrrCoef<double>& cf) { C::template vrr<double>(F, cf, acc); });
  double ABx = a.A[0] - b.A[0], ABy = a.A[1] - b.A[1], ABz = a.A[2] - b.A[2];
  double CDx = c.A[0] - d.A[0], CDy = c.A[1] - d.A[1], CDz = c.A[2] - d.A[2];
  for (int cd = 0; cd < C::NC * C::ND; ++cd) {
    double Dab[64] = {0}, Dcd[64] = {0}, Z[64] = {0};
    Dcd[cd] = 1.0;
    double jab[64] = {0}, jcd[64] = {0}, kac[64] = {0}, kad[64] = {0}, kbc[64] = {0}, kbd[64] = {0};
    C::template hrr_digest<double>(acc, ABx, ABy, ABz, CDx, CDy, CDz, 1.0, Dab, Dcd, Z, Z, Z, Z,
                                   jab, jcd, kac, kad, kbc, kbd);
    for (int ab = 0; ab < C::NA * C::NB; ++ab) out[ab * C::NC * C::ND + cd] = jab[ab];
  }
}

template <class C, int J>
static void passes(const Sh& a, const Sh& b, const Sh& c, const Sh& d, double* cacc) {
  constexpr int NEJ = C::template Pass<J>::NE, E0 = C::template Pass<J>::E0;
  double acc[NEJ * C::NF] = {0};
  contract<C>(a, b, c, d, [&](const double* F, const VrrCoef<double>& cf) { C::template vrr_pass<J, double>(F, cf, acc); });
  for (int t = 0; t < NEJ * C::NF; ++t) cacc[E0 * C::NF + t] = acc[t];
  if constexpr (J + 1 < C::NPASS) passes<C, J + 1>(a, b, c, d, cacc);
}

template <class C>
static void block_split(const Sh& a, const Sh& b, const Sh& c, const Sh& d, double* out) {
  static double cacc[C::NACC];
  passes<C, 0>(a, b, c, d, cacc);
  double ABx = a.A[0] - b.A[0], ABy = a.A[1] - b.A[1], ABz = a.A[2] - b.A[2];
  double CDx = c.A[0] - d.A[0], CDy = c.A[1] - d.A[1], CDz = c.A[2] - d.A[2];
  constexpr int NCD = C::NC * C::ND;
  static double X[C::NE * NCD];
  for (int e = 0; e < C::NE; ++e) C::template ket_hrr<double>(cacc + e * C::NF, CDx, CDy, CDz, X + e * NCD);
  for (int cd = 0; cd < NCD; ++cd) {
    double ev[C::NE], ab[C::NA * C::NB];
    for (int e = 0; e < C::NE; ++e) ev[e] = X[e * NCD + cd];
    C::template bra_hrr<double>(ev, ABx, ABy, ABz, ab);
    for (int t = 0; t < C::NA * C::NB; ++t) out[t * NCD + cd] = ab[t];
  }
}

// single-pass classes have no NPASS member; multi-pass classes do
template <class C, class = void>
struct is_split : std::false_type {};
template <class C>
struct is_split<C, std::void_t<decltype(C::NPASS)>> : std::true_type {};

template <class C>
static void block(const Sh& a, const Sh& b, const Sh& c, const Sh& d, double* out) {
  if constexpr (is_split<C>::value) block_split<C>(a, b, c, d, out);
  else block_single<C>(a, b, c, d, out);
}

extern "C" int emu_block(int cls, const int* l, const int* np, const double* A, const double* e,
                         const double* c, double* out) {
  Sh s[4];
  for (int k = 0; k < 4; ++k) {
    s[k].l = l[k]; s[k].np = np[k];
    for (int x = 0; x < 3; ++x) s[k].A[x] = A[3 * k + x];
    for (int i = 0; i < np[k]; ++i) { s[k].e[i] = e[8 * k + i]; s[k].c[i] = c[8 * k + i]; }
  }
  switch (cls) {
#define S1(i, N) case i: block<Cls_##N>(s[0], s[1], s[2], s[3], out); break;
    S1(0, ssss) S1(1, psss) S1(2, psps) S1(3, ppss) S1(4, ppps) S1(5, pppp) S1(6, dsss) S1(7, dsps)
    S1(8, dspp) S1(9, dsds) S1(10, dpss) S1(11, dpps) S1(12, dppp) S1(13, dpds) S1(14, dpdp)
    S1(15, ddss) S1(16, ddps) S1(17, ddpp) S1(18, ddds) S1(19, dddp) S1(20, dddd)
    default: return -1;
  }
  return 0;
}

// The FP32 layouts of the multi-pass classes (their own pass sizes, or one
// pass), evaluated here in double precision like the others.
extern "C" int emu_block32(int cls, const int* l, const int* np, const double* A, const double* e,
                           const double* c, double* out) {
  Sh s[4];
  for (int k = 0; k < 4; ++k) {
    s[k].l = l[k]; s[k].np = np[k];
    for (int x = 0; x < 3; ++x) s[k].A[x] = A[3 * k + x];
    for (int i = 0; i < np[k]; ++i) { s[k].e[i] = e[8 * k + i]; s[k].c[i] = c[8 * k + i]; }
  }
  switch (cls) {
#define S3(i, N) case i: block<Cls_##N##_f32>(s[0], s[1], s[2], s[3], out); break;
    S3(12, dppp) S3(14, dpdp) S3(17, ddpp) S3(18, ddds) S3(19, dddp) S3(20, dddd)
    default: return -1;
  }
  return 0;
}

// The five digestion sweeps of a single-pass class against its one-sweep
// digestion, on arbitrary contracted values and D blocks; returns the largest
// difference over all six blocks (multi-pass classes: 0, they have no sweeps).
template <class C>
static double sweeps_diff() {
  if constexpr (is_split<C>::value) {
    return 0.0;
  } else {
    double acc[C::NACC];
    unsigned s = 12345u;
    auto rnd = [&]() { s = s * 1103515245u + 12345u; return ((s >> 8) & 0xffff) / 65536.0 - 0.5; };
    for (int t = 0; t < C::NACC; ++t) acc[t] = rnd();
    double D6[6][64];
    for (auto& blk : D6) for (double& v : blk) v = rnd();
    const double AB[3] = {0.3, -0.7, 1.1}, CD[3] = {-0.4, 0.9, 0.2};
    double r1[6][64] = {{0}}, r2[6][64] = {{0}};
    C::template hrr_digest<double>(acc, AB[0], AB[1], AB[2], CD[0], CD[1], CD[2], 0.75, D6[0], D6[1],
                                   D6[2], D6[3], D6[4], D6[5], r1[0], r1[1], r1[2], r1[3], r1[4],
                                   r1[5]);
    C::template digest_j<double>(acc, AB[0], AB[1], AB[2], CD[0], CD[1], CD[2], 0.75, D6[0], D6[1],
                                 r2[0], r2[1]);
    C::template digest_kac<double>(acc, AB[0], AB[1], AB[2], CD[0], CD[1], CD[2], 0.75, D6[5], r2[2]);
    C::template digest_kad<double>(acc, AB[0], AB[1], AB[2], CD[0], CD[1], CD[2], 0.75, D6[4], r2[3]);
    C::template digest_kbc<double>(acc, AB[0], AB[1], AB[2], CD[0], CD[1], CD[2], 0.75, D6[3], r2[4]);
    C::template digest_kbd<double>(acc, AB[0], AB[1], AB[2], CD[0], CD[1], CD[2], 0.75, D6[2], r2[5]);
    double d = 0.0, mx = 0.0;
    for (int b = 0; b < 6; ++b)
      for (int t = 0; t < 64; ++t) {
        d = std::max(d, std::fabs(r1[b][t] - r2[b][t]));
        mx = std::max(mx, std::fabs(r1[b][t]));
      }
    return mx > 0.0 ? d / mx : -1.0;
  }
}

extern "C" double emu_sweeps(int cls) {
  switch (cls) {
#define S2(i, N) case i: return sweeps_diff<Cls_##N>();
    S2(0, ssss) S2(1, psss) S2(2, psps) S2(3, ppss) S2(4, ppps) S2(5, pppp) S2(6, dsss) S2(7, dsps)
    S2(8, dspp) S2(9, dsds) S2(10, dpss) S2(11, dpps) S2(12, dppp) S2(13, dpds) S2(14, dpdp)
    S2(15, ddss) S2(16, ddps) S2(17, ddpp) S2(18, ddds) S2(19, dddp) S2(20, dddd)
    default: return -2.0;
  }
}
