// Host build of the generated gradient-class code: the full nuclear gradient of a small
// molecule summed over unique quartets, for comparison with the oracle (test harness).
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>
#include <algorithm>
#define __device__
#define __forceinline__ inline
namespace jk {
template <typename T> struct VrrCoef {
  T PAx, PAy, PAz, WPx, WPy, WPz, QCx, QCy, QCz, WQx, WQy, WQz;
  T oo2p, oo2p_rp, oo2q, oo2q_rq, oo2pq;
};
#include "gcls_ssss.inc"
#include "gcls_psss.inc"
#include "gcls_psps.inc"
#include "gcls_ppss.inc"
#include "gcls_ppps.inc"
#include "gcls_pppp.inc"
#include "gcls_dsss.inc"
#include "gcls_dsps.inc"
#include "gcls_dspp.inc"
#include "gcls_dsds.inc"
#include "gcls_dpss.inc"
#include "gcls_dpps.inc"
#include "gcls_dppp.inc"
#include "gcls_dpds.inc"
#include "gcls_dpdp.inc"
#include "gcls_ddss.inc"
#include "gcls_ddps.inc"
#include "gcls_ddpp.inc"
#include "gcls_ddds.inc"
#include "gcls_dddp.inc"
#include "gcls_dddd.inc"
}
using namespace jk;
static double boys_exact(int m, double T) {
  long double term = 1.0L / (2 * m + 1), sum = term;
  for (int k = 1; k < 100000; ++k) { term *= 2.0L * T / (2 * m + 2 * k + 1); sum += term; if (term < sum * 1e-21L) break; }
  return (double)(std::exp(-(long double)T) * sum);
}
struct Sh { int l, np, bf, atom; double A[3]; double e[8], c[8]; };
struct Arr { std::vector<double> v; double& operator[](int i) { return v[i]; } };
struct ArrRef { double* p; double& operator[](int i) const { return p[i]; } };

template <class C, int J>
static void passes(const Sh& a, const Sh& b, const Sh& c, const Sh& d, double* G) {
  constexpr int N = C::template Pass<J>::N;
  double acc[N] = {0};
  const double PI = 3.14159265358979323846;
  for (int i = 0; i < a.np; ++i) for (int j = 0; j < b.np; ++j)
  for (int k = 0; k < c.np; ++k) for (int l = 0; l < d.np; ++l) {
    double p = a.e[i] + b.e[j], q = c.e[k] + d.e[l];
    double P[3], Q[3], AB2 = 0, CD2 = 0;
    for (int x = 0; x < 3; ++x) {
      P[x] = (a.e[i] * a.A[x] + b.e[j] * b.A[x]) / p; Q[x] = (c.e[k] * c.A[x] + d.e[l] * d.A[x]) / q;
      AB2 += (a.A[x] - b.A[x]) * (a.A[x] - b.A[x]); CD2 += (c.A[x] - d.A[x]) * (c.A[x] - d.A[x]);
    }
    double W[3], PQ2 = 0;
    for (int x = 0; x < 3; ++x) { W[x] = (p * P[x] + q * Q[x]) / (p + q); PQ2 += (P[x] - Q[x]) * (P[x] - Q[x]); }
    double rho = p * q / (p + q), T = rho * PQ2;
    double pref = 2 * std::pow(PI, 2.5) / (p * q * std::sqrt(p + q)) * a.c[i] * b.c[j] * c.c[k] * d.c[l] *
                  std::exp(-a.e[i] * b.e[j] / p * AB2) * std::exp(-c.e[k] * d.e[l] / q * CD2);
    double F[16];
    for (int m = 0; m <= C::L; ++m) F[m] = pref * boys_exact(m, T);
    VrrCoef<double> cf;
    cf.PAx = P[0] - a.A[0]; cf.PAy = P[1] - a.A[1]; cf.PAz = P[2] - a.A[2];
    cf.WPx = W[0] - P[0]; cf.WPy = W[1] - P[1]; cf.WPz = W[2] - P[2];
    cf.QCx = Q[0] - c.A[0]; cf.QCy = Q[1] - c.A[1]; cf.QCz = Q[2] - c.A[2];
    cf.WQx = W[0] - Q[0]; cf.WQy = W[1] - Q[1]; cf.WQz = W[2] - Q[2];
    cf.oo2p = 0.5 / p; cf.oo2p_rp = 0.5 / p * rho / p; cf.oo2q = 0.5 / q; cf.oo2q_rq = 0.5 / q * rho / q;
    cf.oo2pq = 0.5 / (p + q);
    C::template vrr_pass<J, double>(F, cf, 2 * a.e[i], 2 * b.e[j], 2 * c.e[k], acc);
  }
  C::template store_pass<J, double, ArrRef>(acc, ArrRef{G}, 0);
  if constexpr (J + 1 < C::NPASS) passes<C, J + 1>(a, b, c, d, G);
}

// gradient contributions gA, gB, gC (per density, nd=1) of one quartet, times f
template <class C>
static void quartet(const Sh& a, const Sh& b, const Sh& c, const Sh& d, const double* D, int n,
                    double f, double* grad) {
  constexpr int NCD = C::NC * C::ND, NAB = C::NA * C::NB;
  std::vector<double> G(C::NG), XA(C::NE_A * NCD), XB(C::NE_B * NCD), XC(C::NE_C * C::NCP),
      XU(std::max(1, C::NE_U * NCD)), XV(std::max(1, C::NE_U * std::max(1, C::NCM)));
  passes<C, 0>(a, b, c, d, G.data());
  double ABx = a.A[0] - b.A[0], ABy = a.A[1] - b.A[1], ABz = a.A[2] - b.A[2];
  double CDx = c.A[0] - d.A[0], CDy = c.A[1] - d.A[1], CDz = c.A[2] - d.A[2];
  for (int e = 0; e < C::NE_A; ++e) C::template ket_b<double>(&G[C::OFF_A + e * C::NF_A], CDx, CDy, CDz, &XA[e * NCD]);
  for (int e = 0; e < C::NE_B; ++e) C::template ket_b<double>(&G[C::OFF_B + e * C::NF_B], CDx, CDy, CDz, &XB[e * NCD]);
  for (int e = 0; e < C::NE_C; ++e) C::template ket_p<double>(&G[C::OFF_C + e * C::NF_C], CDx, CDy, CDz, &XC[e * C::NCP]);
  if constexpr (C::USE_U) {
    for (int e = 0; e < C::NE_U; ++e) {
      C::template ket_b<double>(&G[C::OFF_U + e * C::NF_U] + C::U_FB, CDx, CDy, CDz, &XU[e * NCD]);
      if constexpr (C::NCM > 0) C::template ket_m<double>(&G[C::OFF_U + e * C::NF_U], CDx, CDy, CDz, &XV[e * C::NCM]);
    }
  }
  double gA[3] = {0}, gB[3] = {0}, gC[3] = {0};
  int a0 = a.bf, b0 = b.bf, c0 = c.bf, d0 = d.bf;
  for (int cd = 0; cd < NCD; ++cd) {
    int cc = cd / C::ND, dd = cd % C::ND;
    double Gam[NAB];
    for (int x = 0; x < C::NA; ++x) for (int y = 0; y < C::NB; ++y)
      Gam[x * C::NB + y] = 0.5 * D[(a0 + x) * n + b0 + y] * D[(c0 + cc) * n + d0 + dd] -
                           0.125 * (D[(a0 + x) * n + c0 + cc] * D[(b0 + y) * n + d0 + dd] + D[(a0 + x) * n + d0 + dd] * D[(b0 + y) * n + c0 + cc]);
    double ea[64], eb[64], xap[128], xbp[128], xam[64] = {0}, xbm[64] = {0};
    for (int e = 0; e < C::NE_A; ++e) ea[e] = XA[e * NCD + cd];
    for (int e = 0; e < C::NE_B; ++e) eb[e] = XB[e * NCD + cd];
    C::template bra_ap<double>(ea, ABx, ABy, ABz, xap);
    C::template bra_bp<double>(eb, ABx, ABy, ABz, xbp);
    if constexpr (C::LA >= 1) { double em[64]; for (int e = 0; e < C::NE_AM; ++e) em[e] = XU[e * NCD + cd]; C::template bra_am<double>(em, ABx, ABy, ABz, xam); }
    if constexpr (C::LB >= 1) { double em[64]; for (int e = 0; e < C::NE_BM; ++e) em[e] = XU[(C::U_EB + e) * NCD + cd]; C::template bra_bm<double>(em, ABx, ABy, ABz, xbm); }
    C::template contract_ab<double>(Gam, xap, xam, xbp, xbm, gA, gB);
    for (int x = 0; x < 3; ++x) {
      int cp = C::CPLUS[cc][x];
      double e0[64], x0[64];
      for (int e = 0; e < C::NE_0; ++e) e0[e] = XC[e * C::NCP + cp * C::ND + dd];
      C::template bra_0<double>(e0, ABx, ABy, ABz, x0);
      gC[x] += C::template dot0<double>(Gam, x0);
      if constexpr (C::LC >= 1) {
        int pw = C::CPOW[cc][x];
        if (pw > 0) {
          int cm = C::CMINUS[cc][x];
          for (int e = 0; e < C::NE_0; ++e) e0[e] = XV[(C::U_EB + e) * C::NCM + cm * C::ND + dd];
          C::template bra_0<double>(e0, ABx, ABy, ABz, x0);
          gC[x] -= pw * C::template dot0<double>(Gam, x0);
        }
      }
    }
  }
  for (int x = 0; x < 3; ++x) {
    grad[a.atom * 3 + x] += f * gA[x]; grad[b.atom * 3 + x] += f * gB[x]; grad[c.atom * 3 + x] += f * gC[x];
    grad[d.atom * 3 + x] -= f * (gA[x] + gB[x] + gC[x]);
  }
}

extern "C" int emu_grad(int ns, const int* l, const int* atom, const double* xyz, const double* e,
                        const double* cf, const int* prim0, const int* np, const double* D, int n, double* grad) {
  std::vector<Sh> sh(ns);
  int bf = 0;
  for (int s = 0; s < ns; ++s) {
    sh[s].l = l[s]; sh[s].np = np[s]; sh[s].atom = atom[s]; sh[s].bf = bf; bf += (l[s] + 1) * (l[s] + 2) / 2;
    for (int x = 0; x < 3; ++x) sh[s].A[x] = xyz[3 * atom[s] + x];
    for (int k = 0; k < np[s]; ++k) { sh[s].e[k] = e[prim0[s] + k]; sh[s].c[k] = cf[prim0[s] + k]; }
  }
  // canonical pairs (higher l first); pair classes
  static const int PC[3][3] = {{0, -1, -1}, {1, 2, -1}, {3, 4, 5}};
  struct Pr { int s1, s2, cls; };
  std::vector<Pr> pr;
  for (int i = 0; i < ns; ++i) for (int j = 0; j <= i; ++j) {
    int s1 = i, s2 = j; if (sh[s2].l > sh[s1].l) std::swap(s1, s2);
    pr.push_back({s1, s2, PC[sh[s1].l][sh[s2].l]});
  }
  for (size_t P = 0; P < pr.size(); ++P) for (size_t Q = 0; Q <= P; ++Q) {
    Pr bra = pr[P], ket = pr[Q];
    if (ket.cls > bra.cls) std::swap(bra, ket);
    double f = 8.0;
    if (bra.s1 == bra.s2) f *= 0.5; if (ket.s1 == ket.s2) f *= 0.5; if (P == Q) f *= 0.5;
    const Sh &a = sh[bra.s1], &b = sh[bra.s2], &c = sh[ket.s1], &d = sh[ket.s2];
    int q = bra.cls * (bra.cls + 1) / 2 + ket.cls;
    switch (q) {
#define Q1(i, N) case i: quartet<GCls_##N>(a, b, c, d, D, n, f, grad); break;
      Q1(0, ssss) Q1(1, psss) Q1(2, psps) Q1(3, ppss) Q1(4, ppps) Q1(5, pppp) Q1(6, dsss) Q1(7, dsps)
      Q1(8, dspp) Q1(9, dsds) Q1(10, dpss) Q1(11, dpps) Q1(12, dppp) Q1(13, dpds) Q1(14, dpdp)
      Q1(15, ddss) Q1(16, ddps) Q1(17, ddpp) Q1(18, ddds) Q1(19, dddp) Q1(20, dddd)
    }
  }
  return 0;
}
