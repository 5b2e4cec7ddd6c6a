// Device-side building blocks of the J/K build for gfx950 (CDNA4, wave64).
//
// Layout of one "bin" (all unique shell pairs of one angular-momentum class and
// one primitive-pair count, sorted by Schwarz bound Q, descending):
//   prim  [npp][kPrimFields][n]  per primitive pair (SoA over pairs, so lanes
//                                that hold consecutive ket pairs load coalesced)
//   A     [3][n]   centre of the first shell        AB [3][n]  A - B
//   bf    [2][n]   first basis function of each shell
//   atoms [2][n]   atom of each shell               fpair [n]  1/2 if both shells coincide
//   Q     [n]      Cauchy-Schwarz factor sqrt(max (ab|ab))
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace jk {

constexpr int kWave = 64;
constexpr int kWavesPerBlock = 4;
constexpr int kBlock = kWave * kWavesPerBlock;
constexpr int kChunksPerItem = 16;          // ket chunks of one wave-width per work item
constexpr int kItemKets = kWave * kChunksPerItem;

// primitive-pair fields
enum : int { kP = 0, kOo2p = 1, kPAx = 2, kPAy = 3, kPAz = 4, kKt = 5, kTwoA = 6, kTwoB = 7,
             kPrimFields = 8 };

// FP64 Boys table: rows T_i = i * 0.05, i = 0..kBoysRows-1 (T < 64); columns
// F_m(T_i), m = 0..kBoysM-1, then exp(-T_i).
constexpr double kBoysStep = 0.05;
constexpr double kBoysInvStep = 20.0;
constexpr double kBoysTmax = 64.0;
constexpr int kBoysRows = 1281;
constexpr int kBoysM = 17;
constexpr int kBoysStride = 18;
// FP32 Boys table: rows T_i = i * 0.05 for T <= 30; columns m = 0..14, exp(-T_i).
constexpr float kBoys32Step = 0.05f;
constexpr float kBoys32InvStep = 20.0f;
constexpr int kBoys32Rows = 602;
constexpr int kBoys32M = 15;
constexpr int kBoys32Stride = 16;

struct BinView {
  int n, npp;
  const double* prim;
  const double* A;
  const double* AB;
  const int* bf;
  const int* atoms;
  const double* fpair;
  const double* Q;
};

struct EriLaunch {
  BinView bra, ket;
  const int4* items;  // {bra pair, first ket, end ket, unused}
  int nitems;
  int same_bin;       // bra and ket bins coincide (then ket == bra is a self-pair quartet)
  const double* D;
  double* J;
  double* K;
  int n;              // basis functions
  int n_dm;
  const double* boys64;
  const float* boys32;
  float boys_fp64_T;  // FP32 kernels: F_m in FP64 above this T
};

template <typename T>
struct VrrCoef {
  T PAx, PAy, PAz, WPx, WPy, WPz, QCx, QCy, QCz, WQx, WQy, WQz;
  T oo2p, oo2p_rp, oo2q, oo2q_rq, oo2pq;
};

__device__ constexpr double kInvOdd[24] = {
    1.0 / 1,  1.0 / 3,  1.0 / 5,  1.0 / 7,  1.0 / 9,  1.0 / 11, 1.0 / 13, 1.0 / 15,
    1.0 / 17, 1.0 / 19, 1.0 / 21, 1.0 / 23, 1.0 / 25, 1.0 / 27, 1.0 / 29, 1.0 / 31,
    1.0 / 33, 1.0 / 35, 1.0 / 37, 1.0 / 39, 1.0 / 41, 1.0 / 43, 1.0 / 45, 1.0 / 47};

constexpr double kPiOver4 = 0.78539816339744830961566084581988;

// F_m(T), m = 0..L, FP64.  T < 64: seven-term Taylor expansion about the nearest
// table point (|dT| <= 0.025, truncation below 2e-15 relative) for F_L, e^{-T}
// from the table value times a Taylor series of e^{-dT}, then the stable
// downward recursion F_m = (2T F_{m+1} + e^{-T}) / (2m+1).  T >= 64: the
// asymptotic F_0 = sqrt(pi/(4T)) and upward recursion F_{m+1} = (2m+1)/(2T) F_m
// (the dropped e^{-T} terms are below 1e-15 relative there for m <= 10).
template <int L>
__device__ __forceinline__ void boys_f64(double T, const double* __restrict__ tab, double* F) {
  if (T < kBoysTmax) {
    const int i = static_cast<int>(T * kBoysInvStep + 0.5);
    const double x = i * kBoysStep - T;
    const double* r = tab + i * kBoysStride;
    double s = r[L + 6];
    s = r[L + 5] + x * s * (1.0 / 6.0);
    s = r[L + 4] + x * s * (1.0 / 5.0);
    s = r[L + 3] + x * s * 0.25;
    s = r[L + 2] + x * s * (1.0 / 3.0);
    s = r[L + 1] + x * s * 0.5;
    s = r[L] + x * s;
    F[L] = s;
    if constexpr (L > 0) {
      double e = 1.0 + x * (1.0 / 6.0);
      e = 1.0 + x * 0.2 * e;
      e = 1.0 + x * 0.25 * e;
      e = 1.0 + x * (1.0 / 3.0) * e;
      e = 1.0 + x * 0.5 * e;
      e = 1.0 + x * e;
      e *= r[kBoysStride - 1];
      const double T2 = 2.0 * T;
#pragma unroll
      for (int m = L - 1; m >= 0; --m) F[m] = (T2 * F[m + 1] + e) * kInvOdd[m];
    }
  } else {
    const double rT = 1.0 / T;
    F[0] = sqrt(kPiOver4 * rT);
    const double h = 0.5 * rT;
#pragma unroll
    for (int m = 0; m < L; ++m) F[m + 1] = F[m] * ((2 * m + 1) * h);
  }
}

// F_m(T), m = 0..L, for the FP32 kernels.  T <= boys_fp64_T (<= 30): four-term
// Taylor expansion in FP32 from the FP32 table and downward recursion in FP32.
// Larger T: evaluated in FP64 (asymptotic F_0, upward recursion with the
// e^{-T} term) and rounded to FP32.
template <int L>
__device__ __forceinline__ void boys_f32(float T, float tcut, const float* __restrict__ tab,
                                         float* F) {
  if (T <= tcut) {
    const int i = static_cast<int>(T * kBoys32InvStep + 0.5f);
    const float x = i * kBoys32Step - T;
    const float* r = tab + i * kBoys32Stride;
    float s = r[L + 3];
    s = r[L + 2] + x * s * (1.0f / 3.0f);
    s = r[L + 1] + x * s * 0.5f;
    s = r[L] + x * s;
    F[L] = s;
    if constexpr (L > 0) {
      float e = 1.0f + x * 0.25f;
      e = 1.0f + x * (1.0f / 3.0f) * e;
      e = 1.0f + x * 0.5f * e;
      e = 1.0f + x * e;
      e *= r[kBoys32Stride - 1];
      const float T2 = 2.0f * T;
#pragma unroll
      for (int m = L - 1; m >= 0; --m) F[m] = (T2 * F[m + 1] + e) * static_cast<float>(kInvOdd[m]);
    }
  } else {
    const double Td = static_cast<double>(T);
    const double rT = 1.0 / Td;
    double f = sqrt(kPiOver4 * rT);
    F[0] = static_cast<float>(f);
    if constexpr (L > 0) {
      const double e = exp(-Td);
      const double h = 0.5 * rT;
#pragma unroll
      for (int m = 0; m < L; ++m) {
        f = ((2 * m + 1) * f - e) * h;
        F[m + 1] = static_cast<float>(f);
      }
    }
  }
}

template <int L, typename T>
struct Boys;
template <int L>
struct Boys<L, double> {
  __device__ __forceinline__ static void eval(double T, const EriLaunch& a, double* F) {
    boys_f64<L>(T, a.boys64, F);
  }
};
template <int L>
struct Boys<L, float> {
  __device__ __forceinline__ static void eval(float T, const EriLaunch& a, float* F) {
    boys_f32<L>(T, a.boys_fp64_T, a.boys32, F);
  }
};

// One primitive quartet: Boys values scaled by the prefactor and the
// recurrence coefficients.
//   P - Q = (P - A) - (Q - C) + (A - C)   (keeps FP32 differences small)
//   W - P = -q/(p+q) (P - Q),  W - Q = p/(p+q) (P - Q),  rho = pq/(p+q)
//   prefactor = 2 pi^{5/2} K_AB K_CD / (p q sqrt(p+q)) = Kt_AB Kt_CD / sqrt(p+q)
template <int L, typename T>
__device__ __forceinline__ void prim_setup(T p, T oo2p, T PAx, T PAy, T PAz, T Kab, T q, T oo2q,
                                           T QCx, T QCy, T QCz, T Kcd, T ACx, T ACy, T ACz,
                                           const EriLaunch& a, T* F, VrrCoef<T>& c) {
  const T rpq = T(1) / (p + q);
  const T qr = q * rpq, pr = p * rpq;
  const T PQx = PAx - QCx + ACx, PQy = PAy - QCy + ACy, PQz = PAz - QCz + ACz;
  const T Tb = p * qr * (PQx * PQx + PQy * PQy + PQz * PQz);
  Boys<L, T>::eval(Tb, a, F);
  const T pref = Kab * Kcd * sqrt(rpq);
#pragma unroll
  for (int m = 0; m <= L; ++m) F[m] *= pref;
  c.PAx = PAx; c.PAy = PAy; c.PAz = PAz;
  c.QCx = QCx; c.QCy = QCy; c.QCz = QCz;
  c.WPx = -qr * PQx; c.WPy = -qr * PQy; c.WPz = -qr * PQz;
  c.WQx = pr * PQx; c.WQy = pr * PQy; c.WQz = pr * PQz;
  c.oo2p = oo2p; c.oo2p_rp = oo2p * qr;
  c.oo2q = oo2q; c.oo2q_rq = oo2q * pr;
  c.oo2pq = T(0.5) * rpq;
}

// Contraction loop of one shell quartet: bra pair i (uniform in the ERI
// kernels), ket pair k (one per lane); `vrr(F, c)` adds one primitive quartet
// to the caller's accumulators.
template <int L, typename T, class V>
__device__ __forceinline__ void contract(const EriLaunch& a, int i, int k, T ACx, T ACy, T ACz,
                                         V&& vrr) {
  const int nb = a.bra.n, nk = a.ket.n;
  const int nppb = a.bra.npp, nppk = a.ket.npp;
  for (int kl = 0; kl < nppk; ++kl) {
    const double* kp = a.ket.prim + static_cast<size_t>(kl) * kPrimFields * nk + k;
    const T q = T(kp[kP * nk]), oo2q = T(kp[kOo2p * nk]);
    const T QCx = T(kp[kPAx * nk]), QCy = T(kp[kPAy * nk]), QCz = T(kp[kPAz * nk]);
    const T Kcd = T(kp[kKt * nk]);
    for (int ij = 0; ij < nppb; ++ij) {
      const double* bp = a.bra.prim + static_cast<size_t>(ij) * kPrimFields * nb + i;
      T F[L + 1];
      VrrCoef<T> c;
      prim_setup<L, T>(T(bp[kP * nb]), T(bp[kOo2p * nb]), T(bp[kPAx * nb]), T(bp[kPAy * nb]),
                       T(bp[kPAz * nb]), T(bp[kKt * nb]), q, oo2q, QCx, QCy, QCz, Kcd, ACx, ACy,
                       ACz, a, F, c);
      vrr(F, c);
    }
  }
}

// A zero the compiler cannot see through: indexing a private array with it
// keeps the array in scratch memory instead of registers.
__device__ __forceinline__ int opaque_zero() {
  int z;
  asm volatile("s_mov_b32 %0, 0" : "=s"(z));
  return z;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

__device__ __forceinline__ void atomic_add(double* addr, double v) {
  unsafeAtomicAdd(addr, v);
}

// Integral + digestion kernel of one class and precision.  One wavefront per
// work item: the bra pair is uniform across the wave (scalar data), each lane
// takes one ket pair of the current 64-wide chunk of the item's ket range.
template <class C, typename T>
__global__ __launch_bounds__(kBlock) void eri_jk_kernel(const EriLaunch a) {
  const int lane = threadIdx.x & (kWave - 1);
  const int item = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  if (item >= a.nitems) return;
  const int4 w = a.items[item];
  const int i = __builtin_amdgcn_readfirstlane(w.x);
  const int kbeg = __builtin_amdgcn_readfirstlane(w.y);
  const int kend = __builtin_amdgcn_readfirstlane(w.z);
  const int nb = a.bra.n, nk = a.ket.n;
  const size_t nn = static_cast<size_t>(a.n) * a.n;

  const double Ax = a.bra.A[i], Ay = a.bra.A[nb + i], Az = a.bra.A[2 * nb + i];
  const T ABx = T(a.bra.AB[i]), ABy = T(a.bra.AB[nb + i]), ABz = T(a.bra.AB[2 * nb + i]);
  const int a0 = a.bra.bf[i], b0 = a.bra.bf[nb + i];
  const double fbra = a.bra.fpair[i];

  for (int kc = kbeg; kc < kend; kc += kWave) {
    const bool active = kc + lane < kend;
    const int k = active ? kc + lane : kend - 1;
    const T ACx = T(Ax - a.ket.A[k]), ACy = T(Ay - a.ket.A[nk + k]),
            ACz = T(Az - a.ket.A[2 * nk + k]);
    T acc[C::NACC];
#pragma unroll
    for (int t = 0; t < C::NACC; ++t) acc[t] = T(0);
    contract<C::L, T>(a, i, k, ACx, ACy, ACz,
                      [&](const T* F, const VrrCoef<T>& c) { C::template vrr<T>(F, c, acc); });

    const T CDx = T(a.ket.AB[k]), CDy = T(a.ket.AB[nk + k]), CDz = T(a.ket.AB[2 * nk + k]);
    const int c0 = a.ket.bf[k], d0 = a.ket.bf[nk + k];
    const double fq =
        active ? fbra * a.ket.fpair[k] * ((a.same_bin && k == i) ? 0.5 : 1.0) : 0.0;

    for (int m = 0; m < a.n_dm; ++m) {
      const double* Dm = a.D + m * nn;
      double Dab[C::NA * C::NB], Dcd[C::NC * C::ND], Dac[C::NA * C::NC], Dad[C::NA * C::ND],
          Dbc[C::NB * C::NC], Dbd[C::NB * C::ND];
#pragma unroll
      for (int x = 0; x < C::NA; ++x) {
#pragma unroll
        for (int y = 0; y < C::NB; ++y) Dab[x * C::NB + y] = Dm[(a0 + x) * static_cast<size_t>(a.n) + b0 + y];
#pragma unroll
        for (int y = 0; y < C::NC; ++y) Dac[x * C::NC + y] = Dm[(a0 + x) * static_cast<size_t>(a.n) + c0 + y];
#pragma unroll
        for (int y = 0; y < C::ND; ++y) Dad[x * C::ND + y] = Dm[(a0 + x) * static_cast<size_t>(a.n) + d0 + y];
      }
#pragma unroll
      for (int x = 0; x < C::NB; ++x) {
#pragma unroll
        for (int y = 0; y < C::NC; ++y) Dbc[x * C::NC + y] = Dm[(b0 + x) * static_cast<size_t>(a.n) + c0 + y];
#pragma unroll
        for (int y = 0; y < C::ND; ++y) Dbd[x * C::ND + y] = Dm[(b0 + x) * static_cast<size_t>(a.n) + d0 + y];
      }
#pragma unroll
      for (int x = 0; x < C::NC; ++x)
#pragma unroll
        for (int y = 0; y < C::ND; ++y) Dcd[x * C::ND + y] = Dm[(c0 + x) * static_cast<size_t>(a.n) + d0 + y];

      double jab[C::NA * C::NB], jcd[C::NC * C::ND], kac[C::NA * C::NC], kad[C::NA * C::ND],
          kbc[C::NB * C::NC], kbd[C::NB * C::ND];
#pragma unroll
      for (int t = 0; t < C::NA * C::NB; ++t) jab[t] = 0.0;
#pragma unroll
      for (int t = 0; t < C::NC * C::ND; ++t) jcd[t] = 0.0;
#pragma unroll
      for (int t = 0; t < C::NA * C::NC; ++t) kac[t] = 0.0;
#pragma unroll
      for (int t = 0; t < C::NA * C::ND; ++t) kad[t] = 0.0;
#pragma unroll
      for (int t = 0; t < C::NB * C::NC; ++t) kbc[t] = 0.0;
#pragma unroll
      for (int t = 0; t < C::NB * C::ND; ++t) kbd[t] = 0.0;

      C::template hrr_digest<T>(acc, ABx, ABy, ABz, CDx, CDy, CDz, fq, Dab, Dcd, Dac, Dad, Dbc,
                                Dbd, jab, jcd, kac, kad, kbc, kbd);

      double* Jm = a.J + m * nn;
      double* Km = a.K + m * nn;
#pragma unroll
      for (int t = 0; t < C::NA * C::NB; ++t) {
        const double s = wave_sum(jab[t]);
        if (lane == 0)
          atomic_add(&Jm[(a0 + t / C::NB) * static_cast<size_t>(a.n) + b0 + t % C::NB], 2.0 * s);
      }
      if (active) {
#pragma unroll
        for (int t = 0; t < C::NC * C::ND; ++t)
          atomic_add(&Jm[(c0 + t / C::ND) * static_cast<size_t>(a.n) + d0 + t % C::ND], 2.0 * jcd[t]);
#pragma unroll
        for (int t = 0; t < C::NA * C::NC; ++t)
          atomic_add(&Km[(a0 + t / C::NC) * static_cast<size_t>(a.n) + c0 + t % C::NC], kac[t]);
#pragma unroll
        for (int t = 0; t < C::NA * C::ND; ++t)
          atomic_add(&Km[(a0 + t / C::ND) * static_cast<size_t>(a.n) + d0 + t % C::ND], kad[t]);
#pragma unroll
        for (int t = 0; t < C::NB * C::NC; ++t)
          atomic_add(&Km[(b0 + t / C::NC) * static_cast<size_t>(a.n) + c0 + t % C::NC], kbc[t]);
#pragma unroll
        for (int t = 0; t < C::NB * C::ND; ++t)
          atomic_add(&Km[(b0 + t / C::ND) * static_cast<size_t>(a.n) + d0 + t % C::ND], kbd[t]);
      }
    }
  }
}

// Cauchy-Schwarz factor of every pair of a bin: Q = sqrt(max_ab (ab|ab)).
// One lane per pair; bra and ket are the same pair, so A - C = 0.
template <class C>
__global__ __launch_bounds__(kBlock) void schwarz_kernel(const EriLaunch a, double* Qout) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  const int n = a.bra.n;
  if (t >= n) return;
  double acc[C::NACC];
#pragma unroll
  for (int s = 0; s < C::NACC; ++s) acc[s] = 0.0;
  contract<C::L, double>(a, t, t, 0.0, 0.0, 0.0, [&](const double* F, const VrrCoef<double>& c) {
    C::template vrr<double>(F, c, acc);
  });
  const double mx = C::template diag_max<double>(acc, a.bra.AB[t], a.bra.AB[n + t], a.bra.AB[2 * n + t]);
  Qout[t] = sqrt(fmax(mx, 0.0));
}

// ---------------------------------------------------------------------------------
// Multi-pass form for the classes with many contracted intermediates.  Pass J
// accumulates [e0|f0] for every e and a chunk of f in registers over the whole
// primitive loop and parks the chunk in a private (scratch) array; the
// horizontal recurrences then run as short loops: the ket step for one e at a
// time into X[e][cd], the bra step plus digestion for one (c, d) at a time.
template <class C, typename T, int J>
__device__ __forceinline__ void split_passes(const EriLaunch& a, int i, int k, T ACx, T ACy,
                                             T ACz, T* cacc, int z) {
  constexpr int NFJ = C::template Pass<J>::NF, F0 = C::template Pass<J>::F0;
  T acc[C::NE * NFJ];
#pragma unroll
  for (int t = 0; t < C::NE * NFJ; ++t) acc[t] = T(0);
  contract<C::L, T>(a, i, k, ACx, ACy, ACz, [&](const T* F, const VrrCoef<T>& c) {
    C::template vrr_pass<J, T>(F, c, acc);
  });
#pragma unroll
  for (int e = 0; e < C::NE; ++e)
#pragma unroll
    for (int f = 0; f < NFJ; ++f) cacc[z + e * C::NF + F0 + f] = acc[e * NFJ + f];
  if constexpr (J + 1 < C::NPASS) split_passes<C, T, J + 1>(a, i, k, ACx, ACy, ACz, cacc, z);
}

template <class C, typename T>
__device__ __forceinline__ void split_ket_hrr(const T* cacc, T* X, int z, T CDx, T CDy, T CDz) {
  constexpr int NCD = C::NC * C::ND;
#pragma nounroll
  for (int e = 0; e < C::NE; ++e) {
    T f[C::NF];
#pragma unroll
    for (int t = 0; t < C::NF; ++t) f[t] = cacc[z + e * C::NF + t];
    T o[NCD];
    C::template ket_hrr<T>(f, CDx, CDy, CDz, o);
#pragma unroll
    for (int t = 0; t < NCD; ++t) X[z + e * NCD + t] = o[t];
  }
}

template <class C, typename T>
__global__ __launch_bounds__(kBlock) void eri_jk_split_kernel(const EriLaunch a) {
  constexpr int NCD = C::NC * C::ND;
  const int lane = threadIdx.x & (kWave - 1);
  const int item = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  if (item >= a.nitems) return;
  const int4 w = a.items[item];
  const int i = __builtin_amdgcn_readfirstlane(w.x);
  const int kbeg = __builtin_amdgcn_readfirstlane(w.y);
  const int kend = __builtin_amdgcn_readfirstlane(w.z);
  const int nb = a.bra.n, nk = a.ket.n;
  const size_t n = static_cast<size_t>(a.n);
  const size_t nn = n * n;
  const double Ax = a.bra.A[i], Ay = a.bra.A[nb + i], Az = a.bra.A[2 * nb + i];
  const T ABx = T(a.bra.AB[i]), ABy = T(a.bra.AB[nb + i]), ABz = T(a.bra.AB[2 * nb + i]);
  const int a0 = a.bra.bf[i], b0 = a.bra.bf[nb + i];
  const double fbra = a.bra.fpair[i];
  const int z = opaque_zero();

  for (int kc = kbeg; kc < kend; kc += kWave) {
    const bool active = kc + lane < kend;
    const int k = active ? kc + lane : kend - 1;
    const T ACx = T(Ax - a.ket.A[k]), ACy = T(Ay - a.ket.A[nk + k]),
            ACz = T(Az - a.ket.A[2 * nk + k]);
    T cacc[C::NACC];
    split_passes<C, T, 0>(a, i, k, ACx, ACy, ACz, cacc, z);
    const T CDx = T(a.ket.AB[k]), CDy = T(a.ket.AB[nk + k]), CDz = T(a.ket.AB[2 * nk + k]);
    T X[C::NE * NCD];
    split_ket_hrr<C, T>(cacc, X, z, CDx, CDy, CDz);
    const int c0 = a.ket.bf[k], d0 = a.ket.bf[nk + k];
    const double fq =
        active ? fbra * a.ket.fpair[k] * ((a.same_bin && k == i) ? 0.5 : 1.0) : 0.0;

    for (int m = 0; m < a.n_dm; ++m) {
      const double* Dm = a.D + m * nn;
      double* Jm = a.J + m * nn;
      double* Km = a.K + m * nn;
      double Dab[C::NA * C::NB], jab[C::NA * C::NB];
#pragma unroll
      for (int x = 0; x < C::NA; ++x)
#pragma unroll
        for (int y = 0; y < C::NB; ++y) {
          Dab[x * C::NB + y] = Dm[(a0 + x) * n + b0 + y];
          jab[x * C::NB + y] = 0.0;
        }
      double kac[C::NA * C::NC], kad[C::NA * C::ND], kbc[C::NB * C::NC], kbd[C::NB * C::ND];
#pragma unroll
      for (int t = 0; t < C::NA * C::NC; ++t) kac[z + t] = 0.0;
#pragma unroll
      for (int t = 0; t < C::NA * C::ND; ++t) kad[z + t] = 0.0;
#pragma unroll
      for (int t = 0; t < C::NB * C::NC; ++t) kbc[z + t] = 0.0;
#pragma unroll
      for (int t = 0; t < C::NB * C::ND; ++t) kbd[z + t] = 0.0;

#pragma nounroll
      for (int cd = 0; cd < NCD; ++cd) {
        const int c = cd / C::ND, d = cd % C::ND;
        T ev[C::NE];
#pragma unroll
        for (int e = 0; e < C::NE; ++e) ev[e] = X[z + e * NCD + cd];
        T ab[C::NA * C::NB];
        C::template bra_hrr<T>(ev, ABx, ABy, ABz, ab);
        const double Dcd = Dm[(c0 + c) * n + d0 + d];
        double Dbd[C::NB], Dbc[C::NB], Dad[C::NA], Dac[C::NA];
#pragma unroll
        for (int y = 0; y < C::NB; ++y) {
          Dbd[y] = Dm[(b0 + y) * n + d0 + d];
          Dbc[y] = Dm[(b0 + y) * n + c0 + c];
        }
#pragma unroll
        for (int x = 0; x < C::NA; ++x) {
          Dad[x] = Dm[(a0 + x) * n + d0 + d];
          Dac[x] = Dm[(a0 + x) * n + c0 + c];
        }
        double jcd = 0.0, tac[C::NA], tad[C::NA], tbc[C::NB], tbd[C::NB];
#pragma unroll
        for (int x = 0; x < C::NA; ++x) tac[x] = tad[x] = 0.0;
#pragma unroll
        for (int y = 0; y < C::NB; ++y) tbc[y] = tbd[y] = 0.0;
#pragma unroll
        for (int x = 0; x < C::NA; ++x)
#pragma unroll
          for (int y = 0; y < C::NB; ++y) {
            const double v = static_cast<double>(ab[x * C::NB + y]) * fq;
            jab[x * C::NB + y] += Dcd * v;
            jcd += Dab[x * C::NB + y] * v;
            tac[x] += Dbd[y] * v;
            tad[x] += Dbc[y] * v;
            tbc[y] += Dad[x] * v;
            tbd[y] += Dac[x] * v;
          }
        if (active) atomic_add(&Jm[(c0 + c) * n + d0 + d], 2.0 * jcd);
#pragma unroll
        for (int x = 0; x < C::NA; ++x) {
          kac[z + x * C::NC + c] += tac[x];
          kad[z + x * C::ND + d] += tad[x];
        }
#pragma unroll
        for (int y = 0; y < C::NB; ++y) {
          kbc[z + y * C::NC + c] += tbc[y];
          kbd[z + y * C::ND + d] += tbd[y];
        }
      }
#pragma unroll
      for (int t = 0; t < C::NA * C::NB; ++t) {
        const double s = wave_sum(jab[t]);
        if (lane == 0) atomic_add(&Jm[(a0 + t / C::NB) * n + b0 + t % C::NB], 2.0 * s);
      }
      if (active) {
#pragma unroll
        for (int t = 0; t < C::NA * C::NC; ++t)
          atomic_add(&Km[(a0 + t / C::NC) * n + c0 + t % C::NC], kac[z + t]);
#pragma unroll
        for (int t = 0; t < C::NA * C::ND; ++t)
          atomic_add(&Km[(a0 + t / C::ND) * n + d0 + t % C::ND], kad[z + t]);
#pragma unroll
        for (int t = 0; t < C::NB * C::NC; ++t)
          atomic_add(&Km[(b0 + t / C::NC) * n + c0 + t % C::NC], kbc[z + t]);
#pragma unroll
        for (int t = 0; t < C::NB * C::ND; ++t)
          atomic_add(&Km[(b0 + t / C::ND) * n + d0 + t % C::ND], kbd[z + t]);
      }
    }
  }
}

template <class C>
__global__ __launch_bounds__(kBlock) void schwarz_split_kernel(const EriLaunch a, double* Qout) {
  constexpr int NCD = C::NC * C::ND;
  const int t = blockIdx.x * kBlock + threadIdx.x;
  const int n = a.bra.n;
  if (t >= n) return;
  const int z = opaque_zero();
  double cacc[C::NACC];
  split_passes<C, double, 0>(a, t, t, 0.0, 0.0, 0.0, cacc, z);
  const double ABx = a.bra.AB[t], ABy = a.bra.AB[n + t], ABz = a.bra.AB[2 * n + t];
  double X[C::NE * NCD];
  split_ket_hrr<C, double>(cacc, X, z, ABx, ABy, ABz);
  double mx = 0.0;
#pragma nounroll
  for (int cd = 0; cd < NCD; ++cd) {
    double ev[C::NE];
#pragma unroll
    for (int e = 0; e < C::NE; ++e) ev[e] = X[z + e * NCD + cd];
    double ab[C::NA * C::NB];
    C::template bra_hrr<double>(ev, ABx, ABy, ABz, ab);
#pragma unroll
    for (int s = 0; s < C::NA * C::NB; ++s)
      if (s == cd) mx = fmax(mx, ab[s]);
  }
  Qout[t] = sqrt(fmax(mx, 0.0));
}

}  // namespace jk
