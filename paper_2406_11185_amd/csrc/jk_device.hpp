// Device-side building blocks of the J/K build for gfx950 (CDNA4, wave64).
//
// Layout of one "bin" (all unique shell pairs of one angular-momentum class and
// one primitive-pair count, sorted by Schwarz bound Q, descending):
//   prim  [npp][kPrimFields][n]  per primitive pair (SoA over pairs, so lanes
//                                that hold consecutive ket pairs load coalesced)
//   primT [n][npp][kPrimFields]  the same, pair-major (one bra pair's primitive
//                                pairs are contiguous: scalar loads)
//   A     [3][n]   centre of the first shell        AB [3][n]  A - B
//   bf    [2][n]   first basis function of each shell
//   atoms [2][n]   atom of each shell               fpair [n]  1/2 if both shells coincide
//   Q     [n]      Cauchy-Schwarz factor sqrt(max (ab|ab))
#pragma once
#include <hip/hip_runtime.h>
#include <algorithm>
#include <cstdint>

namespace jk {

constexpr int kWave = 64;
constexpr int kWavesPerBlock = 4;
constexpr int kBlock = kWave * kWavesPerBlock;
constexpr int kSchwarzSplitLanes = 64;   // multi-pass diagonal classes: lanes per pair
constexpr int kMaxItemChunks = 16;   // a work item covers 1..16 wave-wide ket chunks
#ifndef JK_TARGET_WAVES
#define JK_TARGET_WAVES 8192
#endif
constexpr int kTargetWaves = JK_TARGET_WAVES;   // aim for this many work items per class launch
#ifndef JK_SPLIT_TARGET_WAVES
#define JK_SPLIT_TARGET_WAVES (JK_TARGET_WAVES / 4)
#endif
// multi-pass classes: wavefronts their lane count aims for.  They run one
// wavefront per SIMD, so fewer fill the chip, and fewer lanes per quartet mean
// fewer cross-lane sums of the pass accumulators (measured on gfx950 for the
// 270-function molecule: (dd|dp) 3.25 -> 2.08 ms with 4 instead of 16 lanes at
// 2048; at 1024 (dp|dp) and (dd|ds) lose more than that)
constexpr int kSplitTargetWaves = JK_SPLIT_TARGET_WAVES;

// Wavefronts per SIMD a class kernel is compiled for (its register budget:
// 512 / waves registers per lane), per precision; generated per class as
// C::WAVES64 / C::WAVES32.
template <class C, typename T>
constexpr int class_waves() {
  return sizeof(T) == 8 ? C::WAVES64 : C::WAVES32;
}

// primitive-pair fields
enum : int { kP = 0, kOo2p = 1, kPAx = 2, kPAy = 3, kPAz = 4, kKt = 5, kTwoA = 6, kTwoB = 7,
             kPrimFields = 8 };

// FP64 Boys tables, one per order L = 0..kBoysMaxL: rows T_i = i * 0.05,
// i = 0..kBoysRows-1 (T < 64), each row one 64-byte line
// [F_L(T_i), ..., F_{L+6}(T_i), exp(-T_i)].
constexpr double kBoysStep = 0.05;
constexpr double kBoysInvStep = 20.0;
constexpr double kBoysTmax = 64.0;
constexpr int kBoysRows = 1281;
constexpr int kBoysMaxL = 10;
constexpr int kBoysRow = 8;
// FP32 Boys tables per order L: rows T_i = i * 0.05 for T <= 30, each row 32
// bytes [F_L, F_{L+1}, F_{L+2}, F_{L+3}, exp(-T_i), 0, 0, 0].
constexpr float kBoys32Step = 0.05f;
constexpr float kBoys32InvStep = 20.0f;
constexpr int kBoys32Rows = 602;
constexpr int kBoys32Row = 8;

struct BinView {
  int n, npp;
  const double* prim;
  const double* primT;   // the same primitive-pair fields pair-major: [n][npp][kPrimFields]
  const float* prim32;   // FP32 copies of prim and primT (the FP32 kernels read these)
  const float* primT32;
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
  double* J;           // accumulators A_J, A_K (the build returns A + A^T)
  double* K;
  int ncopy;           // independent accumulator copies (item % ncopy), spreading the
  size_t copy_stride;  // atomic traffic of small matrices over more lines; elements apart
  int n;              // basis functions
  int n_dm;
  const double* boys64;
  const float* boys32;
  float boys_fp64_T;  // FP32 kernels: F_m in FP64 above this T
  int att;            // host only: 1 selects the kernels of erf(omega r12)/r12
  double omega2;      // omega^2 (read by those kernels)
  void* ws;           // multi-pass classes: per-wave workspace (see split_ws_bytes)
  int nwaves;         // multi-pass classes: wavefronts of the launch
  int lanes;          // lanes sharing one shell quartet in this launch (1 or the class maximum)
  int* next;          // persistent kernels: next unclaimed work item (zero before the launch)
  int num_cu;         // compute units of the device (grid of the persistent kernels)
  size_t det_lo;      // 0: J/K accumulate with FP64 atomics; else deterministic mode, the
                      // accumulators are int64 fixed-point pairs (see atomic_add)
  int dry;            // host only: 1 = check the launch (scratch guard) without launching
  int rows;           // light classes: 1 = the bra's exchange rows may be kept in LDS
                      // (atomic accumulation), if they fit
};

// Persistent kernels: each wavefront claims work items one at a time.
__device__ __forceinline__ int claim_item(int* next) {
  int item = 0;
  if ((threadIdx.x & (kWave - 1)) == 0) item = atomicAdd(next, 1);
  return __builtin_amdgcn_readfirstlane(item);
}

// Per-quartet array in a launch workspace.  The QPW quartets of a wavefront
// are interleaved (stride QPW), so the lanes that carry them touch consecutive
// addresses for the same element.
template <typename T, int S>
struct LaneArr {
  T* p;
  __device__ __forceinline__ T& operator[](int i) const { return p[static_cast<size_t>(i) * S]; }
};

// The same pointer, opaque to the optimiser: element addresses derived from it
// are formed where they are used instead of being hoisted out of the loop and
// held (or spilled) across it.
template <typename T>
__device__ __forceinline__ T* opaque(T* p) {
  asm volatile("" : "+v"(p));
  return p;
}

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

// 1/sqrt(x) for positive normal FP64 x: hardware estimate refined by two
// Newton steps y <- y (3/2 - x y^2 / 2) (quadratic convergence, last bit
// rounding only).
__device__ __forceinline__ double rsqrt_f64(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  y = y * (1.5 - h * y * y);
  y = y * (1.5 - h * y * y);
  return y;
}

__device__ __forceinline__ float rsqrt_f32(float x) {
  float y = __builtin_amdgcn_rsqf(x);
  y = y * (1.5f - 0.5f * x * y * y);
  return y;
}

// F_m(T), m = 0..L, FP64.  T < 64: seven-term Taylor expansion about the nearest
// table point (|dT| <= 0.025, truncation below 2e-15 relative) for F_L, e^{-T}
// from the table value times a Taylor series of e^{-dT}, then the stable
// downward recursion F_m = (2T F_{m+1} + e^{-T}) / (2m+1).  T >= 64: the
// asymptotic F_0 = sqrt(pi/(4T)) and upward recursion F_{m+1} = (2m+1)/(2T) F_m
// (the dropped e^{-T} terms are below 1e-15 relative there for m <= 10).
// Both forms are evaluated and selected per lane, so a wavefront with mixed T
// does not diverge.  The table row is fetched by a separate call from its
// evaluation.
struct BoysRow64 {
  double2 q0, q1, q2, q3;   // F_L(T_i) ... F_{L+6}(T_i), exp(-T_i)
  double x;                 // T_i - T
};

// rows: the table of order L (global memory, or a copy staged in LDS that
// covers T < tmax only).
__device__ __forceinline__ BoysRow64 boys64_fetch(double T, const double* __restrict__ rows,
                                                  double tmax) {
  const double Tt = T < tmax ? T : 0.0;
  const int i = static_cast<int>(Tt * kBoysInvStep + 0.5);
  const double2* r2 = reinterpret_cast<const double2*>(rows + i * kBoysRow);
  return BoysRow64{r2[0], r2[1], r2[2], r2[3], i * kBoysStep - Tt};
}

template <int L>
__device__ __forceinline__ void boys64_taylor(double Tt, const BoysRow64& row, double* F) {
  const double x = row.x;
  const double r[8] = {row.q0.x, row.q0.y, row.q1.x, row.q1.y,
                       row.q2.x, row.q2.y, row.q3.x, row.q3.y};
  // Horner steps with x/k, shared by the Taylor series of F_L and of e^{x}
  const double x2 = x * 0.5, x3 = x * (1.0 / 3.0), x4 = x * 0.25, x5 = x * 0.2,
               x6 = x * (1.0 / 6.0);
  double s = r[6];
  s = r[5] + x6 * s;
  s = r[4] + x5 * s;
  s = r[3] + x4 * s;
  s = r[2] + x3 * s;
  s = r[1] + x2 * s;
  s = r[0] + x * s;
  F[L] = s;
  if constexpr (L > 0) {
    double e = 1.0 + x6;
    e = 1.0 + x5 * e;
    e = 1.0 + x4 * e;
    e = 1.0 + x3 * e;
    e = 1.0 + x2 * e;
    e = 1.0 + x * e;
    e *= r[7];
    const double T2 = 2.0 * Tt;
#pragma unroll
    for (int m = L - 1; m >= 0; --m) F[m] = (T2 * F[m + 1] + e) * kInvOdd[m];
  }
}

template <int L>
__device__ __forceinline__ void boys64_asym(double T, double* F) {
  const double rs = rsqrt_f64(T);
  double fa = 0.88622692545275801364908374167057 * rs;  // sqrt(pi)/2 / sqrt(T)
  const double h = 0.5 * rs * rs;
  F[0] = fa;
#pragma unroll
  for (int m = 0; m < L; ++m) {
    fa *= (2 * m + 1) * h;
    F[m + 1] = fa;
  }
}

// The kets of a wavefront are neighbours in a Q-sorted list, so their T are
// mostly all below or all above tmax: each form is evaluated only if some lane
// of the wavefront needs it.
template <int L>
__device__ __forceinline__ void boys64_eval(double T, const BoysRow64& row, double tmax, double* F) {
  static_assert(L <= kBoysMaxL, "Boys table order");
  const bool near = T < tmax;
  if (__all(near)) {
    boys64_taylor<L>(T, row, F);
  } else if (__all(!near)) {
    boys64_asym<L>(T, F);
  } else {
    double Ft[L + 1], Fa[L + 1];
    boys64_taylor<L>(near ? T : 0.0, row, Ft);
    boys64_asym<L>(near ? tmax : T, Fa);
#pragma unroll
    for (int m = 0; m <= L; ++m) F[m] = near ? Ft[m] : Fa[m];
  }
}

// F_m(T), m = 0..L, for the FP32 kernels.  T <= boys_fp64_T (<= 30): four-term
// Taylor expansion in FP32 from the FP32 table and downward recursion in FP32.
// T > 30: in FP64, the asymptotic F_0 = sqrt(pi/(4T)) (relative error
// erfc(sqrt T) < 2e-14) and upward recursion F_{m+1} = ((2m+1) F_m - e^{-T})/(2T),
// rounded to FP32.  e^{-T} itself enters only through that recursion, where at
// T > 30 it changes F_m by less than 4e-6 of its value for every m <= 9, so
// the FP32 exponential (relative error ~1e-7) leaves the result exact to FP32
// rounding; the reciprocal square root takes one Newton step from the hardware
// estimate (~1e-12 relative, below what the FP32 result keeps).
// boys_fp64_T < T <= 30 (only when the switch-over is set below 30): the FP64
// table evaluation above, exact to FP64 rounding at any T.
struct BoysRow32 {
  float4 q0;    // F_L(T_i) ... F_{L+3}(T_i)
  float e;      // exp(-T_i)
  float x;      // T_i - T
};

constexpr float kBoys32Asym = 30.0f;   // FP64 asymptotic form above this T

// rows: FP32 table of order L.
template <int L>
__device__ __forceinline__ BoysRow32 boys32_fetch(float T, float tcut, const float* __restrict__ rows) {
  BoysRow32 r;
  const float Tl = T <= tcut ? T : 0.0f;
  const int i = static_cast<int>(Tl * kBoys32InvStep + 0.5f);
  const float4* r4 = reinterpret_cast<const float4*>(rows + i * kBoys32Row);
  r.q0 = r4[0];
  r.e = r4[1].x;
  r.x = i * kBoys32Step - Tl;
  return r;
}

// rows64: FP64 table of order L (global), read only for boys_fp64_T < T <= 30.
template <int L>
__device__ __forceinline__ void boys32_eval(float T, float tcut, const BoysRow32& row,
                                            const double* __restrict__ rows64, float* F) {
  if (T <= tcut) {
    const float x = row.x;
    float s = row.q0.w;
    s = row.q0.z + x * s * (1.0f / 3.0f);
    s = row.q0.y + x * s * 0.5f;
    s = row.q0.x + x * s;
    F[L] = s;
    if constexpr (L > 0) {
      float e = 1.0f + x * 0.25f;
      e = 1.0f + x * (1.0f / 3.0f) * e;
      e = 1.0f + x * 0.5f * e;
      e = 1.0f + x * e;
      e *= row.e;
      const float T2 = 2.0f * T;
#pragma unroll
      for (int m = L - 1; m >= 0; --m) F[m] = (T2 * F[m + 1] + e) * static_cast<float>(kInvOdd[m]);
    }
  } else if (T > kBoys32Asym) {
    const double Td = static_cast<double>(T);
    double rs = __builtin_amdgcn_rsq(Td);
    rs = rs * (1.5 - 0.5 * Td * rs * rs);
    double f = 0.88622692545275801364908374167057 * rs;
    F[0] = static_cast<float>(f);
    if constexpr (L > 0) {
      const double e = static_cast<double>(__expf(-T));
      const double h = 0.5 * rs * rs;
#pragma unroll
      for (int m = 0; m < L; ++m) {
        f = ((2 * m + 1) * f - e) * h;
        F[m + 1] = static_cast<float>(f);
      }
    }
  } else {
    const double Td = static_cast<double>(T);
    const BoysRow64 r64 = boys64_fetch(Td, rows64, kBoysTmax);
    double F64[L + 1];
    boys64_eval<L>(Td, r64, kBoysTmax, F64);
#pragma unroll
    for (int m = 0; m <= L; ++m) F[m] = static_cast<float>(F64[m]);
  }
}

// Where a kernel reads the Boys rows of its order L from.  ATT: the kernel
// computes the integrals of erf(omega r12)/r12 (see prim_geo), om2 = omega^2.
template <typename T, bool ATT = false>
struct BoysTab;
template <bool ATT>
struct BoysTab<double, ATT> {
  const double* rows;   // order-L FP64 rows
  double tmax;          // tabulated range T < tmax; asymptotic form beyond
  double om2;
};
template <bool ATT>
struct BoysTab<float, ATT> {
  const float* rows;     // order-L FP32 rows (T <= tcut)
  float tcut;            // FP64 evaluation above
  const double* rows64;  // order-L FP64 rows, for e^{-T} above tcut
  float om2;
};

// The tables in global memory.
template <int L, typename T, bool ATT = false>
__device__ __forceinline__ BoysTab<T, ATT> global_boys(const EriLaunch& a) {
  static_assert(L <= kBoysMaxL, "Boys table order");
  const double* r64 = a.boys64 + static_cast<size_t>(L) * kBoysRows * kBoysRow;
  if constexpr (sizeof(T) == 8) {
    return BoysTab<double, ATT>{r64, kBoysTmax, a.omega2};
  } else {
    return BoysTab<float, ATT>{a.boys32 + static_cast<size_t>(L) * kBoys32Rows * kBoys32Row,
                               a.boys_fp64_T, r64, static_cast<float>(a.omega2)};
  }
}

template <int L, typename T>
struct Boys;
template <int L>
struct Boys<L, double> {
  using Row = BoysRow64;
  template <bool A>
  __device__ __forceinline__ static Row fetch(double T, const BoysTab<double, A>& t) {
    return boys64_fetch(T, t.rows, t.tmax);
  }
  template <bool A>
  __device__ __forceinline__ static void eval(double T, const Row& r, const BoysTab<double, A>& t,
                                              double* F) {
    boys64_eval<L>(T, r, t.tmax, F);
  }
};
template <int L>
struct Boys<L, float> {
  using Row = BoysRow32;
  template <bool A>
  __device__ __forceinline__ static Row fetch(float T, const BoysTab<float, A>& t) {
    return boys32_fetch<L>(T, t.tcut, t.rows);
  }
  template <bool A>
  __device__ __forceinline__ static void eval(float T, const Row& r, const BoysTab<float, A>& t,
                                              float* F) {
    boys32_eval<L>(T, t.tcut, r, t.rows64, F);
  }
};

template <typename T>
__device__ __forceinline__ T rsqrt_t(T x) {
  if constexpr (sizeof(T) == 8) return rsqrt_f64(x);
  else return rsqrt_f32(x);
}

// One primitive quartet in two steps.  prim_geo: Gaussian-product geometry,
// the Boys argument and the fetch of its table row; prim_finish: Boys values
// scaled by the prefactor and the recurrence coefficients.
//   P - Q = (P - A) - (Q - C) + (A - C)   (keeps FP32 differences small)
//   W - P = -q/(p+q) (P - Q),  W - Q = p/(p+q) (P - Q),  rho = pq/(p+q)
//   prefactor = 2 pi^{5/2} K_AB K_CD / (p q sqrt(p+q)) = Kt_AB Kt_CD / sqrt(p+q)
// The erf(omega r12)/r12 operator (ATT) depends on the geometry through T alone,
// like 1/r12, with F_m(T) replaced by sqrt(s) s^m F_m(s T), s = omega^2 /
// (omega^2 + rho): the recurrences are unchanged.  ATT is a compile-time flag, so
// the 1/r12 kernels carry none of it.
template <int L, typename T>
struct PrimGeo {
  T srpq, PQx, PQy, PQz, Tb;
  typename Boys<L, T>::Row row;
};

template <int L, typename T, bool ATT>
__device__ __forceinline__ void prim_geo(T p, T PAx, T PAy, T PAz, T q, T QCx, T QCy, T QCz,
                                         T ACx, T ACy, T ACz, const BoysTab<T, ATT>& bt,
                                         PrimGeo<L, T>& g) {
  g.srpq = rsqrt_t<T>(p + q);   // 1/sqrt(p+q)
  const T rpq = g.srpq * g.srpq;
  g.PQx = PAx - QCx + ACx;
  g.PQy = PAy - QCy + ACy;
  g.PQz = PAz - QCz + ACz;
  g.Tb = p * (q * rpq) * (g.PQx * g.PQx + g.PQy * g.PQy + g.PQz * g.PQz);
  if constexpr (ATT) g.Tb *= bt.om2 / (bt.om2 + p * (q * rpq));
  g.row = Boys<L, T>::fetch(g.Tb, bt);
}

template <int L, typename T, bool ATT>
__device__ __forceinline__ void prim_finish(const PrimGeo<L, T>& g, T p, T oo2p, T PAx, T PAy,
                                            T PAz, T Kab, T q, T oo2q, T QCx, T QCy, T QCz,
                                            T Kcd, const BoysTab<T, ATT>& bt, T* F,
                                            VrrCoef<T>& c) {
  const T rpq = g.srpq * g.srpq;
  const T qr = q * rpq, pr = p * rpq;
  Boys<L, T>::eval(g.Tb, g.row, bt, F);
  const T pref = Kab * Kcd * g.srpq;
  if constexpr (ATT) {
    const T sa = bt.om2 / (bt.om2 + p * qr);
    T f = pref * sqrt(sa);
#pragma unroll
    for (int m = 0; m <= L; ++m) {
      F[m] *= f;
      f *= sa;
    }
  } else {
#pragma unroll
    for (int m = 0; m <= L; ++m) F[m] *= pref;
  }
  c.PAx = PAx; c.PAy = PAy; c.PAz = PAz;
  c.QCx = QCx; c.QCy = QCy; c.QCz = QCz;
  c.WPx = -qr * g.PQx; c.WPy = -qr * g.PQy; c.WPz = -qr * g.PQz;
  c.WQx = pr * g.PQx; c.WQy = pr * g.PQy; c.WQz = pr * g.PQz;
  c.oo2p = oo2p; c.oo2p_rp = oo2p * qr;
  c.oo2q = oo2q; c.oo2q_rq = oo2q * pr;
  c.oo2pq = T(0.5) * rpq;
}

template <int L, typename T>
__device__ __forceinline__ void prim_setup(T p, T oo2p, T PAx, T PAy, T PAz, T Kab, T q, T oo2q,
                                           T QCx, T QCy, T QCz, T Kcd, T ACx, T ACy, T ACz,
                                           const EriLaunch& a, T* F, VrrCoef<T>& c) {
  const BoysTab<T> bt = global_boys<L, T>(a);   // 1/r12 only
  PrimGeo<L, T> g;
  prim_geo<L, T>(p, PAx, PAy, PAz, q, QCx, QCy, QCz, ACx, ACy, ACz, bt, g);
  prim_finish<L, T>(g, p, oo2p, PAx, PAy, PAz, Kab, q, oo2q, QCx, QCy, QCz, Kcd, bt, F, c);
}

// Read-only global data that the kernels never write: the constant address
// space lets the compiler use scalar loads where the address is uniform.
using CDouble = const __attribute__((address_space(4))) double*;
template <typename T>
using CReal = const __attribute__((address_space(4))) T*;

// Primitive-pair fields in the kernel's precision (FP32 kernels read the FP32
// copy: half the bytes and no conversions).
template <typename T>
__device__ __forceinline__ const T* prim_of(const BinView& v) {
  if constexpr (sizeof(T) == 8) return v.prim;
  else return v.prim32;
}
template <typename T>
__device__ __forceinline__ const T* primT_of(const BinView& v) {
  if constexpr (sizeof(T) == 8) return v.primT;
  else return v.primT32;
}

// Contraction loop of one shell quartet: bra pair i, ket pair k.  `vrr(F, c)`
// adds one primitive quartet to the caller's accumulators.
//
// G == 1: the bra pair is uniform across the wavefront; its primitive pairs
// come from the pair-major copy through scalar loads, the ket primitive pair
// of the lane is loaded once per ket primitive.
//
// G > 1: the G lanes of a group share the quartet; lane `sub` takes the
// primitive quartets sub, sub+G, ... as (kl, ij) with ij running fastest; the
// group's accumulators are summed by the caller.
template <int L, typename T, int G, bool ATT, class V>
__device__ __forceinline__ void contract(const EriLaunch& a, const BoysTab<T, ATT>& bt, int i, int k,
                                         int sub, T ACx, T ACy, T ACz, V&& vrr) {
  const int nk = a.ket.n;
  const int nppb = a.bra.npp, nppk = a.ket.npp;
  const T* kprim = prim_of<T>(a.ket);
  if constexpr (G == 1) {
    (void)sub;
    const CReal<T> bra = (CReal<T>)(primT_of<T>(a.bra)) + static_cast<size_t>(i) * nppb * kPrimFields;
    for (int kl = 0; kl < nppk; ++kl) {
      const T* kp = kprim + static_cast<size_t>(kl) * kPrimFields * nk + k;
      const T q = kp[kP * nk], oo2q = kp[kOo2p * nk];
      const T QCx = kp[kPAx * nk], QCy = kp[kPAy * nk], QCz = kp[kPAz * nk];
      const T Kcd = kp[kKt * nk];
      auto geo = [&](int ij, PrimGeo<L, T>& g) {
        const CReal<T> b = bra + ij * kPrimFields;
        prim_geo<L, T>(b[kP], b[kPAx], b[kPAy], b[kPAz], q, QCx, QCy, QCz, ACx, ACy, ACz, bt, g);
      };
      auto finish = [&](int ij, const PrimGeo<L, T>& g) {
        const CReal<T> b = bra + ij * kPrimFields;
        T F[L + 1];
        VrrCoef<T> c;
        prim_finish<L, T>(g, b[kP], b[kOo2p], b[kPAx], b[kPAy], b[kPAz], b[kKt], q, oo2q, QCx,
                          QCy, QCz, Kcd, bt, F, c);
        vrr(F, c);
      };
      for (int ij = 0; ij < nppb; ++ij) {
        PrimGeo<L, T> g;
        geo(ij, g);
        finish(ij, g);
      }
    }
  } else {
    const T* bra = primT_of<T>(a.bra) + static_cast<size_t>(i) * nppb * kPrimFields;
    const int npq = nppb * nppk;
    auto geo = [&](int kl, int ij, PrimGeo<L, T>& g) {
      const T* b = bra + ij * kPrimFields;
      const T* kp = kprim + static_cast<size_t>(kl) * kPrimFields * nk + k;
      prim_geo<L, T>(b[kP], b[kPAx], b[kPAy], b[kPAz], kp[kP * nk], kp[kPAx * nk], kp[kPAy * nk],
                     kp[kPAz * nk], ACx, ACy, ACz, bt, g);
    };
    auto finish = [&](int kl, int ij, const PrimGeo<L, T>& g) {
      const T* b = bra + ij * kPrimFields;
      const T* kp = kprim + static_cast<size_t>(kl) * kPrimFields * nk + k;
      T F[L + 1];
      VrrCoef<T> c;
      prim_finish<L, T>(g, b[kP], b[kOo2p], b[kPAx], b[kPAy], b[kPAz], b[kKt], kp[kP * nk],
                        kp[kOo2p * nk], kp[kPAx * nk], kp[kPAy * nk], kp[kPAz * nk],
                        kp[kKt * nk], bt, F, c);
      vrr(F, c);
    };
    auto step = [&](int& kl, int& ij) {
      ij += G;
      while (ij >= nppb) { ij -= nppb; ++kl; }
    };
    int kl0 = 0, ij0 = sub;
    while (ij0 >= nppb) { ij0 -= nppb; ++kl0; }
    for (int t = sub; t < npq; t += G) {
      PrimGeo<L, T> g;
      geo(kl0, ij0, g);
      finish(kl0, ij0, g);
      step(kl0, ij0);
    }
  }
}

// Cross-lane moves of an FP64 value within rows of 16 lanes (DPP on the two
// 32-bit halves; no LDS traffic).
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ double dpp_f64(double v, double old) {
  const long long b = __builtin_bit_cast(long long, v);
  const long long o = __builtin_bit_cast(long long, old);
  const int lo = __builtin_amdgcn_update_dpp(static_cast<int>(o), static_cast<int>(b), CTRL,
                                             ROW_MASK, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(static_cast<int>(o >> 32), static_cast<int>(b >> 32),
                                             CTRL, ROW_MASK, 0xF, false);
  return __builtin_bit_cast(double, (static_cast<long long>(hi) << 32) |
                                        static_cast<unsigned long long>(static_cast<unsigned>(lo)));
}

template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ float dpp_f32(float v, float old) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, old), __builtin_bit_cast(int, v),
                                         CTRL, ROW_MASK, 0xF, false));
}

template <int CTRL, typename T>
__device__ __forceinline__ T dpp_t(T v) {
  if constexpr (sizeof(T) == 8) return dpp_f64<CTRL>(v, v);
  else return dpp_f32<CTRL>(v, v);
}

// Sum over the G lanes of a group (G = 1, 2, 4, 8 or 16 consecutive lanes);
// every lane of the group ends with the sum.  Steps: swap neighbours, swap
// pairs within a quad, mirror within half-rows, mirror within rows.
template <int G, typename T>
__device__ __forceinline__ T group_sum(T v) {
  static_assert(G == 1 || G == 2 || G == 4 || G == 8 || G == 16 || G == 64, "group size");
  if constexpr (G >= 2) v += dpp_t<0xB1>(v);    // quad_perm [1,0,3,2]
  if constexpr (G >= 4) v += dpp_t<0x4E>(v);    // quad_perm [2,3,0,1]
  if constexpr (G >= 8) v += dpp_t<0x141>(v);   // row_half_mirror
  if constexpr (G >= 16) v += dpp_t<0x140>(v);  // row_mirror
  if constexpr (G == 64) {
    // rows 0..3: row 0 into row 1, rows 0-1 into rows 2-3, then lane 63 to all
    if constexpr (sizeof(T) == 8) {
      v += dpp_f64<0x142, 0xA>(v, 0.0);
      v += dpp_f64<0x143, 0xC>(v, 0.0);
      const long long b = __builtin_bit_cast(long long, v);
      const int lo = __builtin_amdgcn_readlane(static_cast<int>(b), 63);
      const int hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), 63);
      v = __builtin_bit_cast(T, (static_cast<long long>(hi) << 32) |
                                    static_cast<unsigned long long>(static_cast<unsigned>(lo)));
    } else {
      v += dpp_f32<0x142, 0xA>(v, 0.0f);
      v += dpp_f32<0x143, 0xC>(v, 0.0f);
      v = __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
    }
  }
  return v;
}

template <int G, typename T, int N>
__device__ __forceinline__ void group_sum_all(T (&acc)[N]) {
  if constexpr (G > 1) {
#pragma unroll
    for (int t = 0; t < N; ++t) acc[t] = group_sum<G>(acc[t]);
  }
}

// Sum over the wavefront; the result is complete in lane kWaveSumLane only.
// Row sums by DPP, then row 0 is added into row 1 and rows 0-1 into rows 2-3
// (row broadcasts of lanes 15 and 31).
constexpr int kWaveSumLane = kWave - 1;
__device__ __forceinline__ double wave_sum(double v) {
  v = group_sum<16>(v);
  v += dpp_f64<0x142, 0xA>(v, 0.0);   // row_bcast:15 into rows 1 and 3
  v += dpp_f64<0x143, 0xC>(v, 0.0);   // row_bcast:31 into rows 2 and 3
  return v;
}

// Accumulation into J, K (and dE/dR).  lo_off == 0: one FP64 atomic add, whose
// rounding depends on the order in which the adds arrive.  lo_off > 0
// (deterministic mode): the accumulator at addr is a pair of two's-complement
// int64 words, hi at addr and lo at addr + lo_off elements, standing for
// hi 2^-32 + lo 2^-62; v is split into those two words and both are added with
// integer atomics, whose sums do not depend on the order (|v| and every
// accumulated value below 2^31; per add the lo word loses at most 2^-63).
constexpr double kFixHi = 4294967296.0;            // 2^32
constexpr double kFixLo = 1073741824.0;            // 2^30: lo word = 2^62 x the remainder
__device__ __forceinline__ void atomic_add(double* addr, double v, size_t lo_off) {
  if (lo_off == 0) {
    unsafeAtomicAdd(addr, v);
    return;
  }
  const double s = v * kFixHi;
  const double h = rint(s);
  const long long hi = static_cast<long long>(h);
  const long long lo = static_cast<long long>(rint((s - h) * kFixLo));
  unsigned long long* w = reinterpret_cast<unsigned long long*>(addr);
  if (hi != 0) atomicAdd(w, static_cast<unsigned long long>(hi));
  if (lo != 0) atomicAdd(w + lo_off, static_cast<unsigned long long>(lo));
}

// Scatter of per-quartet integral blocks into J or K with few memory-side
// atomic requests.  FP64 atomic adds are executed past the L2, one request per
// 64-byte line and wavefront instruction, whatever the number of lanes that hit
// the line.  A block of NX x NY values per quartet (row-major, rows rx + x,
// columns cy + y of an n x n matrix) is therefore staged in LDS and re-read so
// that groups of P lanes add the S contiguous elements of one row segment
// together.  When NX > NY the block goes in transposed (rows cy + y, columns
// rx + x): the build returns M + M^T, so either orientation gives the same
// result.  Q quartets per wavefront; `writer` marks the lane that holds a
// quartet's block (the first lane of its group), slot = lane / (64 / Q).
template <int NX, int NY, int Q>
struct Scatter {
  static constexpr bool TR = NX > NY;
  static constexpr int S = TR ? NX : NY;   // contiguous segment
  static constexpr int R = TR ? NY : NX;   // segments per quartet
  static constexpr int P = S <= 1 ? 1 : S <= 2 ? 2 : S <= 4 ? 4 : 8;
  static constexpr int GW = kWave / P;     // segments per round
  static constexpr int STAGE = S > 1 ? Q * (S + 1) : 0;   // doubles of LDS per wavefront
};

template <int NX, int NY, int Q>
__device__ __forceinline__ void scatter_block(double* M, size_t n, int rx, int cy,
                                              const double* blk, bool writer, double* stage,
                                              size_t det_lo) {
  using Sc = Scatter<NX, NY, Q>;
  if constexpr (Sc::S == 1) {
    if (writer && blk[0] != 0.0) atomic_add(&M[static_cast<size_t>(rx) * n + cy], blk[0], det_lo);
  } else {
    constexpr int S = Sc::S, R = Sc::R, P = Sc::P, GW = Sc::GW;
    const int lane = threadIdx.x & (kWave - 1);
    const int slot = lane / (kWave / Q);
    const int g = lane / P, e = lane % P;
    double* vals = stage;             // [Q][S] one segment per quartet
    double* base = stage + Q * S;     // [Q] its first element, as a bit pattern
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (writer) {
        const long long b = Sc::TR ? static_cast<long long>(cy + r) * static_cast<long long>(n) + rx
                                   : static_cast<long long>(rx + r) * static_cast<long long>(n) + cy;
        base[slot] = __builtin_bit_cast(double, b);
#pragma unroll
        for (int x = 0; x < S; ++x) vals[slot * S + x] = Sc::TR ? blk[x * NY + r] : blk[r * NY + x];
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
      for (int q0 = 0; q0 < Q; q0 += GW) {
        const int q = q0 + g;
        if (e < S && q < Q) {
          const double v = vals[q * S + e];
          if (v != 0.0) atomic_add(&M[__builtin_bit_cast(long long, base[q]) + e], v, det_lo);
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
}

// LDS staging doubles per wavefront for the scatters of class C with Q quartets
// per wavefront.
template <class C, int Q>
constexpr int stage_doubles() {
  int m = Scatter<C::NC, C::ND, Q>::STAGE;
  m = m > Scatter<C::NA, C::NC, Q>::STAGE ? m : Scatter<C::NA, C::NC, Q>::STAGE;
  m = m > Scatter<C::NA, C::ND, Q>::STAGE ? m : Scatter<C::NA, C::ND, Q>::STAGE;
  m = m > Scatter<C::NB, C::NC, Q>::STAGE ? m : Scatter<C::NB, C::NC, Q>::STAGE;
  m = m > Scatter<C::NB, C::ND, Q>::STAGE ? m : Scatter<C::NB, C::ND, Q>::STAGE;
  return m > 0 ? m : 1;
}

// Bytes of workspace per wavefront of a multi-pass class with G lanes per
// quartet: contracted [e0|f0] and ket-transformed values (type T) and the J_cd
// block per quartet slot, the K partial blocks per lane.  The host sizes the
// workspace with the same expression (generated table).
template <class C, typename T>
__host__ __device__ constexpr size_t split_wave_bytes(int G) {
  constexpr int NCD = C::NC * C::ND;
  constexpr int NT = C::NACC + C::NE * NCD;
  constexpr int NK = C::NA * C::NC + C::NA * C::ND + C::NB * C::NC + C::NB * C::ND;
  return static_cast<size_t>(kWave / G) * (NT * sizeof(T) + NCD * sizeof(double)) +
         static_cast<size_t>(kWave) * NK * sizeof(double);
}

// Workspace written by other lanes of the wavefront becomes visible to all.
__device__ __forceinline__ void lanes_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// The same scatter for blocks parked in a wavefront workspace.  PARTS == 1:
// element t of quartet slot q at w0[t * Q + q]; PARTS == 64 / Q: each lane
// holds a partial block, element t of lane L at w0[t * 64 + L], and a slot's
// value is the sum over its PARTS lanes.  rx and cy are read from the slot's
// first lane; all lanes take part.
template <int NX, int NY, int Q, int PARTS>
__device__ __forceinline__ void scatter_ws(double* M, size_t n, int rx, int cy, const double* w0,
                                           size_t det_lo) {
  using Sc = Scatter<NX, NY, Q>;
  constexpr int S = Sc::S, R = Sc::R, P = Sc::P, GW = Sc::GW;
  constexpr int G = kWave / Q;
  static_assert(PARTS == 1 || PARTS == G, "partial blocks: one per lane of the slot");
  constexpr int STRIDE = PARTS == 1 ? Q : kWave;
  const int lane = threadIdx.x & (kWave - 1);
  const int g = lane / P, e = lane % P;
  lanes_sync();   // the blocks were stored by other lanes of this wavefront
#pragma nounroll
  for (int q0 = 0; q0 < Q; q0 += GW) {
    const int q = q0 + g < Q ? q0 + g : Q - 1;
    const int src = q * G;
    const int rxq = __shfl(rx, src, kWave), cyq = __shfl(cy, src, kWave);
    if (e < S && q0 + g < Q) {
#pragma nounroll
      for (int r = 0; r < R; ++r) {
        const int t = Sc::TR ? e * NY + r : r * NY + e;
        double v = 0.0;
#pragma unroll
        for (int u = 0; u < PARTS; ++u) v += w0[t * STRIDE + (PARTS == 1 ? q : q * G + u)];
        const size_t at = Sc::TR ? static_cast<size_t>(cyq + r) * n + rxq + e
                                 : static_cast<size_t>(rxq + r) * n + cyq + e;
        if (v != 0.0) atomic_add(&M[at], v, det_lo);
      }
    }
  }
  lanes_sync();   // the workspace is rewritten for the next quartets
}

// D block rows r0.., columns c0.. (NR x NCOL) into registers.
template <int NR, int NCOL>
__device__ __forceinline__ void load_block(double* dst, const double* Dm, size_t n, int r0, int c0) {
#pragma unroll
  for (int x = 0; x < NR; ++x)
#pragma unroll
    for (int y = 0; y < NCOL; ++y) dst[x * NCOL + y] = Dm[(r0 + x) * n + c0 + y];
}

// Integral + digestion of one work item {bra pair, ket range} of one class and
// precision by one wavefront: the bra pair is uniform across the wave (scalar
// data), each lane (each group of G lanes) takes one ket pair of the current
// chunk of the item's ket range.
template <class C, typename T, int G, bool ATT>
__device__ __forceinline__ void eri_item(const EriLaunch& a, const BoysTab<T, ATT>& bt, int item,
                                         double* stage) {
  constexpr int QPW = kWave / G;
  const int lane = threadIdx.x & (kWave - 1);
  const int sub = lane & (G - 1), ql = lane / G;
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

  for (int kc = kbeg; kc < kend; kc += QPW) {
    const bool inrange = kc + ql < kend;
    const bool active = inrange && sub == 0;   // one lane of the group digests
    const int k = inrange ? kc + ql : kend - 1;
    const T ACx = T(Ax - a.ket.A[k]), ACy = T(Ay - a.ket.A[nk + k]),
            ACz = T(Az - a.ket.A[2 * nk + k]);
    T acc[C::NACC];
#pragma unroll
    for (int t = 0; t < C::NACC; ++t) acc[t] = T(0);
    contract<C::L, T, G>(a, bt, i, k, sub, ACx, ACy, ACz,
                         [&](const T* F, const VrrCoef<T>& c) { C::template vrr<T>(F, c, acc); });
    group_sum_all<G>(acc);

    const T CDx = T(a.ket.AB[k]), CDy = T(a.ket.AB[nk + k]), CDz = T(a.ket.AB[2 * nk + k]);
    const int c0 = a.ket.bf[k], d0 = a.ket.bf[nk + k];
    const double fq =
        active ? fbra * a.ket.fpair[k] * ((a.same_bin && k == i) ? 0.5 : 1.0) : 0.0;

    for (int m = 0; m < a.n_dm; ++m) {
      const double* Dm = a.D + m * nn;
      if constexpr (C::SWEEPS) {
        // five sweeps, each with one D block and one accumulator block live
        const size_t n = static_cast<size_t>(a.n);
        double* Jm = a.J + (item % a.ncopy) * a.copy_stride + m * nn;
        double* Km = a.K + (item % a.ncopy) * a.copy_stride + m * nn;
        const bool writer = sub == 0;
        {
          double Dab[C::NA * C::NB], Dcd[C::NC * C::ND], jab[C::NA * C::NB], jcd[C::NC * C::ND];
          load_block<C::NA, C::NB>(Dab, Dm, n, a0, b0);
          load_block<C::NC, C::ND>(Dcd, Dm, n, c0, d0);
#pragma unroll
          for (int t = 0; t < C::NA * C::NB; ++t) jab[t] = 0.0;
#pragma unroll
          for (int t = 0; t < C::NC * C::ND; ++t) jcd[t] = 0.0;
          C::template digest_j<T>(acc, ABx, ABy, ABz, CDx, CDy, CDz, fq, Dab, Dcd, jab, jcd);
#pragma unroll
          for (int t = 0; t < C::NA * C::NB; ++t) {
            const double sj = wave_sum(jab[t]);
            if (lane == kWaveSumLane)
              atomic_add(&Jm[(a0 + t / C::NB) * n + b0 + t % C::NB], 2.0 * sj, a.det_lo);
          }
#pragma unroll
          for (int t = 0; t < C::NC * C::ND; ++t) jcd[t] *= 2.0;
          scatter_block<C::NC, C::ND, QPW>(Jm, n, c0, d0, jcd, writer, stage, a.det_lo);
        }
        {
          double Dx[C::NB * C::ND], kx[C::NA * C::NC];
          load_block<C::NB, C::ND>(Dx, Dm, n, b0, d0);
#pragma unroll
          for (int t = 0; t < C::NA * C::NC; ++t) kx[t] = 0.0;
          C::template digest_kac<T>(acc, ABx, ABy, ABz, CDx, CDy, CDz, fq, Dx, kx);
          scatter_block<C::NA, C::NC, QPW>(Km, n, a0, c0, kx, writer, stage, a.det_lo);
        }
        {
          double Dx[C::NB * C::NC], kx[C::NA * C::ND];
          load_block<C::NB, C::NC>(Dx, Dm, n, b0, c0);
#pragma unroll
          for (int t = 0; t < C::NA * C::ND; ++t) kx[t] = 0.0;
          C::template digest_kad<T>(acc, ABx, ABy, ABz, CDx, CDy, CDz, fq, Dx, kx);
          scatter_block<C::NA, C::ND, QPW>(Km, n, a0, d0, kx, writer, stage, a.det_lo);
        }
        {
          double Dx[C::NA * C::ND], kx[C::NB * C::NC];
          load_block<C::NA, C::ND>(Dx, Dm, n, a0, d0);
#pragma unroll
          for (int t = 0; t < C::NB * C::NC; ++t) kx[t] = 0.0;
          C::template digest_kbc<T>(acc, ABx, ABy, ABz, CDx, CDy, CDz, fq, Dx, kx);
          scatter_block<C::NB, C::NC, QPW>(Km, n, b0, c0, kx, writer, stage, a.det_lo);
        }
        {
          double Dx[C::NA * C::NC], kx[C::NB * C::ND];
          load_block<C::NA, C::NC>(Dx, Dm, n, a0, c0);
#pragma unroll
          for (int t = 0; t < C::NB * C::ND; ++t) kx[t] = 0.0;
          C::template digest_kbd<T>(acc, ABx, ABy, ABz, CDx, CDy, CDz, fq, Dx, kx);
          scatter_block<C::NB, C::ND, QPW>(Km, n, b0, d0, kx, writer, stage, a.det_lo);
        }
        continue;
      }
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

      double* Jm = a.J + (item % a.ncopy) * a.copy_stride + m * nn;
      double* Km = a.K + (item % a.ncopy) * a.copy_stride + m * nn;
#pragma unroll
      for (int t = 0; t < C::NA * C::NB; ++t) {
        const double s = wave_sum(jab[t]);
        if (lane == kWaveSumLane)
          atomic_add(&Jm[(a0 + t / C::NB) * static_cast<size_t>(a.n) + b0 + t % C::NB], 2.0 * s,
                     a.det_lo);
      }
#pragma unroll
      for (int t = 0; t < C::NC * C::ND; ++t) jcd[t] *= 2.0;
      const size_t n = static_cast<size_t>(a.n);
      // every quartet slot is written (out-of-range ones hold zeros, fq = 0)
      const bool writer = sub == 0;
      scatter_block<C::NC, C::ND, QPW>(Jm, n, c0, d0, jcd, writer, stage, a.det_lo);
      scatter_block<C::NA, C::NC, QPW>(Km, n, a0, c0, kac, writer, stage, a.det_lo);
      scatter_block<C::NA, C::ND, QPW>(Km, n, a0, d0, kad, writer, stage, a.det_lo);
      scatter_block<C::NB, C::NC, QPW>(Km, n, b0, c0, kbc, writer, stage, a.det_lo);
      scatter_block<C::NB, C::ND, QPW>(Km, n, b0, d0, kbd, writer, stage, a.det_lo);
    }
  }
}

template <class C, typename T, int G, bool ATT = false>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(class_waves<C, T>())))
void eri_jk_kernel(const EriLaunch a) {
  constexpr int ST = stage_doubles<C, kWave / G>();
  __shared__ double stage[kWavesPerBlock * ST];
  const int item = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  if (item >= a.nitems) return;
  eri_item<C, T, G>(a, global_boys<C::L, T, ATT>(a), item, stage + (threadIdx.x >> 6) * ST);
}

// Light classes (L <= 3, one lane per quartet): the Boys-table gathers, one
// 64-byte row per primitive quartet and lane, would otherwise saturate the
// vector-memory path.  Each workgroup of NT threads stages the rows of its
// order in LDS once (FP64: T < 45, beyond which the asymptotic form is exact to
// 2e-16 relative for orders <= 3; FP32: the whole FP32 table) and its
// wavefronts then claim work items until none is left.  NT = 1024 where the
// class fits in 128 VGPRs, else 512 (256 VGPRs).
constexpr int kLdsMaxL = 3;
constexpr double kLdsTmax = 45.0;
constexpr int kLdsRows64 = 901;   // T_i = 0.05 i <= 45

template <class C, typename T, int NT, bool ATT = false>
__global__ __launch_bounds__(NT) void eri_jk_lds_kernel(const EriLaunch a) {
  static_assert(C::L <= kLdsMaxL, "LDS Boys table: orders <= 3");
  constexpr int W = NT / kWave;
  const BoysTab<T, ATT> g = global_boys<C::L, T, ATT>(a);
  BoysTab<T, ATT> bt = g;
  if constexpr (sizeof(T) == 8) {
    __shared__ double2 rows[kLdsRows64 * kBoysRow / 2];
    const double2* src = reinterpret_cast<const double2*>(g.rows);
    for (int t = threadIdx.x; t < kLdsRows64 * kBoysRow / 2; t += NT) rows[t] = src[t];
    bt.rows = reinterpret_cast<const double*>(rows);
    bt.tmax = kLdsTmax;
  } else {
    __shared__ float4 rows[kBoys32Rows * kBoys32Row / 4];
    const float4* src = reinterpret_cast<const float4*>(g.rows);
    for (int t = threadIdx.x; t < kBoys32Rows * kBoys32Row / 4; t += NT) rows[t] = src[t];
    bt.rows = reinterpret_cast<const float*>(rows);
  }
  constexpr int ST = stage_doubles<C, kWave>();
  __shared__ double stage[W * ST];
  __syncthreads();
  (void)W;
  for (int item = claim_item(a.next); item < a.nitems; item = claim_item(a.next))
    eri_item<C, T, 1>(a, bt, item, stage + (threadIdx.x >> 6) * ST);
}

// Light classes with the bra's exchange rows kept in LDS.  A work item's bra
// pair (a, b) is shared by every quartet of the item, so the exchange blocks
// K_ac, K_ad, K_bc, K_bd all fall into the rows a0.., b0.. of K (only K + K^T is
// returned, so K_ac may stand in row a, column c).  The workgroup keeps those
// NA + NB rows over all n columns in LDS, its wavefronts add every quartet's
// blocks there with LDS atomics, and the rows reach K with one dense flush per
// item -- about 0.5 memory-side atomic requests per quartet instead of one per
// block and quartet.  J_ab is summed over the wavefront into LDS the same way;
// J_cd still goes to J per quartet through the staged scatter.

// One 64-ket chunk of a work item, one lane per quartet (one density).
template <class C, typename T, bool ATT>
__device__ __forceinline__ void eri_chunk_rows(const EriLaunch& a, const BoysTab<T, ATT>& bt, int i,
                                               int kc, int kend, double* stage, double* krow,
                                               double* jrow, double* Jm) {
  const int lane = threadIdx.x & (kWave - 1);
  const int nb = a.bra.n, nk = a.ket.n;
  const size_t n = static_cast<size_t>(a.n);
  const double Ax = a.bra.A[i], Ay = a.bra.A[nb + i], Az = a.bra.A[2 * nb + i];
  const T ABx = T(a.bra.AB[i]), ABy = T(a.bra.AB[nb + i]), ABz = T(a.bra.AB[2 * nb + i]);
  const int a0 = a.bra.bf[i], b0 = a.bra.bf[nb + i];
  const double fbra = a.bra.fpair[i];
  const bool inrange = kc + lane < kend;
  const int k = inrange ? kc + lane : kend - 1;
  const T ACx = T(Ax - a.ket.A[k]), ACy = T(Ay - a.ket.A[nk + k]), ACz = T(Az - a.ket.A[2 * nk + k]);
  T acc[C::NACC];
#pragma unroll
  for (int t = 0; t < C::NACC; ++t) acc[t] = T(0);
  contract<C::L, T, 1>(a, bt, i, k, 0, ACx, ACy, ACz,
                       [&](const T* F, const VrrCoef<T>& c) { C::template vrr<T>(F, c, acc); });
  const T CDx = T(a.ket.AB[k]), CDy = T(a.ket.AB[nk + k]), CDz = T(a.ket.AB[2 * nk + k]);
  const int c0 = a.ket.bf[k], d0 = a.ket.bf[nk + k];
  const double fq = inrange ? fbra * a.ket.fpair[k] * ((a.same_bin && k == i) ? 0.5 : 1.0) : 0.0;
  const double* Dm = a.D;
  double Dab[C::NA * C::NB], Dcd[C::NC * C::ND], Dac[C::NA * C::NC], Dad[C::NA * C::ND],
      Dbc[C::NB * C::NC], Dbd[C::NB * C::ND];
  load_block<C::NA, C::NB>(Dab, Dm, n, a0, b0);
  load_block<C::NC, C::ND>(Dcd, Dm, n, c0, d0);
  load_block<C::NA, C::NC>(Dac, Dm, n, a0, c0);
  load_block<C::NA, C::ND>(Dad, Dm, n, a0, d0);
  load_block<C::NB, C::NC>(Dbc, Dm, n, b0, c0);
  load_block<C::NB, C::ND>(Dbd, Dm, n, b0, d0);
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
  C::template hrr_digest<T>(acc, ABx, ABy, ABz, CDx, CDy, CDz, fq, Dab, Dcd, Dac, Dad, Dbc, Dbd,
                            jab, jcd, kac, kad, kbc, kbd);
#pragma unroll
  for (int t = 0; t < C::NA * C::NB; ++t) {
    const double sj = wave_sum(jab[t]);
    if (lane == kWaveSumLane && sj != 0.0)
      __hip_atomic_fetch_add(&jrow[t], 2.0 * sj, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
#pragma unroll
  for (int t = 0; t < C::NC * C::ND; ++t) jcd[t] *= 2.0;
  scatter_block<C::NC, C::ND, kWave>(Jm, n, c0, d0, jcd, true, stage, 0);
  if (fq != 0.0) {
    auto add = [&](int row, int col, double v) {
      if (v != 0.0)
        __hip_atomic_fetch_add(&krow[static_cast<size_t>(row) * n + col], v, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
    };
#pragma unroll
    for (int x = 0; x < C::NA; ++x) {
#pragma unroll
      for (int y = 0; y < C::NC; ++y) add(x, c0 + y, kac[x * C::NC + y]);
#pragma unroll
      for (int y = 0; y < C::ND; ++y) add(x, d0 + y, kad[x * C::ND + y]);
    }
#pragma unroll
    for (int x = 0; x < C::NB; ++x) {
#pragma unroll
      for (int y = 0; y < C::NC; ++y) add(C::NA + x, c0 + y, kbc[x * C::NC + y]);
#pragma unroll
      for (int y = 0; y < C::ND; ++y) add(C::NA + x, d0 + y, kbd[x * C::ND + y]);
    }
  }
}

// Dynamic LDS of the rows kernel: NA + NB rows of n doubles, then NA * NB for J_ab.
template <class C>
__host__ __device__ constexpr size_t rows_lds_doubles(int n) {
  return static_cast<size_t>(C::NA + C::NB) * n + C::NA * C::NB;
}

template <class C, typename T, int NT, bool ATT = false>
__global__ __launch_bounds__(NT) void eri_jk_rows_kernel(const EriLaunch a) {
  static_assert(C::L <= kLdsMaxL, "LDS Boys table: orders <= 3");
  constexpr int W = NT / kWave;
  constexpr int NR = C::NA + C::NB;
  const BoysTab<T, ATT> g = global_boys<C::L, T, ATT>(a);
  BoysTab<T, ATT> bt = g;
  if constexpr (sizeof(T) == 8) {
    __shared__ double2 rows[kLdsRows64 * kBoysRow / 2];
    const double2* src = reinterpret_cast<const double2*>(g.rows);
    for (int t = threadIdx.x; t < kLdsRows64 * kBoysRow / 2; t += NT) rows[t] = src[t];
    bt.rows = reinterpret_cast<const double*>(rows);
    bt.tmax = kLdsTmax;
  } else {
    __shared__ float4 rows[kBoys32Rows * kBoys32Row / 4];
    const float4* src = reinterpret_cast<const float4*>(g.rows);
    for (int t = threadIdx.x; t < kBoys32Rows * kBoys32Row / 4; t += NT) rows[t] = src[t];
    bt.rows = reinterpret_cast<const float*>(rows);
  }
  constexpr int ST = Scatter<C::NC, C::ND, kWave>::STAGE > 0 ? Scatter<C::NC, C::ND, kWave>::STAGE : 1;
  __shared__ double stage[W * ST];
  __shared__ int s_item;
  extern __shared__ double dyn[];
  const int n = a.n;
  double* const krow = dyn;
  double* const jrow = dyn + static_cast<size_t>(NR) * n;
  const int tot = static_cast<int>(rows_lds_doubles<C>(n));
  for (int t = threadIdx.x; t < tot; t += NT) dyn[t] = 0.0;
  __syncthreads();
  const int wave = threadIdx.x >> 6;
  const int nb = a.bra.n;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(a.next, 1);
    __syncthreads();
    const int item = s_item;
    if (item >= a.nitems) break;   // uniform over the workgroup
    const int4 w4 = a.items[item];
    const int i = __builtin_amdgcn_readfirstlane(w4.x);
    const int kbeg = __builtin_amdgcn_readfirstlane(w4.y);
    const int kend = __builtin_amdgcn_readfirstlane(w4.z);
    double* Jm = a.J + (item % a.ncopy) * a.copy_stride;
    double* Km = a.K + (item % a.ncopy) * a.copy_stride;
    for (int kc = kbeg + wave * kWave; kc < kend; kc += W * kWave)
      eri_chunk_rows<C, T>(a, bt, i, kc, kend, stage + wave * ST, krow, jrow, Jm);
    __syncthreads();
    // flush: the bra's rows of K (and J_ab) to the accumulators, zero them again
    const int a0 = a.bra.bf[i], b0 = a.bra.bf[nb + i];
    const size_t ns = static_cast<size_t>(n);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const size_t fn = static_cast<size_t>(r < C::NA ? a0 + r : b0 + (r - C::NA));
      for (int col = threadIdx.x; col < n; col += NT) {
        const double v = krow[r * ns + col];
        if (v != 0.0) {
          atomic_add(&Km[fn * ns + col], v, 0);
          krow[r * ns + col] = 0.0;
        }
      }
    }
    for (int t = threadIdx.x; t < C::NA * C::NB; t += NT) {
      const double v = jrow[t];
      if (v != 0.0) {
        atomic_add(&Jm[(a0 + t / C::NB) * ns + b0 + t % C::NB], v, 0);
        jrow[t] = 0.0;
      }
    }
    __syncthreads();
  }
}

// Cauchy-Schwarz factor of every pair of a bin: Q = sqrt(max_ab (ab|ab)).
// One lane per pair; bra and ket are the same pair, so A - C = 0.
template <class C>
__global__ __launch_bounds__(kBlock) void schwarz_kernel(const EriLaunch a, double* Qout) {
  constexpr int G = C::GMAX;
  const int gt = blockIdx.x * kBlock + threadIdx.x;
  const int n = a.bra.n;
  if (gt / kWave * (kWave / G) >= n) return;   // whole wave past the end
  const int sub = gt & (G - 1);
  const int t0 = gt / G;
  const int t = t0 < n ? t0 : n - 1;
  double acc[C::NACC];
#pragma unroll
  for (int s = 0; s < C::NACC; ++s) acc[s] = 0.0;
  contract<C::L, double, G>(a, global_boys<C::L, double>(a), t, t, sub, 0.0, 0.0, 0.0,
                            [&](const double* F, const VrrCoef<double>& c) {
                              C::template vrr<double>(F, c, acc);
                            });
  group_sum_all<G>(acc);
  const double mx = C::template diag_max<double>(acc, a.bra.AB[t], a.bra.AB[n + t], a.bra.AB[2 * n + t]);
  if (t0 < n && sub == 0) Qout[t] = sqrt(fmax(mx, 0.0));
}

// ---------------------------------------------------------------------------------
// Multi-pass form for the classes with many contracted intermediates.  Pass J
// accumulates [e0|f0] for every e and a chunk of f in registers over the whole
// primitive loop and parks the chunk in the wavefront's workspace; the
// horizontal recurrences then run as short loops: the ket step for one e at a
// time into X[e][cd], the bra step plus digestion for one (c, d) at a time.
template <class C, typename T, int G, int J, class A, bool ATT = false>
__device__ __forceinline__ void split_passes(const EriLaunch& a, int i, int k, int sub, T ACx,
                                             T ACy, T ACz, A cacc, int z) {
  // pass J accumulates the rows e = E0 .. E0+NEJ-1 of the contracted [e0|f0]
  constexpr int NEJ = C::template Pass<J>::NE, E0 = C::template Pass<J>::E0;
  T acc[NEJ * C::NF];
#pragma unroll
  for (int t = 0; t < NEJ * C::NF; ++t) acc[t] = T(0);
  contract<C::L, T, G>(a, global_boys<C::L, T, ATT>(a), i, k, sub, ACx, ACy, ACz,
                                      [&](const T* F, const VrrCoef<T>& c) {
    C::template vrr_pass<J, T>(F, c, acc);
  });
  group_sum_all<G>(acc);
  if (sub == 0) {  // the group's first lane carries the quartet from here on
#pragma unroll
    for (int t = 0; t < NEJ * C::NF; ++t) cacc[z + E0 * C::NF + t] = acc[t];
  }
  if constexpr (J + 1 < C::NPASS)
    split_passes<C, T, G, J + 1, A, ATT>(a, i, k, sub, ACx, ACy, ACz, cacc, z);
}

template <class C, typename T, class A>
__device__ __forceinline__ void split_ket_hrr(A cacc, A X, int z, T CDx, T CDy, T CDz, int e0,
                                              int de) {
  constexpr int NCD = C::NC * C::ND;
#pragma nounroll
  for (int e = e0; e < C::NE; e += de) {
    T f[C::NF];
#pragma unroll
    for (int t = 0; t < C::NF; ++t) f[t] = cacc[z + e * C::NF + t];
    T o[NCD];
    C::template ket_hrr<T>(f, CDx, CDy, CDz, o);
#pragma unroll
    for (int t = 0; t < NCD; ++t) X[z + e * NCD + t] = o[t];
  }
}

template <class C, typename T, int G, bool ATT = false>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(class_waves<C, T>())))
void eri_jk_split_kernel(const EriLaunch a) {
  constexpr int NCD = C::NC * C::ND;
  constexpr int QPW = kWave / G;
  const int lane = threadIdx.x & (kWave - 1);
  const int sub = lane & (G - 1), ql = lane / G;
  const int wave = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  if (wave >= a.nwaves) return;
  // workspace of this wave: T values (contracted [e0|f0], ket-transformed X),
  // then FP64 exchange accumulators; one slot per quartet of the wave step
  constexpr int NT = C::NACC + C::NE * NCD;
  constexpr int NK = C::NA * C::NC + C::NA * C::ND + C::NB * C::NC + C::NB * C::ND;
  using AT = LaneArr<T, QPW>;
  using AD = LaneArr<double, kWave>;
  char* wbase = static_cast<char*>(a.ws) + static_cast<size_t>(wave) * split_wave_bytes<C, T>(G);
  T* const cacc0 = reinterpret_cast<T*>(wbase) + ql;
  // FP64 K partial blocks of every lane (the G lanes of a quartet split its
  // (c, d) loop) and the J_cd block of every quartet slot
  double* const kw0 = reinterpret_cast<double*>(wbase + static_cast<size_t>(QPW) * NT * sizeof(T));
  double* const kac0 = kw0;
  double* const kad0 = kac0 + C::NA * C::NC * kWave;
  double* const kbc0 = kad0 + C::NA * C::ND * kWave;
  double* const kbd0 = kbc0 + C::NB * C::NC * kWave;
  double* const jcd0 = kbd0 + C::NB * C::ND * kWave;
  const int z = 0;
  const int nb = a.bra.n, nk = a.ket.n;
  const size_t n = static_cast<size_t>(a.n);
  const size_t nn = n * n;
  for (int item = claim_item(a.next); item < a.nitems; item = claim_item(a.next)) {
  const int4 w = a.items[item];
  const int i = __builtin_amdgcn_readfirstlane(w.x);
  const int kbeg = __builtin_amdgcn_readfirstlane(w.y);
  const int kend = __builtin_amdgcn_readfirstlane(w.z);
  const double Ax = a.bra.A[i], Ay = a.bra.A[nb + i], Az = a.bra.A[2 * nb + i];
  const T ABx = T(a.bra.AB[i]), ABy = T(a.bra.AB[nb + i]), ABz = T(a.bra.AB[2 * nb + i]);
  const int a0 = a.bra.bf[i], b0 = a.bra.bf[nb + i];
  const double fbra = a.bra.fpair[i];

  for (int kc = kbeg; kc < kend; kc += QPW) {
    // the workspace arrays, re-derived per ket step through opaque(): their
    // hundreds of element addresses are then formed at each use rather than
    // kept live across the loop, which spilled them to scratch
    const AT cacc{opaque(cacc0)};
    const AT X{opaque(cacc0 + static_cast<size_t>(C::NACC) * QPW)};
    const AD kac{opaque(kac0 + lane)}, kad{opaque(kad0 + lane)}, kbc{opaque(kbc0 + lane)},
        kbd{opaque(kbd0 + lane)};
    const LaneArr<double, QPW> jcdw{opaque(jcd0 + ql)};
    const bool inrange = kc + ql < kend;
    const bool active = inrange && sub == 0;
    const int k = inrange ? kc + ql : kend - 1;
    const T ACx = T(Ax - a.ket.A[k]), ACy = T(Ay - a.ket.A[nk + k]),
            ACz = T(Az - a.ket.A[2 * nk + k]);
    split_passes<C, T, G, 0, AT, ATT>(a, i, k, sub, ACx, ACy, ACz, cacc, z);
    const T CDx = T(a.ket.AB[k]), CDy = T(a.ket.AB[nk + k]), CDz = T(a.ket.AB[2 * nk + k]);
    // the G lanes of a quartet share the horizontal recurrences and the
    // digestion: lane `sub` takes e = sub, sub+G, ... and (c,d) = sub, sub+G, ...
    lanes_sync();   // cacc was written by the group's first lane
    split_ket_hrr<C, T, AT>(cacc, X, z, CDx, CDy, CDz, sub, G);
    lanes_sync();   // X rows come from all lanes of the group
    const int c0 = a.ket.bf[k], d0 = a.ket.bf[nk + k];
    (void)active;
    const double fq =
        inrange ? fbra * a.ket.fpair[k] * ((a.same_bin && k == i) ? 0.5 : 1.0) : 0.0;

    for (int m = 0; m < a.n_dm; ++m) {
      const double* Dm = a.D + m * nn;
      double* Jm = a.J + (item % a.ncopy) * a.copy_stride + m * nn;
      double* Km = a.K + (item % a.ncopy) * a.copy_stride + m * nn;
      double Dab[C::NA * C::NB], jab[C::NA * C::NB];
#pragma unroll
      for (int x = 0; x < C::NA; ++x)
#pragma unroll
        for (int y = 0; y < C::NB; ++y) {
          Dab[x * C::NB + y] = Dm[(a0 + x) * n + b0 + y];
          jab[x * C::NB + y] = 0.0;
        }
#pragma unroll
      for (int t = 0; t < C::NA * C::NC; ++t) kac[z + t] = 0.0;
#pragma unroll
      for (int t = 0; t < C::NA * C::ND; ++t) kad[z + t] = 0.0;
#pragma unroll
      for (int t = 0; t < C::NB * C::NC; ++t) kbc[z + t] = 0.0;
#pragma unroll
      for (int t = 0; t < C::NB * C::ND; ++t) kbd[z + t] = 0.0;

#pragma nounroll
      for (int cd = sub; cd < NCD; cd += G) {
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
        jcdw[z + cd] = 2.0 * jcd;
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
        if (lane == kWaveSumLane)
          atomic_add(&Jm[(a0 + t / C::NB) * n + b0 + t % C::NB], 2.0 * s, a.det_lo);
      }
      // out-of-range slots hold zeros (fq = 0); K blocks are summed over the
      // G lanes of each slot
      scatter_ws<C::NC, C::ND, QPW, 1>(Jm, n, c0, d0, jcd0, a.det_lo);
      scatter_ws<C::NA, C::NC, QPW, G>(Km, n, a0, c0, kac0, a.det_lo);
      scatter_ws<C::NA, C::ND, QPW, G>(Km, n, a0, d0, kad0, a.det_lo);
      scatter_ws<C::NB, C::NC, QPW, G>(Km, n, b0, c0, kbc0, a.det_lo);
      scatter_ws<C::NB, C::ND, QPW, G>(Km, n, b0, d0, kbd0, a.det_lo);
    }
  }
  }
}

template <class C>
__global__ __launch_bounds__(kBlock) void schwarz_split_kernel(const EriLaunch a, double* Qout) {
  constexpr int NCD = C::NC * C::ND;
  constexpr int G = kSchwarzSplitLanes;   // one wavefront per pair
  constexpr int NT = C::NACC + C::NE * NCD;
  static_assert(C::NA * C::NB == NCD, "diagonal class");
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  if (wave >= a.nwaves) return;
  const int n = a.bra.n;
  using AD = LaneArr<double, 1>;
  double* wl = static_cast<double*>(a.ws) + static_cast<size_t>(wave) * NT;
  const AD cacc{wl};
  const AD X{wl + C::NACC};
  const int z = 0;
  for (int t = wave; t < n; t += a.nwaves) {
    split_passes<C, double, G, 0, AD>(a, t, t, lane, 0.0, 0.0, 0.0, cacc, z);
    const double ABx = a.bra.AB[t], ABy = a.bra.AB[n + t], ABz = a.bra.AB[2 * n + t];
    lanes_sync();
    split_ket_hrr<C, double, AD>(cacc, X, z, ABx, ABy, ABz, lane, G);
    lanes_sync();
    // diagonal (ab|ab): lane cd takes component cd of the bra recurrence
    double mx = 0.0;
    if (lane < NCD) {
      double ev[C::NE];
#pragma unroll
      for (int e = 0; e < C::NE; ++e) ev[e] = X[z + e * NCD + lane];
      double ab[C::NA * C::NB];
      C::template bra_hrr<double>(ev, ABx, ABy, ABz, ab);
#pragma unroll
      for (int s = 0; s < C::NA * C::NB; ++s)
        if (s == lane) mx = ab[s];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, kWave));
    if (lane == 0) Qout[t] = sqrt(fmax(mx, 0.0));
    lanes_sync();   // the workspace is rewritten for the next pair
  }
}

}  // namespace jk
