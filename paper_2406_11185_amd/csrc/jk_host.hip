// Host side of the J/K library: C ABI, basis bookkeeping, setup kernels
// (shell-pair data, Cauchy-Schwarz factors, screening and work lists) and the
// dispatch of the per-class integral kernels.
//
// Steps of one jk_build (all device work on the caller's stream):
//   1. shell pairs grouped into bins (angular-momentum class, primitive-pair
//      count) on the host -- integer bookkeeping only;
//   2. pair_data_kernel: Gaussian-product data of every primitive pair;
//   3. schwarz_kernel per bin: Q_AB = sqrt(max (ab|ab)) with the class's own
//      integral code;
//   4. segmented radix sort of each bin by Q (descending), pair data rebuilt
//      in that order;
//   5. ranges_kernel: for each bra pair and ket bin, binary searches give the
//      contiguous ket ranges with Q_bra*Q_ket >= fp32_below (FP64),
//      tol <= Q_bra*Q_ket < fp32_below (FP32 in mixed mode), and the rest is
//      skipped -- the paper's skip / single / double dispatch ("Electron
//      Repulsion Integrals" paragraph, third item) without materialising
//      quartet lists;
//   6. the kept-quartet counts come back to the host, which picks for each bin
//      pair the item size (64 to 1024 kets) that gives enough wavefronts;
//      count + scan + expand_kernel write work items {bra, ket begin, ket end};
//      a second small device->host copy returns the item ranges per launch;
//   7. J, K cleared, one integral+digestion launch per (class pair, precision),
//      spread over the context's streams so that small classes overlap, then
//      J = A + A^T, K = B + B^T in place (finalize_kernel).
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "jk.h"
#include "jk_device.hpp"
#include "jk_classes.hpp"
#include "jk_grad_device.hpp"
#include "jk_guard.hpp"

using namespace jk;

namespace {

constexpr int kPairClass[3][3] = {{0, -1, -1}, {1, 2, -1}, {3, 4, 5}};  // [la][lb], la >= lb
constexpr int kPairL[6][2] = {{0, 0}, {1, 0}, {1, 1}, {2, 0}, {2, 1}, {2, 2}};

inline int ncart(int l) { return (l + 1) * (l + 2) / 2; }
inline int quartet_class(int X, int Y) { return X * (X + 1) / 2 + Y; }  // X >= Y

struct Fail {
  int code;
  std::string msg;
};

#define HIP_OK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      throw Fail{JK_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)};          \
  } while (0)

// ---------------------------------------------------------------------------------
// Boys-function tables (host generation).  Each entry is the power series
//   F_m(T) = e^{-T} sum_{k>=0} (2T)^k / ((2m+1)(2m+3)...(2m+2k+1))
// summed in long double until the terms stop contributing.
long double boys_series(int m, long double T) {
  long double term = 1.0L / (2 * m + 1), sum = term;
  for (int k = 1; k < 100000; ++k) {
    term *= 2.0L * T / (2 * m + 2 * k + 1);
    sum += term;
    if (term < sum * 1e-21L) break;
  }
  return std::exp(-T) * sum;
}

void make_boys_tables(std::vector<double>& t64, std::vector<float>& t32) {
  const int nL = kBoysMaxL + 1;
  t64.assign(static_cast<size_t>(nL) * kBoysRows * kBoysRow, 0.0);
  t32.assign(static_cast<size_t>(nL) * kBoys32Rows * kBoys32Row, 0.0f);
  std::vector<long double> F(kBoysMaxL + 7);
  for (int i = 0; i < kBoysRows; ++i) {
    const long double T = static_cast<long double>(i) * 0.05L;
    for (int m = 0; m < kBoysMaxL + 7; ++m) F[m] = boys_series(m, T);
    const long double eT = std::exp(-T);
    for (int L = 0; L < nL; ++L) {
      double* row = &t64[(static_cast<size_t>(L) * kBoysRows + i) * kBoysRow];
      for (int k = 0; k < 7; ++k) row[k] = static_cast<double>(F[L + k]);
      row[7] = static_cast<double>(eT);
      if (i < kBoys32Rows) {
        float* r32 = &t32[(static_cast<size_t>(L) * kBoys32Rows + i) * kBoys32Row];
        for (int k = 0; k < 4; ++k) r32[k] = static_cast<float>(F[L + k]);
        r32[4] = static_cast<float>(eT);
      }
    }
  }
}

// ---------------------------------------------------------------------------------
// Device data of the setup kernels.
struct ShellDev {
  const double* xyz;   // [n_shells][3] centre
  const int* l;
  const int* nprim;
  const int* prim0;
  const int* bf0;
  const int* atom;
  const double* exps;
  const double* coefs;
};

struct PairOut {
  double* prim;        // all bins, bin b at prim_off[b]
  double* primT;       // pair-major copy, same offsets
  float* prim32;       // FP32 copies of prim and primT (null: not written)
  float* primT32;
  double* A;           // bin b at 3*pair_off[b], [3][n_b]
  double* AB;
  int* bf;             // bin b at 2*pair_off[b]
  int* atoms;
  double* fpair;       // bin b at pair_off[b]
};

__device__ __forceinline__ int find_bin(const int* off, int nbins, int g) {
  int lo = 0, hi = nbins;  // off[lo] <= g < off[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= g) lo = mid; else hi = mid;
  }
  return lo;
}

// Step 2: primitive-pair data.  For primitives a (on A) and b (on B):
//   p = a + b,  P = (aA + bB)/p,  K_AB = c_a c_b exp(-ab/p |A-B|^2),
//   Kt = sqrt(2) pi^{5/4} K_AB / p  (so that Kt_AB Kt_CD / sqrt(p+q) is the
//   prefactor 2 pi^{5/2} K_AB K_CD / (pq sqrt(p+q)) of (00|00)^(m)).
// Slot g of the output holds pair src[g] (identity if src is null).
__global__ void pair_data_kernel(int npairs, const int* __restrict__ pair_s1,
                                 const int* __restrict__ pair_s2, const int* __restrict__ src,
                                 const int* __restrict__ bin_off, const int* __restrict__ bin_npp,
                                 const long long* __restrict__ bin_prim_off, int nbins,
                                 ShellDev sh, PairOut out) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= npairs) return;
  const int b = find_bin(bin_off, nbins, g);
  const int n = bin_off[b + 1] - bin_off[b];
  const int t = g - bin_off[b];
  const int s = src ? src[g] : g;
  const int s1 = pair_s1[s], s2 = pair_s2[s];
  const double A[3] = {sh.xyz[3 * s1], sh.xyz[3 * s1 + 1], sh.xyz[3 * s1 + 2]};
  const double B[3] = {sh.xyz[3 * s2], sh.xyz[3 * s2 + 1], sh.xyz[3 * s2 + 2]};
  const double AB[3] = {A[0] - B[0], A[1] - B[1], A[2] - B[2]};
  const double AB2 = AB[0] * AB[0] + AB[1] * AB[1] + AB[2] * AB[2];
  const int po = 3 * bin_off[b];
  for (int c = 0; c < 3; ++c) {
    out.A[po + c * n + t] = A[c];
    out.AB[po + c * n + t] = AB[c];
  }
  out.bf[2 * bin_off[b] + t] = sh.bf0[s1];
  out.bf[2 * bin_off[b] + n + t] = sh.bf0[s2];
  out.atoms[2 * bin_off[b] + t] = sh.atom[s1];
  out.atoms[2 * bin_off[b] + n + t] = sh.atom[s2];
  out.fpair[bin_off[b] + t] = (s1 == s2) ? 0.5 : 1.0;
  const double kSqrt2Pi54 = 5.9149671727956128778;  // sqrt(2) * pi^(5/4)
  const int n1 = sh.nprim[s1], n2 = sh.nprim[s2];
  double* prim = out.prim + bin_prim_off[b];
  double* primT = out.primT + bin_prim_off[b] + static_cast<size_t>(t) * n1 * n2 * kPrimFields;
  for (int u = 0; u < n1; ++u)
    for (int v = 0; v < n2; ++v) {
      const int pp = u * n2 + v;
      const double ea = sh.exps[sh.prim0[s1] + u], eb = sh.exps[sh.prim0[s2] + v];
      const double ca = sh.coefs[sh.prim0[s1] + u], cb = sh.coefs[sh.prim0[s2] + v];
      const double p = ea + eb, rp = 1.0 / p;
      const double Kab = ca * cb * exp(-ea * eb * rp * AB2);
      double* f = prim + static_cast<size_t>(pp) * kPrimFields * n + t;
      f[kP * n] = p;
      f[kOo2p * n] = 0.5 * rp;
      f[kPAx * n] = -eb * rp * AB[0];   // P - A = b/p (B - A)
      f[kPAy * n] = -eb * rp * AB[1];
      f[kPAz * n] = -eb * rp * AB[2];
      f[kKt * n] = kSqrt2Pi54 * Kab * rp;
      f[kTwoA * n] = 2.0 * ea;
      f[kTwoB * n] = 2.0 * eb;
      double* h = primT + static_cast<size_t>(pp) * kPrimFields;
      for (int x = 0; x < kPrimFields; ++x) h[x] = f[x * n];
      if (out.prim32) {
        const size_t o = bin_prim_off[b] + static_cast<size_t>(pp) * kPrimFields * n + t;
        const size_t oT = bin_prim_off[b] + (static_cast<size_t>(t) * n1 * n2 + pp) * kPrimFields;
        for (int x = 0; x < kPrimFields; ++x) {
          out.prim32[o + static_cast<size_t>(x) * n] = static_cast<float>(f[x * n]);
          out.primT32[oT + x] = static_cast<float>(f[x * n]);
        }
      }
    }
  (void)bin_npp;
}

__global__ void iota_kernel(int n, const int* __restrict__ bin_off, int nbins, int* out) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  out[g] = g - bin_off[find_bin(bin_off, nbins, g)];
}

__global__ void local_to_global_kernel(int n, const int* __restrict__ bin_off, int nbins,
                                       const int* __restrict__ local, int* out) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  out[g] = bin_off[find_bin(bin_off, nbins, g)] + local[g];
}

// Step 5: screening and precision dispatch of one (bin pair, bra pair).
struct RangeArgs {
  int nt;                       // threads = sum over bin pairs of bra pairs
  int nbp;
  const int* bp_x;              // bra bin of each bin pair
  const int* bp_y;              // ket bin
  const int* bp_t0;             // first thread of each bin pair, [nbp+1]
  const int* bin_off;           // pair offsets of the bins
  const double* Q;              // sorted Q, all bins
  double tol, thr;
  int mixed;
  int* rng;                     // [3][nt] k_lo, k_64, k_tol
  unsigned long long* qstat;    // [nbp][3] FP64 quartets, FP32 quartets, skipped
};

__device__ __forceinline__ int first_below(const double* Qk, int lo, int hi, double qi, double bound) {
  // first k in [lo, hi) with qi * Qk[k] < bound (Qk descending), hi if none
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (qi * Qk[mid] < bound) hi = mid; else lo = mid + 1;
  }
  return lo;
}

__global__ void ranges_kernel(RangeArgs r) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = t < r.nt;
  const int bp = live ? find_bin(r.bp_t0, r.nbp, t) : -1;
  unsigned long long cnt[3] = {0, 0, 0};
  if (live) {
    const int X = r.bp_x[bp], Y = r.bp_y[bp];
    const int i = t - r.bp_t0[bp];
    const double* QX = r.Q + r.bin_off[X];
    const double* QY = r.Q + r.bin_off[Y];
    const int nY = r.bin_off[Y + 1] - r.bin_off[Y];
    const int klo = (X == Y) ? i : 0;
    const double qi = QX[i];
    const int ktol = (r.tol > 0.0) ? first_below(QY, klo, nY, qi, r.tol) : nY;
    int k64 = ktol;
    if (r.mixed) k64 = first_below(QY, klo, ktol, qi, r.thr);
    r.rng[t] = klo;
    r.rng[r.nt + t] = k64;
    r.rng[2 * r.nt + t] = ktol;
    cnt[0] = static_cast<unsigned long long>(k64 - klo);
    cnt[1] = static_cast<unsigned long long>(ktol - k64);
    cnt[2] = static_cast<unsigned long long>(nY - ktol);
  }
  // quartet counts per bin pair: one atomic per wavefront when all its lanes
  // belong to the same bin pair (the usual case), else one per lane
  const int bp0 = __shfl(bp, 0, 64);
  if (__all(bp == bp0 || bp < 0)) {
#pragma unroll
    for (int x = 0; x < 3; ++x)
      for (int off = 32; off > 0; off >>= 1) cnt[x] += __shfl_xor(cnt[x], off, 64);
    if ((threadIdx.x & 63) == 0 && bp0 >= 0)
      for (int x = 0; x < 3; ++x) atomicAdd(&r.qstat[3 * bp0 + x], cnt[x]);
  } else if (live) {
    for (int x = 0; x < 3; ++x) atomicAdd(&r.qstat[3 * bp + x], cnt[x]);
  }
}

// Work items per (thread, precision) for the item sizes chosen per bin pair.
__global__ void count_kernel(int nt, const int* __restrict__ bp_t0, int nbp,
                             const int* __restrict__ rng, const int* __restrict__ chunk, int* cnt) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  const int bp = find_bin(bp_t0, nbp, t);
  const int klo = rng[t], k64 = rng[nt + t], ktol = rng[2 * nt + t];
  const int c0 = chunk[bp], c1 = chunk[nbp + bp];
  cnt[t] = (k64 - klo + c0 - 1) / c0;
  cnt[nt + t] = (ktol - k64 + c1 - 1) / c1;
}

__global__ void expand_kernel(int nt, const int* __restrict__ bp_t0, int nbp,
                              const int* __restrict__ cnt, const int* __restrict__ off,
                              const int* __restrict__ rng, const int* __restrict__ chunk,
                              int4* items) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  const int bp = find_bin(bp_t0, nbp, t);
  const int i = t - bp_t0[bp];
  const int klo = rng[t], k64 = rng[nt + t], ktol = rng[2 * nt + t];
  for (int pr = 0; pr < 2; ++pr) {
    const int beg = pr == 0 ? klo : k64, end = pr == 0 ? k64 : ktol;
    const int ch = chunk[pr * nbp + bp];
    const int c = cnt[pr * nt + t];
    const int base = off[pr * nt + t];
    for (int j = 0; j < c; ++j) {
      const int k0 = beg + j * ch;
      items[base + j] = make_int4(i, k0, min(k0 + ch, end), 0);
    }
  }
}

// seg[pr][bp] = first item of bin pair bp in precision pr; seg[1][nbp] = total.
__global__ void segments_kernel(int nt, int nbp, const int* __restrict__ bp_t0,
                                const int* __restrict__ cnt, const int* __restrict__ off,
                                int* seg) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j > 2 * nbp + 1) return;
  const int pr = j / (nbp + 1), bp = j % (nbp + 1);
  const int t = pr * nt + bp_t0[bp];  // bp == nbp -> first thread of the next precision
  seg[j] = (t < 2 * nt) ? off[t] : off[2 * nt - 1] + cnt[2 * nt - 1];
}

template <typename T>
__global__ void fill_kernel(size_t n, T* a) {
  const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) a[i] = T(0);
}

// Accumulator element idx: an FP64 value, or in deterministic mode the int64
// fixed-point pair (hi at idx, lo at idx + det_lo) summed over the copies and
// over idx, idx2 (the element and its transpose) before one conversion.
__device__ __forceinline__ double acc_sum(const double* A, size_t idx, size_t idx2, int ncopy,
                                          size_t stride, size_t det_lo) {
  if (!det_lo) {
    double v = 0.0;
    for (int c = 0; c < ncopy; ++c) v += A[c * stride + idx] + A[c * stride + idx2];
    return v;
  }
  const unsigned long long* w = reinterpret_cast<const unsigned long long*>(A);
  unsigned long long hi = 0, lo = 0;
  for (int c = 0; c < ncopy; ++c) {
    hi += w[c * stride + idx] + w[c * stride + idx2];
    lo += w[c * stride + idx + det_lo] + w[c * stride + idx2 + det_lo];
  }
  return static_cast<double>(static_cast<long long>(hi)) * (1.0 / kFixHi) +
         static_cast<double>(static_cast<long long>(lo)) * (1.0 / (kFixHi * kFixLo));
}

// Step a7 (finalize): J = sum over the accumulator copies of A_J + A_J^T, K the
// same from A_K; optionally dE/dD = J - K/2 and the per-block partial sums of
// <D, J> and <D, K> (each symmetric pair (i, j), (j, i) once, weighted by
// D_ij + D_ji).  One thread per element with j >= i; grid (blocks, n_dm).
struct FinArgs {
  int n, ncopy;
  size_t stride;        // elements between accumulator copies
  size_t det_lo;        // deterministic mode: offset of the lo words (else 0)
  const double* AJ;     // accumulators [ncopy][n_dm][n][n] (== J, K in place when
  const double* AK;     //   ncopy == 1 outside deterministic mode)
  const double* D;
  double* J;
  double* K;
  double* dEdD;         // optional [n_dm][n][n]
  double* epart;        // optional [n_dm][gridDim.x][2]
};

constexpr int kFinBlock = 256;

__global__ __launch_bounds__(kFinBlock) void finalize_kernel(FinArgs f) {
  const size_t nn = static_cast<size_t>(f.n) * f.n;
  const int m = blockIdx.y;
  const size_t r = static_cast<size_t>(blockIdx.x) * kFinBlock + threadIdx.x;
  double ej = 0.0, ek = 0.0;
  if (r < nn) {
    const int i = static_cast<int>(r / f.n), j = static_cast<int>(r % f.n);
    if (j >= i) {
      const size_t ij = m * nn + static_cast<size_t>(i) * f.n + j;
      const size_t ji = m * nn + static_cast<size_t>(j) * f.n + i;
      const double sj = acc_sum(f.AJ, ij, ji, f.ncopy, f.stride, f.det_lo);
      const double sk = acc_sum(f.AK, ij, ji, f.ncopy, f.stride, f.det_lo);
      f.J[ij] = sj;
      f.J[ji] = sj;
      f.K[ij] = sk;
      f.K[ji] = sk;
      if (f.dEdD) {
        f.dEdD[ij] = sj - 0.5 * sk;
        f.dEdD[ji] = sj - 0.5 * sk;
      }
      const double w = (i == j) ? f.D[ij] : f.D[ij] + f.D[ji];
      ej = w * sj;
      ek = w * sk;
    }
  }
  if (!f.epart) return;
  __shared__ double red[2][kFinBlock];
  red[0][threadIdx.x] = ej;
  red[1][threadIdx.x] = ek;
  __syncthreads();
  for (int h = kFinBlock / 2; h > 0; h >>= 1) {   // fixed pairing: same order every run
    if (static_cast<int>(threadIdx.x) < h) {
      red[0][threadIdx.x] += red[0][threadIdx.x + h];
      red[1][threadIdx.x] += red[1][threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double* p = f.epart + (static_cast<size_t>(m) * gridDim.x + blockIdx.x) * 2;
    p[0] = red[0][0];
    p[1] = red[1][0];
  }
}

// E_J = 1/2 <D, J>, E_K = 1/4 <D, K>, E = E_J - E_K from the partial sums, one
// workgroup per density, summed in a fixed order.
__global__ __launch_bounds__(kFinBlock) void energy_kernel(int nblk, const double* epart, double* E) {
  const int m = blockIdx.x;
  __shared__ double red[2][kFinBlock];
  double sj = 0.0, sk = 0.0;
  for (int b = threadIdx.x; b < nblk; b += kFinBlock) {
    sj += epart[(static_cast<size_t>(m) * nblk + b) * 2];
    sk += epart[(static_cast<size_t>(m) * nblk + b) * 2 + 1];
  }
  red[0][threadIdx.x] = sj;
  red[1][threadIdx.x] = sk;
  __syncthreads();
  for (int h = kFinBlock / 2; h > 0; h >>= 1) {
    if (static_cast<int>(threadIdx.x) < h) {
      red[0][threadIdx.x] += red[0][threadIdx.x + h];
      red[1][threadIdx.x] += red[1][threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double ej = 0.5 * red[0][0], ek = 0.25 * red[1][0];
    E[3 * m] = ej;
    E[3 * m + 1] = ek;
    E[3 * m + 2] = ej - ek;
  }
}

// Deterministic gradient: dE/dR from its int64 fixed-point pairs.
__global__ void fix_to_double_kernel(size_t n, const unsigned long long* w, size_t lo, double* out) {
  const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[i] = static_cast<double>(static_cast<long long>(w[i])) * (1.0 / kFixHi) +
           static_cast<double>(static_cast<long long>(w[i + lo])) * (1.0 / (kFixHi * kFixLo));
}

inline unsigned grid_of(size_t n, int block) { return static_cast<unsigned>((n + block - 1) / block); }

// Upper bound of the workspace one launch of a multi-pass or gradient kernel
// uses; the launch then loops over its items with correspondingly few waves.
constexpr size_t kWsBudget = size_t(1) << 30;
constexpr size_t kGradLdsBytes = 48 << 10;   // workgroup copy of dE/dR in LDS up to this size
constexpr size_t kMaxCopies = 8;                  // accumulator copies of J and K
constexpr size_t kAccBudget = size_t(256) << 20;   // bytes for them

// ---------------------------------------------------------------------------------
// Grow-only device buffers owned by a context.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

enum Slot {
  sShellXyz, sShellI, sExps, sCoefs, sPairS, sBinOff, sBinNpp, sBinPrim, sPrimTmp, sPrim, sPrimTmpT, sPrimT,
  sA, sAB, sBf, sAtoms, sFpair, sAtmp, sABtmp, sBftmp, sAtomstmp, sFpairtmp, sQtmp, sQ,
  sIdx, sIdxSorted, sPerm, sPrim32, sPrimT32, sBp, sCnt, sOff, sRng, sQstat, sSeg, sItems, sCub, sChunk, sWs0, sWs1,
  sWs2, sWs3, sWsSchwarz, sNext, sAcc, sEpart, sGradAcc, sNumSlots
};

}  // namespace

namespace jk {
namespace {
thread_local std::string g_guard_err;

struct GuardKey {
  const void* fn;
  int device;
  unsigned block;
  size_t lds;
  bool operator<(const GuardKey& o) const {
    if (fn != o.fn) return fn < o.fn;
    if (device != o.device) return device < o.device;
    if (block != o.block) return block < o.block;
    return lds < o.lds;
  }
};
struct GuardInfo {
  size_t private_per_lane;
  int blocks_per_cu;
  int num_cu;
};
std::map<GuardKey, GuardInfo> g_guard_cache;
}  // namespace

// Scratch guard of every kernel launch: the kernel's private-segment bytes
// per lane (from the runtime's function attributes) times the lanes of its
// resident wavefronts must fit kScratchBudget.  Attributes are read once per
// (kernel, device, block, LDS) and cached.
int guard_launch(const void* kernel, unsigned grid_blocks, unsigned block_threads, size_t lds_bytes) {
  int device = 0;
  if (hipGetDevice(&device) != hipSuccess) device = 0;
  const GuardKey key{kernel, device, block_threads, lds_bytes};
  auto it = g_guard_cache.find(key);
  if (it == g_guard_cache.end()) {
    hipFuncAttributes attr{};
    GuardInfo gi{0, 1, 1};
    if (hipFuncGetAttributes(&attr, kernel) == hipSuccess) gi.private_per_lane = attr.localSizeBytes;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, static_cast<int>(block_threads),
                                                     lds_bytes) == hipSuccess && nb > 0)
      gi.blocks_per_cu = nb;
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess &&
        ncu > 0)
      gi.num_cu = ncu;
    (void)hipGetLastError();
    it = g_guard_cache.emplace(key, gi).first;
  }
  const GuardInfo& gi = it->second;
  const size_t wpb = (block_threads + kWave - 1) / kWave;
  const size_t need = launch_scratch_bytes(gi.private_per_lane, size_t(grid_blocks) * wpb,
                                           gi.num_cu, gi.blocks_per_cu, wpb);
  if (launch_scratch_ok(need)) return 0;
  g_guard_err = "a kernel launch would need " + std::to_string(need >> 20) +
                " MiB of scratch (" + std::to_string(gi.private_per_lane) +
                " bytes per lane), over the " + std::to_string(kScratchBudget >> 20) + " MiB limit";
  return 1;
}

// The guard's message since the last call, cleared.
std::string take_guard_error() {
  std::string m;
  m.swap(g_guard_err);
  return m;
}
}  // namespace jk

// Device scratch of jk_build_noalloc: a file-scope array each GPU holds once
// the library's code object is loaded on it, until the process ends.  Host code
// never uses its name as an address: jk_ctx_create asks the runtime for the
// array's device address (hipGetSymbolAddress) with the context's device
// current and keeps that pointer in the context.
constexpr size_t kNoAllocBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kNoAllocBytes];
// Host staging of the two small device-to-host copies in jk_build_noalloc.
constexpr size_t kNoAllocHostBytes = size_t(1) << 20;

namespace {
struct Setup;
}  // namespace

struct jk_ctx {
  int device = 0;
  char* noalloc_base = nullptr;    // device address of `scratch` on this context's device
  bool noalloc = false;            // inside jk_build_noalloc: buffers come from scratch
  size_t noalloc_off = 0;          // bytes of scratch handed out in this call
  std::vector<char> noalloc_host;  // kNoAllocHostBytes, allocated with the context
  size_t ws_budget = 0;            // workspace bytes a multi-pass launch may use
  // setup kept for jk_opts.reuse_setup: its key (basis arrays, tol and the
  // options the setup depends on) and the setup itself, whose device arrays
  // live in this context's buffers until a later setup replaces them
  std::vector<char> setup_key;
  std::shared_ptr<Setup> setup_kept;
  int num_cu = 0;
  std::string err;
  DevBuf buf[sNumSlots];
  size_t scratch_limit = 0;
  double* boys64 = nullptr;
  float* boys32 = nullptr;
  jk_stats stats{};
  bool timed = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  struct Timed { int cls; int fp32; size_t e0; };
  std::vector<Timed> timed_launches;
  size_t ev_setup0 = 0, ev_setup1 = 0, ev_end = 0;
  void* host_pinned = nullptr;
  size_t host_pinned_bytes = 0;
#ifndef JK_STREAMS
#define JK_STREAMS 3
#endif
  // class launches are spread over these (measured on gfx950 for the 270-function
  // molecule: 1 stream 33.5 ms, 2 streams 29.1 ms, 3 streams 28.8 ms per build)
  static constexpr int kStreams = JK_STREAMS;
  hipStream_t streams[kStreams] = {};
  hipEvent_t fork_ev = nullptr;
  hipEvent_t join_ev[kStreams] = {};
};

namespace {

thread_local std::string g_create_err;

template <typename T>
T* dev(jk_ctx* c, Slot s, size_t count) {
  const size_t bytes = std::max<size_t>(count * sizeof(T), 256);
  if (c->noalloc) {   // bump allocation from the static scratch array, 256-byte aligned
    const size_t at = (c->noalloc_off + 255) & ~size_t(255);
    if (at + bytes > kNoAllocBytes)
      throw Fail{JK_ENOMEM, "jk_build_noalloc: the call needs more than the " +
                                std::to_string(kNoAllocBytes >> 20) + " MiB of static scratch"};
    c->noalloc_off = at + bytes;
    return reinterpret_cast<T*>(c->noalloc_base + at);
  }
  DevBuf& b = c->buf[s];
  if (c->scratch_limit) {
    size_t total = 0;
    for (int i = 0; i < sNumSlots; ++i) total += (i == s) ? std::max(b.bytes, bytes) : c->buf[i].bytes;
    if (total > c->scratch_limit)
      throw Fail{JK_ENOMEM, "scratch need of " + std::to_string(total) + " bytes is over max_scratch_bytes"};
  }
  if (b.bytes < bytes) {
    if (b.p) HIP_OK(hipFree(b.p));
    b.p = nullptr;
    b.bytes = 0;
    if (hipMalloc(&b.p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      throw Fail{JK_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed"};
    }
    b.bytes = bytes;
  }
  return static_cast<T*>(b.p);
}

void* pinned(jk_ctx* c, size_t bytes) {
  if (c->noalloc) {   // pageable staging allocated with the context (copies complete on sync)
    if (bytes > c->noalloc_host.size())
      throw Fail{JK_ENOMEM, "jk_build_noalloc: host staging of " + std::to_string(bytes) +
                                " bytes is over its " + std::to_string(kNoAllocHostBytes) + " bytes"};
    return c->noalloc_host.data();
  }
  if (c->host_pinned_bytes < bytes) {
    if (c->host_pinned) HIP_OK(hipHostFree(c->host_pinned));
    c->host_pinned = nullptr;
    c->host_pinned_bytes = 0;
    HIP_OK(hipHostMalloc(&c->host_pinned, bytes, hipHostMallocDefault));
    c->host_pinned_bytes = bytes;
  }
  return c->host_pinned;
}

size_t event(jk_ctx* c, hipStream_t s) {  // records on s, returns its index
  if (c->ev_used == c->ev_pool.size()) {
    hipEvent_t e;
    HIP_OK(hipEventCreate(&e));
    c->ev_pool.push_back(e);
  }
  HIP_OK(hipEventRecord(c->ev_pool[c->ev_used], s));
  return c->ev_used++;
}

int validate(const jk_basis* b, int32_t* nbf) {
  if (!b) return JK_EINVAL;
  if (b->n_atoms < 1 || b->n_shells < 1 || !b->xyz || !b->shell_atom || !b->shell_l ||
      !b->shell_nprim || !b->shell_prim0 || !b->exps || !b->coefs)
    return JK_EINVAL;
  for (int a = 0; a < 3 * b->n_atoms; ++a)
    if (!std::isfinite(b->xyz[a])) return JK_EINVAL;
  long long n = 0;
  for (int s = 0; s < b->n_shells; ++s) {
    const int l = b->shell_l[s], np = b->shell_nprim[s], p0 = b->shell_prim0[s];
    if (b->shell_atom[s] < 0 || b->shell_atom[s] >= b->n_atoms) return JK_EINVAL;
    if (l < 0 || np < 1 || p0 < 0) return JK_EINVAL;
    if (l > JK_MAX_L || np > JK_MAX_NPRIM) return JK_EUNSUPPORTED;
    for (int k = 0; k < np; ++k) {
      const double e = b->exps[p0 + k], cf = b->coefs[p0 + k];
      if (!(e > 0.0) || !std::isfinite(e) || !std::isfinite(cf)) return JK_EINVAL;
    }
    n += ncart(l);
    if (n > (1 << 15)) return JK_EUNSUPPORTED;
  }
  if (nbf) *nbf = static_cast<int32_t>(n);
  return JK_OK;
}

std::string validate_msg(int rc) {
  return rc == JK_EUNSUPPORTED
             ? "basis outside the supported set (l <= 2, <= 8 primitives, <= 32768 functions)"
             : "malformed basis (counts, NULL arrays, atom index, exponents or coefficients)";
}

// Host bookkeeping of the shell pairs and their bins.
struct Plan {
  int n_bf = 0, n_shells = 0, n_atoms = 0, npairs = 0, nbins = 0;
  std::vector<int> bin_cls, bin_npp, bin_off;      // bin_off [nbins+1]
  std::vector<long long> bin_prim;                 // offset into prim (doubles), [nbins+1]
  std::vector<int> pair_s1, pair_s2;               // canonical pairs in bin order
  std::vector<int> bf0;
  std::vector<int> bp_x, bp_y, bp_t0;              // bin pairs
  int nt = 0;
};

Plan make_plan(const jk_basis* b) {
  Plan P;
  P.n_shells = b->n_shells;
  P.n_atoms = b->n_atoms;
  P.bf0.resize(b->n_shells);
  int n = 0;
  for (int s = 0; s < b->n_shells; ++s) { P.bf0[s] = n; n += ncart(b->shell_l[s]); }
  P.n_bf = n;
  // bins keyed by (pair class, primitive-pair count)
  std::map<std::pair<int, int>, std::vector<std::pair<int, int>>> bins;
  for (int i = 0; i < b->n_shells; ++i)
    for (int j = 0; j <= i; ++j) {
      int s1 = i, s2 = j;
      if (b->shell_l[s2] > b->shell_l[s1]) std::swap(s1, s2);
      const int cls = kPairClass[b->shell_l[s1]][b->shell_l[s2]];
      const int npp = b->shell_nprim[s1] * b->shell_nprim[s2];
      bins[{cls, npp}].push_back({s1, s2});
    }
  P.bin_off.push_back(0);
  P.bin_prim.push_back(0);
  for (auto& kv : bins) {
    P.bin_cls.push_back(kv.first.first);
    P.bin_npp.push_back(kv.first.second);
    for (auto& pr : kv.second) { P.pair_s1.push_back(pr.first); P.pair_s2.push_back(pr.second); }
    const int nb = static_cast<int>(kv.second.size());
    P.bin_off.push_back(P.bin_off.back() + nb);
    P.bin_prim.push_back(P.bin_prim.back() + static_cast<long long>(kv.first.second) * kPrimFields * nb);
  }
  P.nbins = static_cast<int>(P.bin_cls.size());
  P.npairs = P.bin_off.back();
  P.bp_t0.push_back(0);
  for (int X = 0; X < P.nbins; ++X)
    for (int Y = 0; Y <= X; ++Y) {
      P.bp_x.push_back(X);
      P.bp_y.push_back(Y);
      P.bp_t0.push_back(P.bp_t0.back() + (P.bin_off[X + 1] - P.bin_off[X]));
    }
  P.nt = P.bp_t0.back();
  return P;
}

template <typename T>
void upload(const std::vector<T>& v, T* d, hipStream_t s) {
  if (!v.empty()) HIP_OK(hipMemcpyAsync(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

BinView bin_view(const Plan& P, int b, double* prim, double* primT, double* A, double* AB, int* bf,
                 int* atoms, double* fpair, double* Q, float* prim32 = nullptr,
                 float* primT32 = nullptr) {
  BinView v;
  const int o = P.bin_off[b];
  v.n = P.bin_off[b + 1] - o;
  v.npp = P.bin_npp[b];
  v.prim = prim + P.bin_prim[b];
  v.primT = primT + P.bin_prim[b];
  v.prim32 = prim32 ? prim32 + P.bin_prim[b] : nullptr;
  v.primT32 = primT32 ? primT32 + P.bin_prim[b] : nullptr;
  v.A = A + 3 * o;
  v.AB = AB + 3 * o;
  v.bf = bf + 2 * o;
  v.atoms = atoms + 2 * o;
  v.fpair = fpair + o;
  v.Q = Q + o;
  return v;
}

struct Setup {
  Plan P;
  double *prim, *primT, *A, *AB, *fpair, *Q;
  float *prim32, *primT32;
  int *bf, *atoms;
  int4* items;
  std::vector<int> seg;   // [2][nbp+1]
  std::vector<unsigned long long> qstat;
  std::vector<int> chunk; // [2][nbp] kets per work item
  std::vector<int> lanes; // [2][nbp] lanes per shell quartet
};

// Steps 1-6.  Returns the sorted pair data, the work items and their segments.
Setup setup(jk_ctx* c, const jk_basis* b, double tol, const jk_opts& o, hipStream_t s,
            bool grad) {
  Setup S;
  S.P = make_plan(b);
  Plan& P = S.P;
  const int ns = P.n_shells, np = P.npairs;
  int nprim_total = 0;
  for (int sh = 0; sh < ns; ++sh)
    nprim_total = std::max(nprim_total, b->shell_prim0[sh] + b->shell_nprim[sh]);

  // shells
  std::vector<double> sxyz(3 * ns);
  std::vector<int> si(5 * ns);
  for (int sh = 0; sh < ns; ++sh) {
    for (int k = 0; k < 3; ++k) sxyz[3 * sh + k] = b->xyz[3 * b->shell_atom[sh] + k];
    si[sh] = b->shell_l[sh];
    si[ns + sh] = b->shell_nprim[sh];
    si[2 * ns + sh] = b->shell_prim0[sh];
    si[3 * ns + sh] = P.bf0[sh];
    si[4 * ns + sh] = b->shell_atom[sh];
  }
  double* d_sxyz = dev<double>(c, sShellXyz, sxyz.size());
  int* d_si = dev<int>(c, sShellI, si.size());
  double* d_exps = dev<double>(c, sExps, nprim_total);
  double* d_coefs = dev<double>(c, sCoefs, nprim_total);
  int* d_pairs = dev<int>(c, sPairS, 2 * static_cast<size_t>(np));
  int* d_binoff = dev<int>(c, sBinOff, P.nbins + 1);
  int* d_binnpp = dev<int>(c, sBinNpp, P.nbins);
  long long* d_binprim = dev<long long>(c, sBinPrim, P.nbins + 1);
  const size_t nprimd = static_cast<size_t>(P.bin_prim.back());
  double* d_primtmp = dev<double>(c, sPrimTmp, nprimd);
  S.prim = dev<double>(c, sPrim, nprimd);
  S.primT = dev<double>(c, sPrimT, nprimd);
  S.prim32 = dev<float>(c, sPrim32, nprimd);
  S.primT32 = dev<float>(c, sPrimT32, nprimd);
  double* d_primtmpT = dev<double>(c, sPrimTmpT, nprimd);
  S.A = dev<double>(c, sA, 3 * static_cast<size_t>(np));
  S.AB = dev<double>(c, sAB, 3 * static_cast<size_t>(np));
  S.bf = dev<int>(c, sBf, 2 * static_cast<size_t>(np));
  S.atoms = dev<int>(c, sAtoms, 2 * static_cast<size_t>(np));
  S.fpair = dev<double>(c, sFpair, np);
  double* d_Atmp = dev<double>(c, sAtmp, 3 * static_cast<size_t>(np));
  double* d_ABtmp = dev<double>(c, sABtmp, 3 * static_cast<size_t>(np));
  int* d_bftmp = dev<int>(c, sBftmp, 2 * static_cast<size_t>(np));
  int* d_atomstmp = dev<int>(c, sAtomstmp, 2 * static_cast<size_t>(np));
  double* d_fpairtmp = dev<double>(c, sFpairtmp, np);
  double* d_Qtmp = dev<double>(c, sQtmp, np);
  S.Q = dev<double>(c, sQ, np);
  int* d_idx = dev<int>(c, sIdx, np);
  int* d_idxs = dev<int>(c, sIdxSorted, np);
  int* d_perm = dev<int>(c, sPerm, np);

  HIP_OK(hipMemcpyAsync(d_sxyz, sxyz.data(), sxyz.size() * 8, hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(d_si, si.data(), si.size() * 4, hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(d_exps, b->exps, nprim_total * 8, hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(d_coefs, b->coefs, nprim_total * 8, hipMemcpyHostToDevice, s));
  std::vector<int> pairs(2 * static_cast<size_t>(np));
  std::copy(P.pair_s1.begin(), P.pair_s1.end(), pairs.begin());
  std::copy(P.pair_s2.begin(), P.pair_s2.end(), pairs.begin() + np);
  upload(pairs, d_pairs, s);
  upload(P.bin_off, d_binoff, s);
  upload(P.bin_npp, d_binnpp, s);
  upload(P.bin_prim, d_binprim, s);

  ShellDev sd{d_sxyz, d_si, d_si + ns, d_si + 2 * ns, d_si + 3 * ns, d_si + 4 * ns, d_exps, d_coefs};
  // step 2 (unsorted), step 3
  PairOut tmp{d_primtmp, d_primtmpT, nullptr, nullptr, d_Atmp, d_ABtmp, d_bftmp, d_atomstmp, d_fpairtmp};
  hipLaunchKernelGGL(pair_data_kernel, dim3(grid_of(np, 256)), dim3(256), 0, s, np, d_pairs,
                     d_pairs + np, static_cast<const int*>(nullptr), d_binoff, d_binnpp,
                     d_binprim, P.nbins, sd, tmp);
  HIP_OK(hipGetLastError());
  for (int bb = 0; bb < P.nbins; ++bb) {
    EriLaunch a{};
    a.bra = bin_view(P, bb, d_primtmp, d_primtmpT, d_Atmp, d_ABtmp, d_bftmp, d_atomstmp, d_fpairtmp, d_Qtmp);
    a.ket = a.bra;
    a.boys64 = c->boys64;
    a.boys32 = c->boys32;
    const int dcls = quartet_class(P.bin_cls[bb], P.bin_cls[bb]);
    const size_t per_wave = split_schwarz_ws_bytes(dcls) / kSchwarzSplitLanes;
    if (per_wave) {  // multi-pass diagonal class: workspace, waves loop over the pairs
      const int pairs_per_wave = kWave / kSchwarzSplitLanes;
      const size_t want = (static_cast<size_t>(a.bra.n) + pairs_per_wave - 1) / pairs_per_wave;
      const size_t cap = std::max<size_t>(64, c->ws_budget / per_wave);
      a.nwaves = static_cast<int>(std::min(want, cap));
      a.ws = dev<char>(c, sWsSchwarz, per_wave * a.nwaves);
    }
    launch_schwarz(P.bin_cls[bb], a, d_Qtmp + P.bin_off[bb], s);
    const std::string gm = take_guard_error();
    if (!gm.empty()) throw Fail{JK_EUNSUPPORTED, gm};
  }
  // step 4: segmented sort by Q, descending, then pair data in sorted order
  hipLaunchKernelGGL(iota_kernel, dim3(grid_of(np, 256)), dim3(256), 0, s, np, d_binoff, P.nbins, d_idx);
  size_t cub_bytes = 0;
  HIP_OK(hipcub::DeviceSegmentedRadixSort::SortPairsDescending(
      nullptr, cub_bytes, d_Qtmp, S.Q, d_idx, d_idxs, np, P.nbins, d_binoff, d_binoff + 1, 0,
      64, s));
  void* d_cub = dev<char>(c, sCub, cub_bytes);
  HIP_OK(hipcub::DeviceSegmentedRadixSort::SortPairsDescending(
      d_cub, cub_bytes, d_Qtmp, S.Q, d_idx, d_idxs, np, P.nbins, d_binoff, d_binoff + 1, 0,
      64, s));
  hipLaunchKernelGGL(local_to_global_kernel, dim3(grid_of(np, 256)), dim3(256), 0, s, np,
                     d_binoff, P.nbins, d_idxs, d_perm);
  PairOut fin{S.prim, S.primT, S.prim32, S.primT32, S.A, S.AB, S.bf, S.atoms, S.fpair};
  hipLaunchKernelGGL(pair_data_kernel, dim3(grid_of(np, 256)), dim3(256), 0, s, np, d_pairs,
                     d_pairs + np, d_perm, d_binoff, d_binnpp, d_binprim, P.nbins, sd, fin);
  HIP_OK(hipGetLastError());

  // step 5: ranges
  const int nbp = static_cast<int>(P.bp_x.size());
  const int nt = P.nt;
  std::vector<int> bpv;
  bpv.insert(bpv.end(), P.bp_x.begin(), P.bp_x.end());
  bpv.insert(bpv.end(), P.bp_y.begin(), P.bp_y.end());
  bpv.insert(bpv.end(), P.bp_t0.begin(), P.bp_t0.end());
  int* d_bp = dev<int>(c, sBp, bpv.size());
  upload(bpv, d_bp, s);
  int* d_cnt = dev<int>(c, sCnt, 2 * static_cast<size_t>(nt));
  int* d_off = dev<int>(c, sOff, 2 * static_cast<size_t>(nt));
  int* d_rng = dev<int>(c, sRng, 3 * static_cast<size_t>(nt));
  unsigned long long* d_qstat = dev<unsigned long long>(c, sQstat, 3 * static_cast<size_t>(nbp));
  hipLaunchKernelGGL(fill_kernel<unsigned long long>, dim3(grid_of(3 * nbp, 256)), dim3(256), 0, s,
                     static_cast<size_t>(3 * nbp), d_qstat);
  RangeArgs ra{nt, nbp, d_bp, d_bp + nbp, d_bp + 2 * nbp, d_binoff, S.Q, tol,
               o.precision == JK_MIXED ? o.fp32_below : 0.0, o.precision == JK_MIXED ? 1 : 0,
               d_rng, d_qstat};
  hipLaunchKernelGGL(ranges_kernel, dim3(grid_of(nt, 256)), dim3(256), 0, s, ra);
  HIP_OK(hipGetLastError());
  // step 6: quartet counts back, item size per (bin pair, precision)
  char* hp = static_cast<char*>(
      pinned(c, 3 * nbp * sizeof(unsigned long long) + 2 * (nbp + 1) * sizeof(int)));
  HIP_OK(hipMemcpyAsync(hp, d_qstat, 3 * nbp * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  const unsigned long long* qs = reinterpret_cast<const unsigned long long*>(hp);
  S.qstat.assign(qs, qs + 3 * nbp);
  std::vector<int> chunk(2 * nbp);
  S.lanes.assign(2 * nbp, 1);
  for (int bp = 0; bp < nbp; ++bp) {
    const int cls = quartet_class(P.bin_cls[P.bp_x[bp]], P.bin_cls[P.bp_y[bp]]);
    for (int pr = 0; pr < 2; ++pr) {
      const int gmax = grad ? grad_lanes(cls) : class_lanes(cls, pr);
      // the fewest lanes per quartet that still give kTargetWaves/2 wavefronts
      const unsigned long long q = S.qstat[3 * bp + pr];
      // (gradient: and whose workspace still lets kTargetWaves/2 wavefronts run)
      int lanes = gmax;
      const int mask = grad ? grad_lane_mask(cls) : class_lane_mask(cls, pr);
      const bool split = !grad && split_ws_bytes(cls, pr, 1) != 0;
      const unsigned long long want = split ? kSplitTargetWaves : kTargetWaves / 2;
      for (int g = 1; g <= gmax; g *= 2) {
        if (!(mask & (1 << g))) continue;
        const size_t ws = grad ? size_t(kWave / g) * grad_ws_elems(cls) * (pr ? 4 : 8) : 0;
        if (g < gmax && ws && c->ws_budget / ws < static_cast<size_t>(kTargetWaves / 2)) continue;
        lanes = g;
        if (q * g >= static_cast<unsigned long long>(kWave) * want) break;
      }
      S.lanes[pr * nbp + bp] = lanes;
      const int qpw = kWave / lanes;  // kets per wave step
      const unsigned long long per =
          S.qstat[3 * bp + pr] / (static_cast<unsigned long long>(qpw) * kTargetWaves);
      const unsigned long long nch =
          std::min<unsigned long long>(std::max<unsigned long long>(per, 1), kMaxItemChunks);
      chunk[pr * nbp + bp] = qpw * static_cast<int>(nch);
    }
  }
  S.chunk = chunk;
  int* d_chunk = dev<int>(c, sChunk, 2 * nbp);
  upload(chunk, d_chunk, s);
  hipLaunchKernelGGL(count_kernel, dim3(grid_of(nt, 256)), dim3(256), 0, s, nt, d_bp + 2 * nbp,
                     nbp, d_rng, d_chunk, d_cnt);
  HIP_OK(hipGetLastError());
  size_t scan_bytes = 0;
  HIP_OK(hipcub::DeviceScan::ExclusiveSum(nullptr, scan_bytes, d_cnt, d_off, 2 * nt, s));
  d_cub = dev<char>(c, sCub, std::max(scan_bytes, cub_bytes));
  HIP_OK(hipcub::DeviceScan::ExclusiveSum(d_cub, scan_bytes, d_cnt, d_off, 2 * nt, s));
  int* d_seg = dev<int>(c, sSeg, 2 * (nbp + 1));
  hipLaunchKernelGGL(segments_kernel, dim3(grid_of(2 * (nbp + 1), 256)), dim3(256), 0, s, nt,
                     nbp, d_bp + 2 * nbp, d_cnt, d_off, d_seg);
  HIP_OK(hipGetLastError());
  int* hseg = reinterpret_cast<int*>(hp + 3 * nbp * sizeof(unsigned long long));
  HIP_OK(hipMemcpyAsync(hseg, d_seg, 2 * (nbp + 1) * sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  S.seg.assign(hseg, hseg + 2 * (nbp + 1));
  const int nitems = S.seg[2 * nbp + 1];
  S.items = dev<int4>(c, sItems, std::max(nitems, 1));
  hipLaunchKernelGGL(expand_kernel, dim3(grid_of(nt, 256)), dim3(256), 0, s, nt, d_bp + 2 * nbp,
                     nbp, d_cnt, d_off, d_rng, d_chunk, S.items);
  HIP_OK(hipGetLastError());
  return S;
}

// Byte string that identifies a setup: the basis arrays element by element,
// tol and the options and context state the setup reads.
std::vector<char> setup_key(const jk_ctx* c, const jk_basis* b, double tol, const jk_opts& o,
                            bool grad) {
  std::vector<char> k;
  auto put = [&k](const void* p, size_t bytes) {
    const char* q = static_cast<const char*>(p);
    k.insert(k.end(), q, q + bytes);
  };
  int np = 0;
  for (int s = 0; s < b->n_shells; ++s) np = std::max(np, b->shell_prim0[s] + b->shell_nprim[s]);
  const int32_t head[4] = {b->n_atoms, b->n_shells, np, grad ? 1 : 0};
  put(head, sizeof(head));
  put(b->xyz, sizeof(double) * 3 * b->n_atoms);
  put(b->shell_atom, sizeof(int32_t) * b->n_shells);
  put(b->shell_l, sizeof(int32_t) * b->n_shells);
  put(b->shell_nprim, sizeof(int32_t) * b->n_shells);
  put(b->shell_prim0, sizeof(int32_t) * b->n_shells);
  put(b->exps, sizeof(double) * np);
  put(b->coefs, sizeof(double) * np);
  const double f[2] = {tol, o.precision == JK_MIXED ? o.fp32_below : 0.0};
  put(f, sizeof(f));
  put(&o.precision, sizeof(o.precision));
  put(&c->ws_budget, sizeof(c->ws_budget));
  return k;
}

// Steps 1-6, or the kept setup of an earlier call when reuse_setup is set and
// nothing it depends on has changed.
Setup get_setup(jk_ctx* c, const jk_basis* b, double tol, const jk_opts& o, hipStream_t s,
                bool grad, bool* reused) {
  *reused = false;
  if (c->noalloc) return setup(c, b, tol, o, s, grad);   // buffers of this call only
  std::vector<char> key;
  if (o.reuse_setup == 1) {
    key = setup_key(c, b, tol, o, grad);
    if (c->setup_kept && key == c->setup_key) {
      *reused = true;
      return *c->setup_kept;
    }
  }
  c->setup_kept.reset();   // the new setup overwrites the kept one's buffers
  Setup S = setup(c, b, tol, o, s, grad);
  if (o.reuse_setup == 1) {
    c->setup_kept = std::make_shared<Setup>(S);
    c->setup_key.swap(key);
  }
  return S;
}

jk_stats base_stats(const Plan& P, const Setup& S) {
  jk_stats st{};
  for (int q = 0; q < JK_NCLASS; ++q) {
    int X = 0;
    while ((X + 1) * (X + 2) / 2 <= q) ++X;
    const int Y = q - X * (X + 1) / 2;
    st.class_l[q][0] = kPairL[X][0];
    st.class_l[q][1] = kPairL[X][1];
    st.class_l[q][2] = kPairL[Y][0];
    st.class_l[q][3] = kPairL[Y][1];
  }
  st.n_pairs = P.npairs;
  const int nbp = static_cast<int>(P.bp_x.size());
  st.work_items = S.seg[2 * nbp + 1];
  for (int bp = 0; bp < nbp; ++bp) {
    const int cls = quartet_class(P.bin_cls[P.bp_x[bp]], P.bin_cls[P.bp_y[bp]]);
    st.quartets_fp64[cls] += static_cast<int64_t>(S.qstat[3 * bp]);
    st.quartets_fp32[cls] += static_cast<int64_t>(S.qstat[3 * bp + 1]);
    st.quartets_skipped += static_cast<int64_t>(S.qstat[3 * bp + 2]);
  }
  return st;
}

EriLaunch launch_args(jk_ctx* c, const Plan& P, const Setup& S, int X, int Y, int i0, int i1,
                      const double* D, double* J, double* K, int nbf, const jk_opts& o) {
  EriLaunch a{};
  a.bra = bin_view(P, X, S.prim, S.primT, S.A, S.AB, S.bf, S.atoms, S.fpair, S.Q, S.prim32, S.primT32);
  a.ket = bin_view(P, Y, S.prim, S.primT, S.A, S.AB, S.bf, S.atoms, S.fpair, S.Q, S.prim32, S.primT32);
  a.items = S.items + i0;
  a.nitems = i1 - i0;
  a.same_bin = X == Y;
  a.D = D;
  a.J = J;
  a.K = K;
  a.ncopy = 1;
  a.copy_stride = 0;
  a.n = nbf;
  a.n_dm = o.n_dm;
  a.boys64 = c->boys64;
  a.boys32 = c->boys32;
  a.boys_fp64_T = static_cast<float>(o.boys_fp64_T);
  a.att = o.omega > 0.0 ? 1 : 0;
  a.omega2 = o.omega * o.omega;
  a.num_cu = c->num_cu;
  return a;
}

struct LaunchRec {
  int cls, pr, X, Y, i0, i1, lanes;
  double cost;
};

// Launches of one build (one per bin pair and precision with work), largest
// estimated cost first, each assigned to the least-loaded context stream.
// The caller's stream forks to the context streams after setup and joins them
// before returning.
struct NoPrepare {
  void operator()(const std::vector<LaunchRec>&, const std::vector<int>&) const {}
};

void check_guard() {
  const std::string m = take_guard_error();
  if (!m.empty()) throw Fail{JK_EUNSUPPORTED, m};
}

// launch_one(rec, stream, stream index, work counter, dry): dry = check only.
template <class Fn, class Prep = NoPrepare>
void dispatch(jk_ctx* c, const Plan& P, const Setup& S, hipStream_t s, jk_stats& st, bool grad,
              bool serial, Fn&& launch_one, Prep&& prepare = Prep()) {
  const int nbp = static_cast<int>(P.bp_x.size());
  std::vector<LaunchRec> recs;
  for (int bp = 0; bp < nbp; ++bp) {
    const int X = P.bp_x[bp], Y = P.bp_y[bp];
    const int cls = quartet_class(P.bin_cls[X], P.bin_cls[Y]);
    for (int pr = 0; pr < 2; ++pr) {
      const int i0 = S.seg[pr * (nbp + 1) + bp], i1 = S.seg[pr * (nbp + 1) + bp + 1];
      if (i1 <= i0) continue;
      const double q = static_cast<double>(S.qstat[3 * bp + pr]);
      const double npp = static_cast<double>(P.bin_npp[X]) * P.bin_npp[Y];
      recs.push_back({cls, pr, X, Y, i0, i1, S.lanes[pr * nbp + bp],
                      q * npp * class_cost(cls, grad ? 1 : 0)});
    }
  }
  std::stable_sort(recs.begin(), recs.end(),
                   [](const LaunchRec& a, const LaunchRec& b) { return a.cost > b.cost; });
  // The launch with the most estimated work runs alone on the caller's stream,
  // with the whole GPU, and its timing events bracket its own run time; the
  // others follow on the internal streams (largest first, each to the least
  // loaded), where launches of different classes share the GPU.  The first
  // launch uses stream 0's workspace, which stream 0 touches only after it.
  // every launch passes the scratch guard before any of them (or any write
  // to the outputs) is enqueued
  (void)take_guard_error();
  for (size_t q = 0; q < recs.size(); ++q) launch_one(recs[q], s, 0, nullptr, true);
  check_guard();
  std::vector<int> where(recs.size(), 0);
  double load[jk_ctx::kStreams] = {};
  // serial: every launch on the caller's stream
  const size_t q0 = serial ? recs.size() : (recs.empty() ? 0 : 1);
  for (size_t q = q0; q < recs.size(); ++q) {
    int k = 0;
    for (int j = 1; j < jk_ctx::kStreams; ++j)
      if (load[j] < load[k]) k = j;
    load[k] += recs[q].cost;
    where[q] = k;
  }
  prepare(recs, where);
  // work-item counters of the persistent kernels, one per launch
  int* next = dev<int>(c, sNext, std::max<size_t>(recs.size(), 1));
  hipLaunchKernelGGL(fill_kernel<int>, dim3(grid_of(std::max<size_t>(recs.size(), 1), 256)),
                     dim3(256), 0, s, recs.size(), next);
  HIP_OK(hipGetLastError());
  for (size_t q = 0; q < recs.size(); ++q) {
    const LaunchRec& r = recs[q];
    const int k = where[q];
    if (q == q0) {
      HIP_OK(hipEventRecord(c->fork_ev, s));
      for (int j = 0; j < jk_ctx::kStreams; ++j)
        HIP_OK(hipStreamWaitEvent(c->streams[j], c->fork_ev, 0));
    }
    hipStream_t ls = q < q0 ? s : c->streams[k];
    size_t e0 = 0;
    if (c->timed) e0 = event(c, ls);
    launch_one(r, ls, k, next + q, false);
    HIP_OK(hipGetLastError());
    check_guard();
    if (c->timed) {
      event(c, ls);
      c->timed_launches.push_back({r.cls, r.pr, e0});
    }
    (r.pr ? st.launches_fp32 : st.launches_fp64)[r.cls] += 1;
  }
  if (recs.size() > q0)
    for (int k = 0; k < jk_ctx::kStreams; ++k) {
      HIP_OK(hipEventRecord(c->join_ev[k], c->streams[k]));
      HIP_OK(hipStreamWaitEvent(s, c->join_ev[k], 0));
    }
}

int check_opts(const jk_opts* o, jk_opts* out, std::string* msg) {
  jk_opts_default(out);
  if (o) *out = *o;
  if (out->precision != JK_FP64 && out->precision != JK_MIXED) { *msg = "opts.precision"; return JK_EINVAL; }
  if (!(out->fp32_below >= 0.0) || !std::isfinite(out->fp32_below)) { *msg = "opts.fp32_below"; return JK_EINVAL; }
  if (!(out->boys_fp64_T > 0.0 && out->boys_fp64_T <= 30.0)) { *msg = "opts.boys_fp64_T must be in (0, 30]"; return JK_EINVAL; }
  if (out->n_dm < 1 || out->n_dm > JK_MAX_NDM) { *msg = "opts.n_dm must be in 1..16"; return JK_EINVAL; }
  if (out->deterministic != 0 && out->deterministic != 1) { *msg = "opts.deterministic must be 0 or 1"; return JK_EINVAL; }
  if (out->timing != 0 && out->timing != 1) { *msg = "opts.timing"; return JK_EINVAL; }
  if (out->acc_copies < 0 || out->acc_copies > static_cast<int32_t>(kMaxCopies)) { *msg = "opts.acc_copies must be in 0..8"; return JK_EINVAL; }
  if (out->serial != 0 && out->serial != 1) { *msg = "opts.serial must be 0 or 1"; return JK_EINVAL; }
  if (out->reuse_setup != 0 && out->reuse_setup != 1) { *msg = "opts.reuse_setup must be 0 or 1"; return JK_EINVAL; }
  if (!(out->omega >= 0.0) || !std::isfinite(out->omega)) { *msg = "opts.omega must be finite and >= 0"; return JK_EINVAL; }
  return JK_OK;
}

}  // namespace

extern "C" {

int jk_opts_default(jk_opts* o) {
  if (!o) return JK_EINVAL;
  o->precision = JK_FP64;
  o->fp32_below = 1e-4;
  o->boys_fp64_T = 30.0;
  o->n_dm = 1;
  o->deterministic = 0;
  o->timing = 0;
  o->max_scratch_bytes = 0;
  o->acc_copies = 0;
  o->serial = 0;
  o->reuse_setup = 0;
  o->energy = nullptr;
  o->dEdD = nullptr;
  o->omega = 0.0;
  return JK_OK;
}

int jk_validate_basis(const jk_basis* basis, int32_t* n_bf_out) { return validate(basis, n_bf_out); }

int jk_ctx_create(jk_ctx** out, int device) {
  if (!out) return JK_EINVAL;
  *out = nullptr;
  jk_ctx* c = new (std::nothrow) jk_ctx;
  if (!c) return JK_ENOMEM;
  try {
    int ndev = 0;
    HIP_OK(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) throw Fail{JK_EINVAL, "no such device"};
    c->device = device;
    HIP_OK(hipSetDevice(device));
    std::vector<double> t64;
    std::vector<float> t32;
    make_boys_tables(t64, t32);
    HIP_OK(hipDeviceGetAttribute(&c->num_cu, hipDeviceAttributeMultiprocessorCount, device));
    HIP_OK(hipGetSymbolAddress(reinterpret_cast<void**>(&c->noalloc_base), HIP_SYMBOL(scratch)));
    c->noalloc_host.assign(kNoAllocHostBytes, 0);
    c->ws_budget = kWsBudget;
    if (c->num_cu < 1) c->num_cu = 1;
    HIP_OK(hipMalloc(&c->boys64, t64.size() * sizeof(double)));
    HIP_OK(hipMalloc(&c->boys32, t32.size() * sizeof(float)));
    HIP_OK(hipMemcpy(c->boys64, t64.data(), t64.size() * sizeof(double), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(c->boys32, t32.data(), t32.size() * sizeof(float), hipMemcpyHostToDevice));
    for (int k = 0; k < jk_ctx::kStreams; ++k) {
      HIP_OK(hipStreamCreateWithFlags(&c->streams[k], hipStreamNonBlocking));
      HIP_OK(hipEventCreateWithFlags(&c->join_ev[k], hipEventDisableTiming));
    }
    HIP_OK(hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming));
  } catch (const Fail& f) {
    g_create_err = f.msg;
    jk_ctx_destroy(c);
    return f.code;
  }
  *out = c;
  return JK_OK;
}

int jk_ctx_destroy(jk_ctx* c) {
  if (!c) return JK_OK;
  (void)hipSetDevice(c->device);
  for (auto& b : c->buf)
    if (b.p) (void)hipFree(b.p);
  if (c->boys64) (void)hipFree(c->boys64);
  if (c->boys32) (void)hipFree(c->boys32);
  for (auto e : c->ev_pool) (void)hipEventDestroy(e);
  if (c->host_pinned) (void)hipHostFree(c->host_pinned);
  for (int k = 0; k < jk_ctx::kStreams; ++k) {
    if (c->streams[k]) (void)hipStreamDestroy(c->streams[k]);
    if (c->join_ev[k]) (void)hipEventDestroy(c->join_ev[k]);
  }
  if (c->fork_ev) (void)hipEventDestroy(c->fork_ev);
  delete c;
  return JK_OK;
}

const char* jk_last_error(const jk_ctx* c) { return c ? c->err.c_str() : g_create_err.c_str(); }

}  // extern "C"

namespace {

int build_impl(jk_ctx* c, const jk_basis* basis, const double* D, double* J, double* K, double tol,
               const jk_opts* opts, void* hip_stream) {
  if (!c) return JK_EINVAL;
  c->err.clear();
  int32_t nbf = 0;
  int rc = validate(basis, &nbf);
  if (rc != JK_OK) { c->err = validate_msg(rc); return rc; }
  if (!D || !J || !K) { c->err = "D, J and K must be device pointers"; return JK_EINVAL; }
  if (!(tol >= 0.0) || !std::isfinite(tol)) { c->err = "tol must be finite and >= 0"; return JK_EINVAL; }
  jk_opts o;
  rc = check_opts(opts, &o, &c->err);
  if (rc != JK_OK) return rc;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  try {
    HIP_OK(hipSetDevice(c->device));
    c->scratch_limit = o.max_scratch_bytes;
    c->timed = o.timing == 1;
    c->ev_used = 0;
    c->timed_launches.clear();
    if (c->timed) c->ev_setup0 = event(c, s);
    bool reused = false;
    Setup S = get_setup(c, basis, tol, o, s, false, &reused);
    const Plan& P = S.P;
    if (c->timed) c->ev_setup1 = event(c, s);
    const size_t nn = static_cast<size_t>(nbf) * nbf;
    const size_t mat = nn * o.n_dm;   // elements of J (and of K)
    const bool det = o.deterministic == 1;
    // Atomic adds to one 64-byte line serialise at the memory side, and a small
    // J/K receives many adds per line: accumulate into up to kMaxCopies copies
    // (item % ncopy) within kAccBudget bytes, then sum them in the finalize.
    // Deterministic mode keeps two int64 words per value.
    const size_t words = det ? 2 : 1;
    int ncopy = o.acc_copies;
    if (ncopy == 0) {
      const size_t acc_budget = c->noalloc ? kNoAllocBytes / 8 : kAccBudget;
      ncopy = static_cast<int>(std::min<size_t>(kMaxCopies, acc_budget / (2 * words * mat * sizeof(double))));
      if (c->scratch_limit)
        ncopy = std::min<int>(ncopy, static_cast<int>(c->scratch_limit / 4 / (2 * words * mat * sizeof(double))));
      ncopy = std::max(ncopy, 1);
    }
    // in place (J, K are the accumulators) only with one FP64 copy
    const bool inplace = ncopy == 1 && !det;
    double* AJ = J;
    double* AK = K;
    size_t det_lo = 0;
    if (!inplace) {
      AJ = dev<double>(c, sAcc, 2 * words * mat * ncopy);
      AK = AJ + mat * ncopy;
      if (det) det_lo = 2 * mat * ncopy;   // [AJ hi][AK hi][AJ lo][AK lo]
    }
    const int fin_blocks = static_cast<int>(grid_of(nn, kFinBlock));
    double* epart = o.energy ? dev<double>(c, sEpart, static_cast<size_t>(2) * fin_blocks * o.n_dm)
                             : nullptr;

    jk_stats st = base_stats(P, S);
    st.setup_reused = reused ? 1 : 0;
    auto waves_of = [&](const LaunchRec& r) {
      const size_t per_wave = split_ws_bytes(r.cls, r.pr, r.lanes);
      if (!per_wave) return std::pair<int, size_t>(0, 0);
      const size_t cap = std::max<size_t>(64, c->ws_budget / per_wave);
      return std::pair<int, size_t>(static_cast<int>(std::min<size_t>(r.i1 - r.i0, cap)), per_wave);
    };
    void* ws[jk_ctx::kStreams] = {};
    dispatch(
        c, P, S, s, st, false, o.serial == 1,
        [&](const LaunchRec& r, hipStream_t ls, int k, int* next, bool dry) {
          EriLaunch a = launch_args(c, P, S, r.X, r.Y, r.i0, r.i1, D, AJ, AK, nbf, o);
          a.ncopy = ncopy;
          a.copy_stride = mat;
          a.det_lo = det_lo;
          a.lanes = r.lanes;
          a.next = next;
          a.ws = ws[k];
          a.nwaves = waves_of(r).first;
          a.dry = dry ? 1 : 0;
          a.rows = det ? 0 : 1;
          launch_eri(r.cls, r.pr, a, ls);
        },
        [&](const std::vector<LaunchRec>& recs, const std::vector<int>& where) {
          size_t need[jk_ctx::kStreams] = {};
          for (size_t q = 0; q < recs.size(); ++q) {
            const auto wv = waves_of(recs[q]);
            need[where[q]] = std::max(need[where[q]], wv.second * wv.first);
          }
          for (int k = 0; k < jk_ctx::kStreams; ++k)
            if (need[k]) ws[k] = dev<char>(c, static_cast<Slot>(sWs0 + k), need[k]);
          // the outputs are first written here, after every check has passed
          if (inplace) {
            hipLaunchKernelGGL(fill_kernel<double>, dim3(grid_of(mat, 256)), dim3(256), 0, s, mat, J);
            hipLaunchKernelGGL(fill_kernel<double>, dim3(grid_of(mat, 256)), dim3(256), 0, s, mat, K);
          } else {
            const size_t tot = 2 * words * mat * ncopy;
            hipLaunchKernelGGL(fill_kernel<double>, dim3(grid_of(tot, 256)), dim3(256), 0, s, tot, AJ);
          }
          HIP_OK(hipGetLastError());
        });
    FinArgs f{nbf, inplace ? 1 : ncopy, mat, det_lo, AJ, AK, D, J, K, o.dEdD, epart};
    hipLaunchKernelGGL(finalize_kernel, dim3(fin_blocks, o.n_dm), dim3(kFinBlock), 0, s, f);
    HIP_OK(hipGetLastError());
    if (o.energy) {
      hipLaunchKernelGGL(energy_kernel, dim3(o.n_dm), dim3(kFinBlock), 0, s, fin_blocks, epart, o.energy);
      HIP_OK(hipGetLastError());
    }
    if (c->timed) c->ev_end = event(c, s);
    c->stats = st;
  } catch (const Fail& f) {
    c->err = f.msg;
    return f.code;
  }
  return JK_OK;
}

}  // namespace

extern "C" {

int jk_build(jk_ctx* c, const jk_basis* basis, const double* D, double* J, double* K, double tol,
             const jk_opts* opts, void* hip_stream) {
  return build_impl(c, basis, D, J, K, tol, opts, hip_stream);
}

int jk_build_noalloc(jk_ctx* c, const jk_basis* basis, const double* D, double* J, double* K,
                     double tol, const jk_opts* opts, void* hip_stream) {
  if (!c) return JK_EINVAL;
  if (opts && opts->timing) {
    c->err = "jk_build_noalloc: timing events are created on demand; use timing = 0";
    return JK_EUNSUPPORTED;
  }
  if (!c->noalloc_base) {
    c->err = "jk_build_noalloc: no static scratch on this context's device";
    return JK_EHIP;
  }
  c->noalloc = true;
  c->noalloc_off = 0;
  c->ws_budget = kNoAllocBytes / 4;   // multi-pass workspaces take at most a quarter
  const int rc = build_impl(c, basis, D, J, K, tol, opts, hip_stream);
  c->noalloc = false;
  c->ws_budget = kWsBudget;
  return rc;
}

int jk_grad(jk_ctx* c, const jk_basis* basis, const double* D, double* dEdR, double tol,
            const jk_opts* opts, void* hip_stream) {
  if (!c) return JK_EINVAL;
  c->err.clear();
  int32_t nbf = 0;
  int rc = validate(basis, &nbf);
  if (rc != JK_OK) { c->err = validate_msg(rc); return rc; }
  if (!D || !dEdR) { c->err = "D and dEdR must be device pointers"; return JK_EINVAL; }
  if (!(tol >= 0.0) || !std::isfinite(tol)) { c->err = "tol must be finite and >= 0"; return JK_EINVAL; }
  jk_opts o;
  rc = check_opts(opts, &o, &c->err);
  if (rc != JK_OK) return rc;
  if (o.omega != 0.0) { c->err = "jk_grad: only the 1/r12 operator (opts.omega = 0)"; return JK_EUNSUPPORTED; }
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  try {
    HIP_OK(hipSetDevice(c->device));
    c->scratch_limit = o.max_scratch_bytes;
    c->timed = o.timing == 1;
    c->ev_used = 0;
    c->timed_launches.clear();
    if (c->timed) c->ev_setup0 = event(c, s);
    bool reused = false;
    Setup S = get_setup(c, basis, tol, o, s, true, &reused);
    const Plan& P = S.P;
    if (c->timed) c->ev_setup1 = event(c, s);
    const size_t ng = static_cast<size_t>(o.n_dm) * basis->n_atoms * 3;
    // deterministic mode: int64 fixed-point pairs [hi ng][lo ng], converted at the end
    const bool det = o.deterministic == 1;
    double* gacc = det ? dev<double>(c, sGradAcc, 2 * ng) : dEdR;
    jk_stats st = base_stats(P, S);
    st.setup_reused = reused ? 1 : 0;
    // gradient work arrays live in a per-stream workspace; a launch uses at most
    // kWsBudget bytes and loops over its items with a fixed number of waves
    auto waves_of = [&](const LaunchRec& r) {
      const size_t per_wave = size_t(kWave / r.lanes) * grad_ws_elems(r.cls) * (r.pr ? 4 : 8);
      const size_t cap = std::max<size_t>(64, c->ws_budget / per_wave);
      return std::pair<int, size_t>(static_cast<int>(std::min<size_t>(r.i1 - r.i0, cap)), per_wave);
    };
    void* ws[jk_ctx::kStreams] = {};
    dispatch(
        c, P, S, s, st, true, o.serial == 1,
        [&](const LaunchRec& r, hipStream_t ls, int k, int* next, bool dry) {
          GradLaunch g{};
          g.e = launch_args(c, P, S, r.X, r.Y, r.i0, r.i1, D, nullptr, nullptr, nbf, o);
          g.e.lanes = r.lanes;
          g.e.next = next;
          g.e.det_lo = det ? ng : 0;
          g.e.dry = dry ? 1 : 0;
          g.dEdR = gacc;
          g.n_atoms = basis->n_atoms;
          const size_t per = (det ? 2 : 1) * sizeof(double);
          g.lds_doubles = ng * per <= kGradLdsBytes ? static_cast<int>(ng) : 0;
          g.lds_bytes = g.lds_doubles * per;
          g.ws = ws[k];
          g.nwaves = waves_of(r).first;
          launch_grad(r.cls, r.pr, g, ls);
        },
        [&](const std::vector<LaunchRec>& recs, const std::vector<int>& where) {
          size_t need[jk_ctx::kStreams] = {};
          for (size_t q = 0; q < recs.size(); ++q) {
            const auto wv = waves_of(recs[q]);
            need[where[q]] = std::max(need[where[q]], wv.second * wv.first);
          }
          for (int k = 0; k < jk_ctx::kStreams; ++k)
            if (need[k]) ws[k] = dev<char>(c, static_cast<Slot>(sWs0 + k), need[k]);
          const size_t tot = (det ? 2 : 1) * ng;
          hipLaunchKernelGGL(fill_kernel<double>, dim3(grid_of(tot, 256)), dim3(256), 0, s, tot, gacc);
          HIP_OK(hipGetLastError());
        });
    if (det) {
      hipLaunchKernelGGL(fix_to_double_kernel, dim3(grid_of(ng, 256)), dim3(256), 0, s, ng,
                         reinterpret_cast<const unsigned long long*>(gacc), ng, dEdR);
      HIP_OK(hipGetLastError());
    }
    if (c->timed) c->ev_end = event(c, s);
    c->stats = st;
  } catch (const Fail& f) {
    c->err = f.msg;
    return f.code;
  }
  return JK_OK;
}

int jk_get_stats(jk_ctx* c, jk_stats* out) {
  if (!c || !out) return JK_EINVAL;
  jk_stats st = c->stats;
  if (c->timed && c->ev_used > 0) {
    try {
      HIP_OK(hipEventSynchronize(c->ev_pool[c->ev_end]));
      float ms = 0.f;
      HIP_OK(hipEventElapsedTime(&ms, c->ev_pool[c->ev_setup0], c->ev_pool[c->ev_setup1]));
      st.ms_setup = ms;
      HIP_OK(hipEventElapsedTime(&ms, c->ev_pool[c->ev_setup0], c->ev_pool[c->ev_end]));
      st.ms_total = ms;
      for (auto& t : c->timed_launches) {
        HIP_OK(hipEventElapsedTime(&ms, c->ev_pool[t.e0], c->ev_pool[t.e0 + 1]));
        (t.fp32 ? st.ms_kernel_fp32 : st.ms_kernel_fp64)[t.cls] += ms;
      }
    } catch (const Fail& f) {
      c->err = f.msg;
      return f.code;
    }
  }
  *out = st;
  return JK_OK;
}

}  // extern "C"
