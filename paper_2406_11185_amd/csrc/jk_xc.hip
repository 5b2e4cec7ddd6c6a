// Grid part of the exchange-correlation integration (paper, "Key Components
// Redesign and Implementation", EXC paragraph): the AO matrix on the grid with
// distance-based sparsity, then the density on the grid and the XC matrix as
// block-sparse matrix products over 32 x 32 blocks.  The functional itself (the
// potential at each point) is the caller's.
//
//   phi[mu][g]  basis function mu at grid point g.  A shell is skipped at points
//               farther from its atom than its cut-off radius, beyond which the
//               bound r^l sum_k |c_k| exp(-a_k r^2) of every component is below eps.
//   blocks      phi is stored dense in 32 x 32 blocks (32 functions x 32 points);
//               a block is zero when all its values are below eps and is then
//               left out of every product.
//   rho_g     = sum_{mu,nu} phi_mu(g) D_mu,nu phi_nu(g): per grid block G and
//               each nonzero AO block I of G, X_IG = sum_J D_IJ phi_JG over the
//               nonzero J of G, then the column sums of phi_IG * X_IG, reduced over
//               I in a fixed order.
//   V_mu,nu   = sum_g wv_g phi_mu(g) phi_nu(g): per block pair I >= J, the sum over
//               the grid blocks where both are nonzero of phi_IG diag(wv_G) phi_JG^T;
//               the upper triangle by symmetry.
//
// Layout in HBM per batch of grid points: phi [NA][GB] row-major (NA = n_ao
// rounded up to 32, GB = points of the batch rounded up to 32), the block mask
// [NA/32][GB/32] and per grid block the list of its nonzero AO blocks.  The tile
// products run on the FP64 matrix cores (their rate on this chip equals the
// vector FP64 rate, but a matrix instruction reads a quarter of the operands
// from LDS per flop that 4 x 4 register tiles would), one wavefront per 32 x 32
// output tile, operands staged in LDS.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "jk.h"

namespace {

constexpr int kB = 32;            // block edge (functions and points)
constexpr int kBatch = 16384;     // grid points per batch
constexpr int kWaveT = 64;
constexpr int kVChunks = 8;       // V: grid blocks of a batch split over this many workgroups

struct XcShell {
  double x, y, z;      // centre
  double rcut2;        // squared cut-off radius
  int l, nprim, bf0, prim0;
};

// Values of shell s at point g of the batch, into phi rows bf0.. (zero beyond the
// cut-off radius or past the batch's end).
__global__ void ao_kernel(const XcShell* __restrict__ sh, const double* __restrict__ exps,
                          const double* __restrict__ coefs, const double* __restrict__ grid,
                          int g0, int ng, int GB, double* __restrict__ phi) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  const int s = blockIdx.y;
  if (g >= GB) return;
  const XcShell S = sh[s];
  double v[6] = {0, 0, 0, 0, 0, 0};
  if (g < ng) {
    const double dx = grid[3 * static_cast<size_t>(g0 + g)] - S.x;
    const double dy = grid[3 * static_cast<size_t>(g0 + g) + 1] - S.y;
    const double dz = grid[3 * static_cast<size_t>(g0 + g) + 2] - S.z;
    const double r2 = dx * dx + dy * dy + dz * dz;
    if (r2 <= S.rcut2) {
      double rad = 0.0;
      for (int k = 0; k < S.nprim; ++k) rad += coefs[S.prim0 + k] * exp(-exps[S.prim0 + k] * r2);
      if (S.l == 0) {
        v[0] = rad;
      } else if (S.l == 1) {
        v[0] = dx * rad; v[1] = dy * rad; v[2] = dz * rad;
      } else {   // xx, xy, xz, yy, yz, zz
        v[0] = dx * dx * rad; v[1] = dx * dy * rad; v[2] = dx * dz * rad;
        v[3] = dy * dy * rad; v[4] = dy * dz * rad; v[5] = dz * dz * rad;
      }
    }
  }
  const int nc = (S.l + 1) * (S.l + 2) / 2;
  for (int c = 0; c < nc; ++c) phi[static_cast<size_t>(S.bf0 + c) * GB + g] = v[c];
}

template <int L>
__device__ __forceinline__ void ao_deriv_values(const double d[3], double R0, double R1,
                                               double v[4][6]) {
  int c = 0;
#pragma unroll
  for (int px = L; px >= 0; --px)
#pragma unroll
    for (int py = L - px; py >= 0; --py, ++c) {
      const int pw[3] = {px, py, L - px - py};
      double xp[3][3];   // xp[a][q] = d_a^q
#pragma unroll
      for (int a = 0; a < 3; ++a) { xp[a][0] = 1.0; xp[a][1] = d[a]; xp[a][2] = d[a] * d[a]; }
      const double P = xp[0][pw[0]] * xp[1][pw[1]] * xp[2][pw[2]];
      v[0][c] = P * R0;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        double dP = 0.0;
        if (pw[a] > 0) {
          dP = pw[a] * xp[a][pw[a] - 1];
#pragma unroll
          for (int b2 = 0; b2 < 3; ++b2)
            if (b2 != a) dP *= xp[b2][pw[b2]];
        }
        v[1 + a][c] = dP * R0 - 2.0 * d[a] * P * R1;
      }
    }
}

template <int L>
__device__ __forceinline__ void ao_deriv_shell(const XcShell& S, const double* __restrict__ exps,
                                              const double* __restrict__ coefs,
                                              const double* __restrict__ grid, int g0, int g,
                                              bool in, int GB, size_t mat,
                                              double* __restrict__ phi, double eps, int nGb,
                                              unsigned char* __restrict__ mask) {
  constexpr int NC = (L + 1) * (L + 2) / 2;
  double v[4][6] = {};
  if (in) {
    const double d[3] = {grid[3 * static_cast<size_t>(g0 + g)] - S.x,
                         grid[3 * static_cast<size_t>(g0 + g) + 1] - S.y,
                         grid[3 * static_cast<size_t>(g0 + g) + 2] - S.z};
    const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (r2 <= S.rcut2) {
      double R0 = 0.0, R1 = 0.0;
      for (int k = 0; k < S.nprim; ++k) {
        const double e = coefs[S.prim0 + k] * exp(-exps[S.prim0 + k] * r2);
        R0 += e;
        R1 += exps[S.prim0 + k] * e;
      }
      ao_deriv_values<L>(d, R0, R1, v);
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int c = 0; c < NC; ++c) phi[q * mat + static_cast<size_t>(S.bf0 + c) * GB + g] = v[q][c];
  // block mask (zeroed before the launch): a block with any value or derivative
  // >= eps is nonzero; every writer stores the same 1
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const double m = fmax(fmax(fabs(v[0][c]), fabs(v[1][c])), fmax(fabs(v[2][c]), fabs(v[3][c])));
    if (m >= eps) mask[static_cast<size_t>((S.bf0 + c) / 32) * nGb + g / 32] = 1;
  }
}

// Values and first derivatives of shell s at point g of the batch: phi, then
// d/dx, d/dy, d/dz phi, each [NA][GB], `mat` doubles apart.  With R0 = sum_k c_k
// e_k and R1 = sum_k c_k a_k e_k (e_k = exp(-a_k r^2)), a component with
// polynomial P (in the offsets from the centre C) has
// d phi / d c = (dP/dc) R0 - 2 (c - C_c) P R1.  The angular momentum is a
// template argument of the evaluation, so every array index is a constant.
__global__ void ao_deriv_kernel(const XcShell* __restrict__ sh, const double* __restrict__ exps,
                               const double* __restrict__ coefs, const double* __restrict__ grid,
                               int g0, int ng, int GB, size_t mat, double* __restrict__ phi,
                               double eps, unsigned char* __restrict__ mask) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  const int s = blockIdx.y;
  if (g >= GB) return;
  const XcShell S = sh[s];
  const bool in = g < ng;
  const int nGb = GB / 32;
  if (S.l == 0) ao_deriv_shell<0>(S, exps, coefs, grid, g0, g, in, GB, mat, phi, eps, nGb, mask);
  else if (S.l == 1) ao_deriv_shell<1>(S, exps, coefs, grid, g0, g, in, GB, mat, phi, eps, nGb, mask);
  else ao_deriv_shell<2>(S, exps, coefs, grid, g0, g, in, GB, mat, phi, eps, nGb, mask);
}

__global__ void fill_bytes_kernel(unsigned char* p, size_t count) {
  const size_t k = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k < count) p[k] = 0;
}

__global__ void fill_kernel(double* p, size_t count, double v) {
  const size_t k = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k < count) p[k] = v;
}

// Block mask: one wavefront per block (I = blockIdx.y, G = blockIdx.x).
__global__ __launch_bounds__(kWaveT) void mask_kernel(const double* __restrict__ phi, int GB,
                                                      double eps, unsigned char* __restrict__ mask) {
  const int G = blockIdx.x, I = blockIdx.y, t = threadIdx.x;
  double m = 0.0;
  for (int e = t; e < kB * kB; e += kWaveT) {
    const int i = e / kB, g = e % kB;
    m = fmax(m, fabs(phi[static_cast<size_t>(I * kB + i) * GB + G * kB + g]));
  }
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
  if (t == 0) mask[static_cast<size_t>(I) * gridDim.x + G] = m >= eps ? 1 : 0;
}

// Nonzero AO blocks of each grid block, in increasing order.
__global__ void list_kernel(const unsigned char* __restrict__ mask, int nIb, int nGb,
                            int* __restrict__ list, int* __restrict__ count) {
  const int G = blockIdx.x * blockDim.x + threadIdx.x;
  if (G >= nGb) return;
  int c = 0;
  for (int I = 0; I < nIb; ++I)
    if (mask[static_cast<size_t>(I) * nGb + G]) list[static_cast<size_t>(G) * nIb + c++] = I;
  count[G] = c;
}

// One 32 x 32 x 32 tile product per wavefront on the FP64 matrix cores: four
// 16 x 16 output sub-tiles, eight steps of k = 4 each.  a[k][i] (k-major) and
// b[k][j] in LDS; for one step lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16], and holds D[l / 16 + 4 r][l % 16], r = 0..3, of each
// sub-tile (layout checked on the device): acc[si][sj][r] is output row
// 16 si + l / 16 + 4 r, column 16 sj + l % 16.
// The LDS rows are padded to kLd doubles: with 64-bit elements every access then
// takes the minimum of two bank passes (an unpadded 32-double row puts the four
// k rows of one step, and the 32 rows of a transposing store, on the same banks).
typedef double dx4 __attribute__((ext_vector_type(4)));
constexpr int kLd = kB + 1;
__device__ __forceinline__ void tile_mfma(const double (*a)[kLd], const double (*b)[kLd], int lane,
                                          dx4 acc[2][2]) {
  const int l16 = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int k0 = 0; k0 < kB; k0 += 4) {
    const double a0 = a[k0 + kq][l16], a1 = a[k0 + kq][16 + l16];
    const double b0 = b[k0 + kq][l16], b1 = b[k0 + kq][16 + l16];
    acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
  }
}

// rho partials: workgroup (G = blockIdx.x, k = blockIdx.y) takes AO block I =
// list[G][k]; X_IG = sum over J in list[G] of D_IJ phi_JG; partial[G][k][g] =
// sum_i phi_IG[i][g] X_IG[i][g].
// GGA: also 2 sum_i d_c phi_IG[i][g] X_IG[i][g] for c = x, y, z (the derivative
// matrices follow phi at `mat` doubles apart), partials [4][nGb][nIb][32].
template <bool GGA>
__global__ __launch_bounds__(kWaveT) void rho_kernel(const double* __restrict__ phi, int GB,
                                                     const double* __restrict__ D, int n,
                                                     const int* __restrict__ list,
                                                     const int* __restrict__ count, int nIb,
                                                     size_t mat, double* __restrict__ partial) {
  const int G = blockIdx.x, k = blockIdx.y, t = threadIdx.x;
  const int cnt = count[G];
  if (k >= cnt) return;
  const int I = list[static_cast<size_t>(G) * nIb + k];
  __shared__ double a[kB][kLd];   // a[jj][i] = D[I*32+i][J*32+jj]
  __shared__ double b[kB][kLd];   // b[jj][g] = phi[J*32+jj][G*32+g]
  dx4 acc[2][2] = {};
  // the next J's operands are loaded into registers while the current tile
  // product runs; element u of lane t is e = t + 64 u: row e / 32, column e % 32
  constexpr int PER = kB * kB / kWaveT;
  double ra[PER], rb[PER];
  auto fetch = [&](int J) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = t + kWaveT * u, r = e / kB, c = e % kB;
      // a[r][c] = D[I*32+c][J*32+r], read as D[J*32+r][I*32+c] (D symmetric) so
      // that consecutive lanes read consecutive columns
      const int row = J * kB + r, col = I * kB + c;
      ra[u] = row < n && col < n ? D[static_cast<size_t>(row) * n + col] : 0.0;
      rb[u] = phi[static_cast<size_t>(J * kB + r) * GB + G * kB + c];
    }
  };
  fetch(list[static_cast<size_t>(G) * nIb]);
  for (int q = 0; q < cnt; ++q) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = t + kWaveT * u;
      a[e / kB][e % kB] = ra[u];
      b[e / kB][e % kB] = rb[u];
    }
    __syncthreads();
    if (q + 1 < cnt) fetch(list[static_cast<size_t>(G) * nIb + q + 1]);
    tile_mfma(a, b, t, acc);
    __syncthreads();
  }
  // column sums of phi_IG * X_IG: each lane sums its 8 rows of its two columns,
  // then the four lane groups that share a column are added
  const int l16 = t & 15, kq = t >> 4;
#pragma unroll
  for (int q = 0; q < (GGA ? 4 : 1); ++q) {
    const double* src = phi + q * mat;
    double part[2];
#pragma unroll
    for (int sj = 0; sj < 2; ++sj) {
      double v = 0.0;
#pragma unroll
      for (int si = 0; si < 2; ++si)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          v += src[static_cast<size_t>(I * kB + 16 * si + kq + 4 * r) * GB + G * kB + 16 * sj + l16] *
               acc[si][sj][r];
      v += __shfl_xor(v, 16);
      v += __shfl_xor(v, 32);
      part[sj] = q ? 2.0 * v : v;
    }
    if (kq == 0) {
      double* out = partial + ((static_cast<size_t>(q) * gridDim.x + G) * nIb + k) * kB;
      out[l16] = part[0];
      out[16 + l16] = part[1];
    }
  }
}

// rho of the batch's points: fixed-order sum of the partials of its grid block.
__global__ void rho_reduce_kernel(const double* __restrict__ partial, const int* __restrict__ count,
                                  int nIb, int ng, double* __restrict__ rho) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ng) return;
  const int G = g / kB;
  double s = 0.0;
  for (int k = 0; k < count[G]; ++k) s += partial[(static_cast<size_t>(G) * nIb + k) * kB + g % kB];
  rho[g] = s;
}

// rho and grad rho of the batch's points (GGA): fixed-order sums of the partials,
// thread (g, q): q = 0 rho, 1..3 the gradient components.
__global__ void rho_gga_reduce_kernel(const double* __restrict__ partial,
                                      const int* __restrict__ count, int nIb, int nGb, int ng,
                                      double* __restrict__ rho, double* __restrict__ grad,
                                      int n_grid) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  if (g >= ng) return;
  const int G = g / kB;
  double s = 0.0;
  for (int k = 0; k < count[G]; ++k)
    s += partial[((static_cast<size_t>(q) * nGb + G) * nIb + k) * kB + g % kB];
  if (q == 0) rho[g] = s;
  else grad[static_cast<size_t>(q - 1) * n_grid + g] = s;
}

// V_acc[z][I][J] (I >= J) += sum over the grid blocks G of chunk z with both
// blocks nonzero of phi_IG diag(wv_G) phi_JG^T; workgroup (J = blockIdx.x,
// I = blockIdx.y, z = blockIdx.z); the chunks are summed in order at the end.
// GGA: every block pair (I, J), with the second operand psi_JG = wv/2 phi_JG +
// sum_c wg_c d_c phi_JG, formed beforehand in the d/dx slot (psi_kernel); V =
// V_acc + V_acc^T then.
template <bool GGA>
__global__ __launch_bounds__(kWaveT) void vmat_kernel(const double* __restrict__ phi, int GB,
                                                      const unsigned char* __restrict__ mask,
                                                      int nGb, const double* __restrict__ wv,
                                                      const double* __restrict__ wg, int n_grid,
                                                      size_t mat, int g0, int ng, int NA,
                                                      double* __restrict__ vacc) {
  const int J = blockIdx.x, I = blockIdx.y, t = threadIdx.x;
  if (!GGA && I < J) return;
  const int per = (nGb + kVChunks - 1) / kVChunks;
  const int Gb = blockIdx.z * per, Ge = min(nGb, Gb + per);
  vacc += static_cast<size_t>(blockIdx.z) * NA * NA;
  __shared__ double a[kB][kLd];   // a[g][i] = phi[I*32+i][G*32+g]
  __shared__ double b[kB][kLd];   // b[g][j] = wv[g] phi[J*32+j][G*32+g]
  dx4 acc[2][2] = {};
  // grid blocks of this chunk where both AO blocks are nonzero, as two 64-bit
  // wavefront ballots (a chunk holds at most 128 grid blocks), taken in order;
  // the next one's operands are loaded into registers while the current tile
  // product runs
  static_assert(kBatch / kB / kVChunks <= 2 * kWaveT, "grid blocks per chunk");
  auto valid = [&](int Gh) {
    return Gh < Ge && mask[static_cast<size_t>(I) * nGb + Gh] && mask[static_cast<size_t>(J) * nGb + Gh];
  };
  unsigned long long bits0 = __ballot(valid(Gb + t)), bits1 = __ballot(valid(Gb + kWaveT + t));
  auto next_g = [&](int) {
    if (bits0) {
      const int q = __ffsll(static_cast<long long>(bits0)) - 1;
      bits0 &= bits0 - 1;
      return Gb + q;
    }
    if (bits1) {
      const int q = __ffsll(static_cast<long long>(bits1)) - 1;
      bits1 &= bits1 - 1;
      return Gb + kWaveT + q;
    }
    return Ge;
  };
  constexpr int PER = kB * kB / kWaveT;
  double ra[PER], rb[PER];
  // element u of lane t is e = t + 64 u: AO row e / 32, grid point e % 32 = t % 32
  // (the same point, so the same weight, for every u)
  auto fetch = [&](int G) {
    const int gg = G * kB + (t % kB);
    const double w = !GGA && gg < ng ? wv[g0 + gg] : 0.0;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int i = (t + kWaveT * u) / kB;
      const size_t oj = static_cast<size_t>(J * kB + i) * GB + gg;
      ra[u] = phi[static_cast<size_t>(I * kB + i) * GB + gg];
      rb[u] = GGA ? phi[mat + oj] : w * phi[oj];
    }
  };
  int G = next_g(0);
  if (G >= Ge) return;
  fetch(G);
  while (G < Ge) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = t + kWaveT * u;
      a[e % kB][e / kB] = ra[u];   // a[g][i]
      b[e % kB][e / kB] = rb[u];   // b[g][j]
    }
    __syncthreads();
    G = next_g(0);
    if (G < Ge) fetch(G);
    tile_mfma(a, b, t, acc);
    __syncthreads();
  }
  const int l16 = t & 15, kq = t >> 4;
#pragma unroll
  for (int si = 0; si < 2; ++si)
#pragma unroll
    for (int sj = 0; sj < 2; ++sj)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        vacc[static_cast<size_t>(I * kB + 16 * si + kq + 4 * r) * NA + J * kB + 16 * sj + l16] +=
            acc[si][sj][r];
}

// V from the lower triangle of the chunk sums of V_acc (mu >= nu lies in a block
// pair I >= J), summed over chunks in order, so that V is exactly symmetric.
__global__ void vmat_finish_kernel(const double* __restrict__ vacc, int NA, int n,
                                   double* __restrict__ V) {
  const size_t e = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= static_cast<size_t>(n) * n) return;
  const int mu = static_cast<int>(e / n), nu = static_cast<int>(e % n);
  const size_t o = mu >= nu ? static_cast<size_t>(mu) * NA + nu : static_cast<size_t>(nu) * NA + mu;
  double s = 0.0;
  for (int z = 0; z < kVChunks; ++z) s += vacc[static_cast<size_t>(z) * NA * NA + o];
  V[e] = s;
}

// psi = wv/2 phi + sum_c wg_c d_c phi, elementwise over the batch, written over
// the d/dx matrix (which is read first at the same element).
__global__ void psi_kernel(double* __restrict__ phi, size_t mat, int GB, const double* __restrict__ wv,
                           const double* __restrict__ wg, int n_grid, int g0, int ng) {
  const size_t e = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= mat) return;
  const int g = static_cast<int>(e % GB);
  double v = 0.0;
  if (g < ng) {
    const size_t p = static_cast<size_t>(g0) + g;
    v = 0.5 * wv[p] * phi[e] + wg[p] * phi[mat + e] + wg[n_grid + p] * phi[2 * mat + e] +
        wg[2 * static_cast<size_t>(n_grid) + p] * phi[3 * mat + e];
  }
  phi[mat + e] = v;
}

// GGA: V = S + S^T with S the chunk sums of V_acc over every block pair.
__global__ void vmat_gga_finish_kernel(const double* __restrict__ vacc, int NA, int n,
                                       double* __restrict__ V) {
  const size_t e = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= static_cast<size_t>(n) * n) return;
  const int mu = static_cast<int>(e / n), nu = static_cast<int>(e % n);
  double a = 0.0, b = 0.0;   // the two chunk sums, added last: V exactly symmetric
  for (int z = 0; z < kVChunks; ++z) {
    const double* vz = vacc + static_cast<size_t>(z) * NA * NA;
    a += vz[static_cast<size_t>(mu) * NA + nu];
    b += vz[static_cast<size_t>(nu) * NA + mu];
  }
  V[e] = a + b;
}

// Cut-off radius of a shell: the largest r with r^l sum_k |c_k| exp(-a_k r^2) >= eps
// (past the last maximum of every term, the bound only decreases).
// With derivatives (deriv), the bound also covers every first derivative:
// sum_k |c_k| (l r^(l-1) + 2 a_k r^(l+1)) exp(-a_k r^2).
double cutoff_radius(int l, const double* a, const double* c, int np, double eps, bool deriv) {
  auto f = [&](double r) {
    double s = 0.0, sd = 0.0;
    for (int k = 0; k < np; ++k) {
      const double e = std::fabs(c[k]) * std::exp(-a[k] * r * r);
      s += e;
      sd += e * ((l > 0 ? l * std::pow(r, l - 1) : 0.0) + 2.0 * a[k] * std::pow(r, l + 1));
    }
    return deriv ? std::max(std::pow(r, l) * s, sd) : std::pow(r, l) * s;
  };
  double lo = 0.0;   // past every term's last maximum (l + 1 covers the derivatives)
  for (int k = 0; k < np; ++k) lo = std::max(lo, std::sqrt(0.5 * (deriv ? l + 1 : l) / a[k]));
  double hi = std::max(2.0 * lo, 1.0);
  while (f(hi) >= eps && hi < 1e4) hi *= 2.0;
  if (f(lo) < eps) return lo;
  for (int it = 0; it < 100; ++it) {
    const double mid = 0.5 * (lo + hi);
    (f(mid) >= eps ? lo : hi) = mid;
  }
  return hi;
}

// Everything a call needs on the device, freed on the stream at the end.
struct XcCall {
  hipStream_t s = nullptr;
  std::vector<void*> bufs;
  int n = 0, NA = 0, nIb = 0, ns = 0;
  bool gga = false;   // phi and its three derivatives
  XcShell* shells = nullptr;
  double *exps = nullptr, *coefs = nullptr, *phi = nullptr;
  unsigned char* mask = nullptr;
  int *list = nullptr, *count = nullptr;

  template <typename T>
  bool alloc(T** p, size_t bytes) {
    void* q = nullptr;
    if (hipMallocAsync(&q, std::max<size_t>(bytes, 8), s) != hipSuccess) return false;
    bufs.push_back(q);
    *p = static_cast<T*>(q);
    return true;
  }
  ~XcCall() {
    for (void* p : bufs) (void)hipFreeAsync(p, s);
  }
};

int xc_setup(XcCall& x, const jk_basis* b, double eps, bool gga) {
  int32_t n = 0;
  const int rc = jk_validate_basis(b, &n);
  if (rc != JK_OK) return rc;
  x.n = n;
  x.NA = (n + kB - 1) / kB * kB;
  x.nIb = x.NA / kB;
  x.ns = b->n_shells;
  x.gga = gga;
  if (x.ns > 65535) return JK_EUNSUPPORTED;
  std::vector<XcShell> hs(x.ns);
  int np = 0, bf = 0;
  for (int s = 0; s < x.ns; ++s) np = std::max(np, b->shell_prim0[s] + b->shell_nprim[s]);
  for (int s = 0; s < x.ns; ++s) {
    const int l = b->shell_l[s], a = b->shell_atom[s];
    const double r = cutoff_radius(l, b->exps + b->shell_prim0[s], b->coefs + b->shell_prim0[s],
                                   b->shell_nprim[s], eps, gga);
    hs[s] = XcShell{b->xyz[3 * a], b->xyz[3 * a + 1], b->xyz[3 * a + 2], r * r, l,
                    b->shell_nprim[s], bf, b->shell_prim0[s]};
    bf += (l + 1) * (l + 2) / 2;
  }
  const int nGb = kBatch / kB;
  if (!x.alloc(&x.shells, hs.size() * sizeof(XcShell)) || !x.alloc(&x.exps, np * 8) ||
      !x.alloc(&x.coefs, np * 8) ||
      !x.alloc(&x.phi, static_cast<size_t>(gga ? 4 : 1) * x.NA * kBatch * 8) ||
      !x.alloc(&x.mask, static_cast<size_t>(x.nIb) * nGb) ||
      !x.alloc(&x.list, static_cast<size_t>(nGb) * x.nIb * 4) || !x.alloc(&x.count, nGb * 4))
    return JK_ENOMEM;
  if (hipMemcpyAsync(x.shells, hs.data(), hs.size() * sizeof(XcShell), hipMemcpyHostToDevice, x.s) != hipSuccess ||
      hipMemcpyAsync(x.exps, b->exps, np * 8, hipMemcpyHostToDevice, x.s) != hipSuccess ||
      hipMemcpyAsync(x.coefs, b->coefs, np * 8, hipMemcpyHostToDevice, x.s) != hipSuccess ||
      hipStreamSynchronize(x.s) != hipSuccess)   // the host tables go out of scope
    return JK_EHIP;
  return JK_OK;
}

// AO values, mask and lists of one batch (points g0 .. g0+ng-1).
void xc_batch(XcCall& x, const double* grid, int g0, int ng, int GB, double eps) {
  const int nGb = GB / kB;
  const size_t mat = static_cast<size_t>(x.NA) * GB;
  // padding rows (functions n .. NA-1) are zero at this batch's row stride
  const size_t pad = static_cast<size_t>(x.NA - x.n) * GB;
  for (int q = 0; q < (x.gga ? 4 : 1); ++q)
    if (pad) hipLaunchKernelGGL(fill_kernel, dim3((pad + 255) / 256), dim3(256), 0, x.s,
                                x.phi + q * mat + static_cast<size_t>(x.n) * GB, pad, 0.0);
  if (x.gga) {
    const size_t nm = static_cast<size_t>(x.nIb) * nGb;
    hipLaunchKernelGGL(fill_bytes_kernel, dim3((nm + 255) / 256), dim3(256), 0, x.s, x.mask, nm);
    hipLaunchKernelGGL(ao_deriv_kernel, dim3((GB + 255) / 256, x.ns), dim3(256), 0, x.s, x.shells,
                       x.exps, x.coefs, grid, g0, ng, GB, mat, x.phi, eps, x.mask);
  } else {
    hipLaunchKernelGGL(ao_kernel, dim3((GB + 255) / 256, x.ns), dim3(256), 0, x.s, x.shells, x.exps,
                       x.coefs, grid, g0, ng, GB, x.phi);
    hipLaunchKernelGGL(mask_kernel, dim3(nGb, x.nIb), dim3(kWaveT), 0, x.s, x.phi, GB, eps, x.mask);
  }
  hipLaunchKernelGGL(list_kernel, dim3((nGb + 63) / 64), dim3(64), 0, x.s, x.mask, x.nIb, nGb,
                     x.list, x.count);
}

bool check_eps(double eps) { return eps > 0.0 && eps < 1.0 && std::isfinite(eps); }

// Tile products of a batch into *tiles: sum over grid blocks of c^2 (rho, per
// density) or c (c + 1) / 2 (V, block pairs I >= J), c = nonzero AO blocks.
__global__ void tiles_kernel(const int* __restrict__ count, int nGb, int pairs, int mult,
                             unsigned long long* tiles) {
  const int G = blockIdx.x * blockDim.x + threadIdx.x;
  if (G >= nGb) return;
  const unsigned long long c = static_cast<unsigned long long>(count[G]);
  atomicAdd(tiles, (pairs ? c * (c + 1) / 2 : c * c) * static_cast<unsigned long long>(mult));
}

}  // namespace

extern "C" {

int jk_xc_rho(const jk_basis* basis, const double* grid, int32_t n_grid, const double* D,
              int32_t n_dm, double eps, double* rho, int64_t* tiles, void* hip_stream) {
  if (!grid || !D || !rho || n_grid < 1 || n_dm < 1 || n_dm > JK_MAX_NDM || !check_eps(eps))
    return JK_EINVAL;
  XcCall x;
  x.s = static_cast<hipStream_t>(hip_stream);
  int rc = xc_setup(x, basis, eps, false);
  if (rc != JK_OK) return rc;
  double* partial = nullptr;
  if (!x.alloc(&partial, static_cast<size_t>(kBatch / kB) * x.nIb * kB * 8)) return JK_ENOMEM;
  for (int g0 = 0; g0 < n_grid; g0 += kBatch) {
    const int ng = std::min(kBatch, n_grid - g0);
    const int GB = (ng + kB - 1) / kB * kB, nGb = GB / kB;
    xc_batch(x, grid, g0, ng, GB, eps);
    if (tiles)
      hipLaunchKernelGGL(tiles_kernel, dim3((nGb + 255) / 256), dim3(256), 0, x.s, x.count, nGb, 0,
                         n_dm, reinterpret_cast<unsigned long long*>(tiles));
    for (int m = 0; m < n_dm; ++m) {
      const double* Dm = D + static_cast<size_t>(m) * x.n * x.n;
      hipLaunchKernelGGL(rho_kernel<false>, dim3(nGb, x.nIb), dim3(kWaveT), 0, x.s, x.phi, GB, Dm,
                         x.n, x.list, x.count, x.nIb, size_t(0), partial);
      hipLaunchKernelGGL(rho_reduce_kernel, dim3((ng + 255) / 256), dim3(256), 0, x.s, partial,
                         x.count, x.nIb, ng, rho + static_cast<size_t>(m) * n_grid + g0);
    }
  }
  return hipGetLastError() == hipSuccess ? JK_OK : JK_EHIP;
}

int jk_xc_vmat(const jk_basis* basis, const double* grid, int32_t n_grid, const double* wv,
               double eps, double* V, int64_t* tiles, void* hip_stream) {
  if (!grid || !wv || !V || n_grid < 1 || !check_eps(eps)) return JK_EINVAL;
  XcCall x;
  x.s = static_cast<hipStream_t>(hip_stream);
  int rc = xc_setup(x, basis, eps, false);
  if (rc != JK_OK) return rc;
  double* vacc = nullptr;
  const size_t na2 = static_cast<size_t>(x.NA) * x.NA * kVChunks;
  if (!x.alloc(&vacc, na2 * 8)) return JK_ENOMEM;
  hipLaunchKernelGGL(fill_kernel, dim3((na2 + 255) / 256), dim3(256), 0, x.s, vacc, na2, 0.0);
  for (int g0 = 0; g0 < n_grid; g0 += kBatch) {
    const int ng = std::min(kBatch, n_grid - g0);
    const int GB = (ng + kB - 1) / kB * kB, nGb = GB / kB;
    xc_batch(x, grid, g0, ng, GB, eps);
    if (tiles)
      hipLaunchKernelGGL(tiles_kernel, dim3((nGb + 255) / 256), dim3(256), 0, x.s, x.count, nGb, 1,
                         1, reinterpret_cast<unsigned long long*>(tiles));
    hipLaunchKernelGGL(vmat_kernel<false>, dim3(x.nIb, x.nIb, kVChunks), dim3(kWaveT), 0, x.s,
                       x.phi, GB, x.mask, nGb, wv, static_cast<const double*>(nullptr), n_grid,
                       size_t(0), g0, ng, x.NA, vacc);
  }
  const size_t nn = static_cast<size_t>(x.n) * x.n;
  hipLaunchKernelGGL(vmat_finish_kernel, dim3((nn + 255) / 256), dim3(256), 0, x.s, vacc, x.NA,
                     x.n, V);
  return hipGetLastError() == hipSuccess ? JK_OK : JK_EHIP;
}

int jk_xc_rho_gga(const jk_basis* basis, const double* grid, int32_t n_grid, const double* D,
                  int32_t n_dm, double eps, double* rho, double* grad_rho, void* hip_stream) {
  if (!grid || !D || !rho || !grad_rho || n_grid < 1 || n_dm < 1 || n_dm > JK_MAX_NDM ||
      !check_eps(eps))
    return JK_EINVAL;
  XcCall x;
  x.s = static_cast<hipStream_t>(hip_stream);
  int rc = xc_setup(x, basis, eps, true);
  if (rc != JK_OK) return rc;
  double* partial = nullptr;
  if (!x.alloc(&partial, static_cast<size_t>(4) * (kBatch / kB) * x.nIb * kB * 8)) return JK_ENOMEM;
  for (int g0 = 0; g0 < n_grid; g0 += kBatch) {
    const int ng = std::min(kBatch, n_grid - g0);
    const int GB = (ng + kB - 1) / kB * kB, nGb = GB / kB;
    const size_t mat = static_cast<size_t>(x.NA) * GB;
    xc_batch(x, grid, g0, ng, GB, eps);
    for (int m = 0; m < n_dm; ++m) {
      const double* Dm = D + static_cast<size_t>(m) * x.n * x.n;
      hipLaunchKernelGGL(rho_kernel<true>, dim3(nGb, x.nIb), dim3(kWaveT), 0, x.s, x.phi, GB, Dm,
                         x.n, x.list, x.count, x.nIb, mat, partial);
      hipLaunchKernelGGL(rho_gga_reduce_kernel, dim3((ng + 255) / 256, 4), dim3(256), 0, x.s,
                         partial, x.count, x.nIb, nGb, ng,
                         rho + static_cast<size_t>(m) * n_grid + g0,
                         grad_rho + static_cast<size_t>(m) * 3 * n_grid + g0, n_grid);
    }
  }
  return hipGetLastError() == hipSuccess ? JK_OK : JK_EHIP;
}

int jk_xc_vmat_gga(const jk_basis* basis, const double* grid, int32_t n_grid, const double* wv,
                   const double* wg, double eps, double* V, void* hip_stream) {
  if (!grid || !wv || !wg || !V || n_grid < 1 || !check_eps(eps)) return JK_EINVAL;
  XcCall x;
  x.s = static_cast<hipStream_t>(hip_stream);
  int rc = xc_setup(x, basis, eps, true);
  if (rc != JK_OK) return rc;
  double* vacc = nullptr;
  const size_t na2 = static_cast<size_t>(x.NA) * x.NA * kVChunks;
  if (!x.alloc(&vacc, na2 * 8)) return JK_ENOMEM;
  hipLaunchKernelGGL(fill_kernel, dim3((na2 + 255) / 256), dim3(256), 0, x.s, vacc, na2, 0.0);
  for (int g0 = 0; g0 < n_grid; g0 += kBatch) {
    const int ng = std::min(kBatch, n_grid - g0);
    const int GB = (ng + kB - 1) / kB * kB, nGb = GB / kB;
    const size_t mat = static_cast<size_t>(x.NA) * GB;
    xc_batch(x, grid, g0, ng, GB, eps);
    hipLaunchKernelGGL(psi_kernel, dim3((mat + 255) / 256), dim3(256), 0, x.s, x.phi, mat, GB, wv,
                       wg, n_grid, g0, ng);
    hipLaunchKernelGGL(vmat_kernel<true>, dim3(x.nIb, x.nIb, kVChunks), dim3(kWaveT), 0, x.s,
                       x.phi, GB, x.mask, nGb, wv, wg, n_grid, mat, g0, ng, x.NA, vacc);
  }
  const size_t nn = static_cast<size_t>(x.n) * x.n;
  hipLaunchKernelGGL(vmat_gga_finish_kernel, dim3((nn + 255) / 256), dim3(256), 0, x.s, vacc, x.NA,
                     x.n, V);
  return hipGetLastError() == hipSuccess ? JK_OK : JK_EHIP;
}

}  // extern "C"
