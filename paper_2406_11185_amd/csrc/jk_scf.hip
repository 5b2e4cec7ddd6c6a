// The SCF steps on either side of the J/K build, on the GPU (paper, "Key
// Components Redesign and Implementation", SCF-iteration paragraph, which puts
// the Fock diagonalisation and the DIIS matrix work on the GPU too, with the
// vendor solver and BLAS; "DFT Calculation Flow" for the steps themselves).
//
//   jk_scf_diag: F C = S C diag(eps) (rocSOLVER's generalised symmetric-definite
//     divide-and-conquer solver) and the closed-shell density D = 2 C_occ C_occ^T
//     (one rocBLAS GEMM).
//   jk_scf_diis: Pulay's extrapolation over a ring of the last `depth` (F, D)
//     pairs: error e = F D S - S D F (two GEMMs and a transposed difference); the
//     Gram matrix B_ij = <e_i, e_j> of the stored errors is kept on the device and
//     only the new error's row is formed per call (m dot products of length n^2 in
//     one pass over the stored errors, block partial sums reduced in a fixed
//     order); the bordered system [B -1; -1^T 0] [c; l] = [0; -1] (rocSOLVER, on
//     the device); F_out = sum c_i F_i (one GEMV over the stored Fock matrices).
//
// The matrices are symmetric, so their row-major storage equals the
// column-major storage the libraries assume.  Eigenvectors come back as the
// columns of a column-major matrix, i.e. the rows of the row-major C: row j of C
// is orbital j.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <new>

#include "jk.h"

struct jk_scf {
  int device = 0;
  int n = 0, depth = 0;
  rocblas_handle blas = nullptr;
  double* A = nullptr;      // n^2: F copy, eigenvectors on exit
  double* B = nullptr;      // n^2: S copy (Cholesky factor on exit); DIIS: F D
  double* E = nullptr;      // n: off-diagonal work of the eigensolver; DIIS: F D S (n^2)
  double* Fh = nullptr;     // depth n^2: stored Fock matrices
  double* Eh = nullptr;     // depth n^2: stored errors
  double* G = nullptr;      // (depth+1)^2 bordered system, then depth^2 Gram matrix,
                            // then kDotBlocks x depth dot-product partials
  double* rhs = nullptr;    // depth+1: right-hand side, then [c; l]
  int* info = nullptr;      // 1
  int* ipiv = nullptr;      // depth+1
  int count = 0;            // pairs pushed since the last reset
};

namespace {

bool blas_ok(rocblas_status s) { return s == rocblas_status_success; }

constexpr int kDotBlocks = 512;
constexpr int kDotThreads = 256;

// Partial dot products of the new error e with the m stored errors: block b
// sums its grid-stride share of the n^2 elements, part[b][j]; pmax[b] = the
// largest |e| of that share.
__global__ __launch_bounds__(kDotThreads) void diis_dots_kernel(const double* __restrict__ e,
                                                                const double* __restrict__ Eh,
                                                                size_t nn, int m,
                                                                double* __restrict__ part,
                                                                double* __restrict__ pmax) {
  __shared__ double red[kDotThreads], rmax[kDotThreads];
  for (int j = 0; j < m; ++j) {
    const double* ej = Eh + static_cast<size_t>(j) * nn;
    double s = 0.0, mx = 0.0;
    for (size_t k = static_cast<size_t>(blockIdx.x) * kDotThreads + threadIdx.x; k < nn;
         k += static_cast<size_t>(kDotBlocks) * kDotThreads) {
      s += e[k] * ej[k];
      if (j == 0) mx = fmax(mx, fabs(e[k]));
    }
    red[threadIdx.x] = s;
    rmax[threadIdx.x] = mx;
    __syncthreads();
    for (int w = kDotThreads / 2; w > 0; w >>= 1) {
      if (threadIdx.x < w) {
        red[threadIdx.x] += red[threadIdx.x + w];
        rmax[threadIdx.x] = fmax(rmax[threadIdx.x], rmax[threadIdx.x + w]);
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      part[static_cast<size_t>(blockIdx.x) * m + j] = red[0];
      if (j == 0) pmax[blockIdx.x] = rmax[0];
    }
    __syncthreads();
  }
}

// Row and column `slot` of the Gram matrix (leading dimension depth) from the
// partials, summed over blocks in a fixed order; *err_out = max |e| if wanted.
__global__ void diis_gram_kernel(const double* __restrict__ part, const double* __restrict__ pmax,
                                 int m, int slot, int depth, double* __restrict__ gram,
                                 double* err_out) {
  const int j = threadIdx.x;
  if (j == 0 && err_out) {
    double mx = 0.0;
    for (int b = 0; b < kDotBlocks; ++b) mx = fmax(mx, pmax[b]);
    *err_out = mx;
  }
  if (j >= m) return;
  double s = 0.0;
  for (int b = 0; b < kDotBlocks; ++b) s += part[static_cast<size_t>(b) * m + j];
  gram[static_cast<size_t>(slot) * depth + j] = s;
  gram[static_cast<size_t>(j) * depth + slot] = s;
}

// Bordered DIIS system from the leading m x m of the Gram matrix (leading
// dimension depth).
__global__ void diis_border_kernel(const double* __restrict__ gram, int m, int depth,
                                   double* __restrict__ G, double* __restrict__ rhs) {
  const int t = threadIdx.x;
  const int M = m + 1;
  for (int k = t; k < M * M; k += blockDim.x) {
    const int i = k % M, j = k / M;   // column-major (i row, j column)
    double v;
    if (i < m && j < m) v = gram[static_cast<size_t>(j) * depth + i];
    else if (i == m && j == m) v = 0.0;
    else v = -1.0;
    G[k] = v;
  }
  for (int k = t; k < M; k += blockDim.x) rhs[k] = k == m ? -1.0 : 0.0;
}

__global__ void fill_zero_kernel(double* p, size_t count) {
  const size_t k = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k < count) p[k] = 0.0;
}

void release(jk_scf* h) {
  if (!h) return;
  if (h->blas) rocblas_destroy_handle(h->blas);
  for (void* p : {static_cast<void*>(h->A), static_cast<void*>(h->B), static_cast<void*>(h->E),
                  static_cast<void*>(h->Fh), static_cast<void*>(h->Eh), static_cast<void*>(h->G),
                  static_cast<void*>(h->rhs), static_cast<void*>(h->info),
                  static_cast<void*>(h->ipiv)})
    if (p) (void)hipFree(p);
  delete h;
}

}  // namespace

extern "C" {

int jk_scf_create(jk_scf** out, int device, int32_t n, int32_t depth) {
  if (!out) return JK_EINVAL;
  *out = nullptr;
  if (n < 1 || n > 46340 || depth < 1 || depth > 32) return JK_EINVAL;   // n^2 < 2^31
  jk_scf* h = new (std::nothrow) jk_scf;
  if (!h) return JK_ENOMEM;
  h->device = device;
  h->n = n;
  h->depth = depth;
  const size_t nn = static_cast<size_t>(n) * n;
  if (hipSetDevice(device) != hipSuccess) { release(h); return JK_EHIP; }
  if (!blas_ok(rocblas_create_handle(&h->blas))) { h->blas = nullptr; release(h); return JK_EHIP; }
  const bool ok = hipMalloc(&h->A, nn * 8) == hipSuccess && hipMalloc(&h->B, nn * 8) == hipSuccess &&
                  hipMalloc(&h->E, nn * 8) == hipSuccess &&
                  hipMalloc(&h->Fh, depth * nn * 8) == hipSuccess &&
                  hipMalloc(&h->Eh, depth * nn * 8) == hipSuccess &&
                  hipMalloc(&h->G, (static_cast<size_t>(depth + 1) * (depth + 1) + depth * depth +
                                    static_cast<size_t>(kDotBlocks) * (depth + 1)) * 8) == hipSuccess &&
                  hipMalloc(&h->rhs, static_cast<size_t>(depth + 1) * 8) == hipSuccess &&
                  hipMalloc(&h->info, sizeof(int)) == hipSuccess &&
                  hipMalloc(&h->ipiv, static_cast<size_t>(depth + 1) * sizeof(int)) == hipSuccess;
  if (!ok) { release(h); return JK_ENOMEM; }
  *out = h;
  return JK_OK;
}

int jk_scf_destroy(jk_scf* h) {
  if (h) {
    (void)hipSetDevice(h->device);
    release(h);
  }
  return JK_OK;
}

int jk_scf_diis_reset(jk_scf* h) {
  if (!h) return JK_EINVAL;
  h->count = 0;
  return JK_OK;
}

int jk_scf_diag(jk_scf* h, const double* F, const double* S, int32_t n_occ, double* C, double* eps,
                double* D, void* hip_stream) {
  if (!h || !F || !S || !eps || n_occ < 0 || n_occ > h->n) return JK_EINVAL;
  const int n = h->n;
  const size_t nn = static_cast<size_t>(n) * n;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if (hipSetDevice(h->device) != hipSuccess) return JK_EHIP;
  if (!blas_ok(rocblas_set_stream(h->blas, s))) return JK_EHIP;
  if (hipMemcpyAsync(h->A, F, nn * 8, hipMemcpyDeviceToDevice, s) != hipSuccess ||
      hipMemcpyAsync(h->B, S, nn * 8, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return JK_EHIP;
  if (!blas_ok(rocsolver_dsygvd(h->blas, rocblas_eform_ax, rocblas_evect_original,
                                rocblas_fill_upper, n, h->A, n, h->B, n, eps, h->E, h->info)))
    return JK_EHIP;
  int info = 0;
  if (hipMemcpyAsync(&info, h->info, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return JK_EHIP;
  if (info != 0) return JK_EINVAL;   // S not positive definite (or no convergence)
  if (C && hipMemcpyAsync(C, h->A, nn * 8, hipMemcpyDeviceToDevice, s) != hipSuccess) return JK_EHIP;
  if (D) {
    const double two = 2.0, zero = 0.0;
    if (n_occ == 0) {
      hipLaunchKernelGGL(fill_zero_kernel, dim3((nn + 255) / 256), dim3(256), 0, s, D, nn);
    } else if (!blas_ok(rocblas_dgemm(h->blas, rocblas_operation_none, rocblas_operation_transpose,
                                      n, n, n_occ, &two, h->A, n, h->A, n, &zero, D, n))) {
      return JK_EHIP;
    }
  }
  return hipGetLastError() == hipSuccess ? JK_OK : JK_EHIP;
}

int jk_scf_diis(jk_scf* h, const double* F, const double* D, const double* S, double* F_out,
                double* err_out, void* hip_stream) {
  if (!h || !F || !D || !S || !F_out) return JK_EINVAL;
  const int n = h->n;
  const size_t nn = static_cast<size_t>(n) * n;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if (hipSetDevice(h->device) != hipSuccess) return JK_EHIP;
  if (!blas_ok(rocblas_set_stream(h->blas, s))) return JK_EHIP;
  const int slot = h->count % h->depth;
  const int m = std::min(h->count + 1, h->depth);
  double* Fs = h->Fh + slot * nn;
  double* Es = h->Eh + slot * nn;
  const double one = 1.0, zero = 0.0, mone = -1.0;
  // e = F D S - (F D S)^T  (= F D S - S D F for symmetric F, D, S)
  if (!blas_ok(rocblas_dgemm(h->blas, rocblas_operation_none, rocblas_operation_none, n, n, n, &one,
                             F, n, D, n, &zero, h->B, n)) ||
      !blas_ok(rocblas_dgemm(h->blas, rocblas_operation_none, rocblas_operation_none, n, n, n, &one,
                             h->B, n, S, n, &zero, h->E, n)) ||
      !blas_ok(rocblas_dgeam(h->blas, rocblas_operation_none, rocblas_operation_transpose, n, n,
                             &one, h->E, n, &mone, h->E, n, Es, n)))
    return JK_EHIP;
  if (hipMemcpyAsync(Fs, F, nn * 8, hipMemcpyDeviceToDevice, s) != hipSuccess) return JK_EHIP;
  // the new error's row of the Gram matrix (slots 0..m-1 are the live ones)
  double* gram = h->G + static_cast<size_t>(h->depth + 1) * (h->depth + 1);
  double* part = gram + static_cast<size_t>(h->depth) * h->depth;
  double* pmax = part + static_cast<size_t>(kDotBlocks) * h->depth;
  const int ldk = static_cast<int>(nn);
  hipLaunchKernelGGL(diis_dots_kernel, dim3(kDotBlocks), dim3(kDotThreads), 0, s, Es, h->Eh, nn,
                     m, part, pmax);
  hipLaunchKernelGGL(diis_gram_kernel, dim3(1), dim3(64), 0, s, part, pmax, m, slot, h->depth, gram,
                     err_out);
  hipLaunchKernelGGL(diis_border_kernel, dim3(1), dim3(256), 0, s, gram, m, h->depth, h->G,
                     h->rhs);
  if (!blas_ok(rocsolver_dgesv(h->blas, m + 1, 1, h->G, m + 1, h->ipiv, h->rhs, m + 1, h->info)))
    return JK_EHIP;
  int info = 0;
  if (hipMemcpyAsync(&info, h->info, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return JK_EHIP;
  h->count += 1;
  if (info != 0) {   // singular system: no extrapolation, the latest F
    return hipMemcpyAsync(F_out, F, nn * 8, hipMemcpyDeviceToDevice, s) == hipSuccess ? JK_OK
                                                                                      : JK_EHIP;
  }
  if (!blas_ok(rocblas_dgemv(h->blas, rocblas_operation_none, ldk, m, &one, h->Fh, ldk, h->rhs, 1,
                             &zero, F_out, 1)))
    return JK_EHIP;
  return hipGetLastError() == hipSuccess ? JK_OK : JK_EHIP;
}

}  // extern "C"
