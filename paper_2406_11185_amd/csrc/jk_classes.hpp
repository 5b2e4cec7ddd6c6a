// Dispatch to the generated per-class kernels (one translation unit per class).
#pragma once
#include "jk_device.hpp"

namespace jk {
// Host check run before every kernel launch (jk_host.hip): 0 if the kernel's
// scratch need fits jk_guard.hpp's budget, else nonzero, with the message kept
// for the calling entry point (take_guard_error).
int guard_launch(const void* kernel, unsigned grid_blocks, unsigned block_threads, size_t lds_bytes);

// Launch `k` with `args` after the guard; dry: run the guard only.
template <typename... P>
inline void launch_kernel(void (*k)(P...), dim3 grid, dim3 block, size_t lds, hipStream_t s,
                          bool dry, P... args) {
  if (guard_launch(reinterpret_cast<const void*>(k), grid.x, block.x, lds) != 0 || dry) return;
  void* argv[] = {static_cast<void*>(&args)...};
  (void)hipLaunchKernel(reinterpret_cast<const void*>(k), grid, block, argv, lds, s);
}

// Work-item counter back to zero between launches that share it.
template <int U>
__global__ void zero_counter_kernel(int* p) {
  if (threadIdx.x == 0) *p = U;
}

// Light class with the bra's exchange rows in LDS (eri_jk_rows_kernel): launched
// if its static and dynamic LDS fit one workgroup on the device, else false and
// nothing is launched.  The kernel attributes are read once per instantiation
// (one device per process).  Several densities (MULTI): one launch per density,
// each recomputing the integrals, since the LDS holds one density's rows; for
// classes whose integrals cost less than the per-density scatter they replace.
// ATT: the erf(omega r12)/r12 kernel.
template <class C, typename T, int NT, bool MULTI, bool ATT>
bool launch_rows(const EriLaunch& a, hipStream_t s) {
  if (a.n_dm > 1 && !MULTI) return false;
  static size_t static_bytes = 0;
  static int max_lds = -1;
  const void* k = reinterpret_cast<const void*>(&eri_jk_rows_kernel<C, T, NT, ATT>);
  if (max_lds < 0) {
    hipFuncAttributes fa{};
    int dev = 0, lds = 0;
    if (hipFuncGetAttributes(&fa, k) == hipSuccess && hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess) {
      static_bytes = fa.sharedSizeBytes;
      max_lds = lds;
    } else {
      max_lds = 0;
    }
    (void)hipGetLastError();
  }
  const size_t dyn = rows_lds_doubles<C>(a.n) * sizeof(double);
  if (static_bytes + dyn > static_cast<size_t>(max_lds)) return false;
  if (!a.dry) (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(dyn));
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, NT, dyn) != hipSuccess || nb < 1) nb = 1;
  (void)hipGetLastError();
  const dim3 grid(static_cast<unsigned>(std::min(a.nitems, nb * a.num_cu)));
  if (a.n_dm == 1) {
    launch_kernel(&eri_jk_rows_kernel<C, T, NT, ATT>, grid, dim3(NT), dyn, s, a.dry != 0, a);
    return true;
  }
  EriLaunch b = a;   // density m: D, J, K (and their accumulator copies) at m n^2
  b.n_dm = 1;
  const size_t nn = static_cast<size_t>(a.n) * a.n;
  for (int m = 0; m < a.n_dm; ++m) {
    b.D = a.D + m * nn;
    b.J = a.J + m * nn;
    b.K = a.K + m * nn;
    if (m > 0 && !a.dry) hipLaunchKernelGGL(zero_counter_kernel<0>, dim3(1), dim3(kWave), 0, s, a.next);
    launch_kernel(&eri_jk_rows_kernel<C, T, NT, ATT>, grid, dim3(NT), dyn, s, a.dry != 0, b);
    if (a.dry) break;   // the guard's answer is the same for every density
  }
  return true;
}

// Integral + digestion kernel of quartet class `cls` (0..20, bra class X >= ket
// class Y, index X(X+1)/2 + Y over pair classes ss, ps, pp, ds, dp, dd).
void launch_eri(int cls, int fp32, const EriLaunch& a, hipStream_t s);
// Workspace bytes per wavefront of the multi-pass classes (0 for the others).
size_t split_ws_bytes(int cls, int fp32, int lanes);
size_t split_schwarz_ws_bytes(int cls);
// Lanes that share one shell quartet in the class's kernel (the most it has),
// and the set of lane counts compiled for it (bit g for g lanes).
int class_lanes(int cls, int fp32);
int class_lane_mask(int cls, int fp32);
// Relative cost per primitive quartet of class `cls` (energy, or gradient if grad).
double class_cost(int cls, int grad);
// Cauchy-Schwarz factors of the pairs of one bin of pair class 0..5.
void launch_schwarz(int pair_class, const EriLaunch& a, double* Q, hipStream_t s);
}  // namespace jk
