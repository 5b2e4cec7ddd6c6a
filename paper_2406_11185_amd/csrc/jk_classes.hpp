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

// Integral + digestion kernel of quartet class `cls` (0..20, bra class X >= ket
// class Y, index X(X+1)/2 + Y over pair classes ss, ps, pp, ds, dp, dd).
void launch_eri(int cls, int fp32, const EriLaunch& a, hipStream_t s);
// Workspace bytes per wavefront of the multi-pass classes (0 for the others).
size_t split_ws_bytes(int cls, int fp32, int lanes);
size_t split_schwarz_ws_bytes(int cls);
// Lanes that share one shell quartet in the class's kernel (the most it has),
// and the set of lane counts compiled for it (bit g for g lanes).
int class_lanes(int cls);
int class_lane_mask(int cls);
// Relative cost per primitive quartet of class `cls` (energy, or gradient if grad).
double class_cost(int cls, int grad);
// Cauchy-Schwarz factors of the pairs of one bin of pair class 0..5.
void launch_schwarz(int pair_class, const EriLaunch& a, double* Q, hipStream_t s);
}  // namespace jk
