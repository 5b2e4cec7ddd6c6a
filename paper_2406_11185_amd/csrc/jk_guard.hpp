// Scratch (private-segment) budget of one kernel launch: a pure host-side
// decision, so that a launch whose spilled registers would need more scratch
// memory than the runtime can back is refused with an error code instead of
// reaching the GPU queue (where it ends in an out-of-resources abort).
#pragma once
#include <cstddef>

namespace jk {

// Scratch bytes the runtime backs for a launch: private bytes per lane x 64
// lanes x the wavefronts that can be resident at once -- the smaller of the
// wavefronts launched and the device's capacity for this kernel (compute units
// x workgroups per compute unit x wavefronts per workgroup).
inline size_t launch_scratch_bytes(size_t private_per_lane, size_t waves_launched, size_t num_cu,
                                   size_t blocks_per_cu, size_t waves_per_block) {
  const size_t resident = num_cu * blocks_per_cu * waves_per_block;
  const size_t waves = waves_launched < resident ? waves_launched : resident;
  return private_per_lane * 64 * waves;
}

// Largest scratch need a launch may have.  On the MI355X, launches needing up
// to ~495 MiB ran and one needing ~654 MiB ended in a queue abort; the limit
// sits between the two.
constexpr size_t kScratchBudget = size_t(576) << 20;

inline bool launch_scratch_ok(size_t need, size_t budget = kScratchBudget) { return need <= budget; }

}  // namespace jk
