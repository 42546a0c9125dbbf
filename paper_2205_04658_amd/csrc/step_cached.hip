// Plain-store instantiations of the step kernels (step_kernels.hpp), for
// launches whose two state copies fit the last-level cache; compiled apart
// from step.hip so that the two halves build in parallel.

#include "step_kernels.hpp"

namespace rlb {

hipError_t launch_tiles_cached(int Q, int sm, bool mask, int mode, int force_mode,
                               const TileArgs& a, int ty, int grid, hipStream_t s) {
  if (Q == 17) by_flags<Dir17, false>(sm, mask, mode, force_mode, ty, a, grid, s);
  else if (Q == 12) by_flags<DirP12, false>(sm, mask, mode, force_mode, ty, a, grid, s);
  else by_flags<Dir26, false>(sm, mask, mode, force_mode, ty, a, grid, s);
  return hipGetLastError();
}

}  // namespace rlb
