// The n = 24 variant of the register-resident PCG kernel (solve_fast.h),
// in a translation unit of its own: the build's instruction-scheduling
// strategy for the n = 12 variants (solve_fast.hip) makes this one slower.
#include "solve_fast.h"

hipError_t bt_launch_fast24(const SolveArgs& a, int grid, hipStream_t s) {
  return btf::launch_ept<24, 6>(a, grid, s);
}

int bt_fast_max_grid24() { return btf::max_grid<24, 6>(); }
