// z passes (with the spectral product) with compile-time plans for every
// 5-smooth length (lists in mvd_exact_lengths.h).  A launch covers jobs whose
// nz is the plan's length.
#include "mvd_ct_passes.h"
#include "mvd_exact_lengths.h"

using namespace mvdk;

hipError_t mvd_launch_z_exact(const LaunchArgs& a, int L, int v, int role, int conjH, int src_saved) {
  switch (L) {
#define X(l, t, tx, ...)                                                                            \
  case l:                                                                                           \
    k_zconv_ct<t, tx, l, __VA_ARGS__><<<a.grid, t, 0, a.stream>>>(a.jobs, a.njobs, a.plans, a.tw, v, \
                                                                   role, conjH, src_saved);         \
    break;
    MVD_EXACT_COL(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
