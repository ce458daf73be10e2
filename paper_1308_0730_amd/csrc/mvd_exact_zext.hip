// The differentiated form's z passes with compile-time plans for every
// 5-smooth length (lists in mvd_exact_lengths.h).
#include "mvd_ct_passes.h"
#include "mvd_exact_lengths.h"

using namespace mvdk;

hipError_t mvd_launch_zext_exact(const LaunchArgs& a, int L, int v, int role, int conjH, float2* s_out,
                                 const float2* s_in, double2* acc, int acc_mode) {
  switch (L) {
#define X(l, t, tx, ...)                                                                                      \
  case l:                                                                                                     \
    k_zext_ct<t, tx, l, __VA_ARGS__><<<a.grid, t, 0, a.stream>>>(a.jobs, a.njobs, a.plans, a.tw, v, role, conjH, \
                                                                  s_out, s_in, acc, acc_mode);                 \
    break;
    MVD_EXACT_COL(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
