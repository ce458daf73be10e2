// y passes with compile-time plans for every 5-smooth length (lists in
// mvd_exact_lengths.h).  A launch covers jobs whose ny is the plan's length.
#include "mvd_ct_passes.h"
#include "mvd_exact_lengths.h"

using namespace mvdk;

int mvd_exact_col_shape(int L, int* threads, int* lines) {
  switch (L) {
#define X(l, t, tx, ...) \
  case l:                \
    *threads = t;        \
    *lines = tx;         \
    return 1;
    MVD_EXACT_COL(X)
#undef X
    default:
      return 0;
  }
}

hipError_t mvd_launch_y_exact(const LaunchArgs& a, int L, int inv, int v) {
  switch (L) {
#define X(l, t, tx, ...)                                                                                  \
  case l:                                                                                                 \
    if (inv)                                                                                              \
      k_ypass_ct<true, t, tx, l, __VA_ARGS__><<<a.grid, t, 0, a.stream>>>(a.jobs, a.njobs, a.plans, a.tw, \
                                                                         v);                              \
    else                                                                                                  \
      k_ypass_ct<false, t, tx, l, __VA_ARGS__><<<a.grid, t, 0, a.stream>>>(a.jobs, a.njobs, a.plans,      \
                                                                          a.tw, v);                       \
    break;
    MVD_EXACT_COL(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
