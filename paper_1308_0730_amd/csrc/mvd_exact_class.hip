// Column passes over blocks of several lengths: one launch per length class
// (lists in mvd_exact_lengths.h); each workgroup runs the compile-time plan
// of its job's length.
#include "mvd_ct_passes.h"
#include "mvd_exact_lengths.h"

using namespace mvdk;

int mvd_col_class(int L) {
  switch (L) {
#define X(l, c) \
  case l:       \
    return c;
    MVD_COL_CLASS_OF(X)
#undef X
    default:
      return -1;
  }
}

hipError_t mvd_launch_y_class(const LaunchArgs& a, int cls, int inv, int v) {
  switch (cls) {
#define X(c, t, tx, lmax, ...)                                                                     \
  case c:                                                                                          \
    if (inv)                                                                                       \
      k_ypass_class<true, t, tx, lmax, __VA_ARGS__><<<a.grid, t, 0, a.stream>>>(a.jobs, a.njobs,    \
                                                                               a.plans, a.tw, v);  \
    else                                                                                           \
      k_ypass_class<false, t, tx, lmax, __VA_ARGS__><<<a.grid, t, 0, a.stream>>>(a.jobs, a.njobs,   \
                                                                                a.plans, a.tw, v); \
    break;
    MVD_COL_CLASSES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t mvd_launch_z_class(const LaunchArgs& a, int cls, int v, int role, int conjH, int src_saved) {
  switch (cls) {
#define X(c, t, tx, lmax, ...)                                                                  \
  case c:                                                                                       \
    k_zconv_class<t, tx, lmax, __VA_ARGS__><<<a.grid, t, 0, a.stream>>>(a.jobs, a.njobs, a.plans, \
                                                                        a.tw, v, role, conjH,     \
                                                                        src_saved);               \
    break;
    MVD_COL_CLASSES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
