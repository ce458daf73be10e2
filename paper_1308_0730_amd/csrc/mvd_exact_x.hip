// x passes of the sequential scheme (modes 0-2) with compile-time plans for
// every 5-smooth half-row length (lists in mvd_exact_lengths.h); the modes
// of the combined updates are in mvd_exact_x_comb.hip.  A launch covers jobs
// whose nx / 2 is the plan's length.
#include "mvd_ct_passes.h"
#include "mvd_exact_lengths.h"

using namespace mvdk;

int mvd_exact_row_shape(int M, int* waves, int* rows) {
  switch (M) {
#define X(m, wpb, rpw, ...) \
  case m:                   \
    *waves = wpb;           \
    *rows = rpw;            \
    return 1;
    MVD_EXACT_ROW(X)
#undef X
    default:
      return 0;
  }
}

hipError_t mvd_launch_x_exact(const LaunchArgs& a, int M, int mode, int v, Partial* parts, int* flags, int opt) {
  if (mode == 3 || mode == 4) return mvd_launch_x_exact_comb(a, M, mode, v, parts, flags, opt);
  if (mode & XMODE_WIN) return mvd_launch_x_exact_win(a, M, mode, v, parts, flags, opt);
  switch (M) {
#define XM(md, m, wpb, rpw, ...)                                                                         \
  case md:                                                                                               \
    k_xpass_ct<md, wpb, rpw, m, __VA_ARGS__><<<a.grid, 64 * wpb, 0, a.stream>>>(a.jobs, a.njobs, a.plans, \
                                                                               a.tw, v, parts, flags,    \
                                                                               opt);                     \
    break;
#define X(m, wpb, rpw, ...)               \
  case m:                                 \
    switch (mode) {                       \
      XM(0, m, wpb, rpw, __VA_ARGS__)     \
      XM(1, m, wpb, rpw, __VA_ARGS__)     \
      XM(2, m, wpb, rpw, __VA_ARGS__)     \
      default:                            \
        return hipErrorInvalidValue;      \
    }                                     \
    break;
    MVD_EXACT_ROW(X)
#undef X
#undef XM
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
