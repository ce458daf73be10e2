// x passes of the block-wise form (modes 0 and 2 with the window bit) with
// compile-time plans for every 5-smooth half-row length (lists in
// mvd_exact_lengths.h).
#include "mvd_ct_passes.h"
#include "mvd_exact_lengths.h"

using namespace mvdk;

hipError_t mvd_launch_x_exact_win(const LaunchArgs& a, int M, int mode, int v, Partial* parts, int* flags,
                                  int opt) {
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
      XM(8, m, wpb, rpw, __VA_ARGS__)     \
      XM(10, m, wpb, rpw, __VA_ARGS__)    \
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
