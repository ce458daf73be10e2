// x passes of the combined updates (modes 3, 4) with compile-time plans for
// every 5-smooth half-row length (lists in mvd_exact_lengths.h).
#include "mvd_ct_passes.h"
#include "mvd_exact_lengths.h"

using namespace mvdk;

hipError_t mvd_launch_x_exact_comb(const LaunchArgs& a, int M, int mode, int v, Partial* parts, int* flags,
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
      XM(3, m, wpb, rpw, __VA_ARGS__)     \
      XM(4, m, wpb, rpw, __VA_ARGS__)     \
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
