// Launch-shape candidates with compile-time plans for the power-of-two
// lengths (the pass kernels are in mvd_ct_passes.h).
#include "mvd_ct_passes.h"

using namespace mvdk;

// ---------------------------------------------------------------------------
// Candidate table.  Columns: (threads, lines per tile, length, radices).
// Rows: (waves per block, rows per wave, half-row length, radices).

#define MVD_CT_COL_CFGS(X)        \
  X(0, 512, 16, 512, 8, 8, 8)     \
  X(1, 256, 16, 512, 8, 8, 8)     \
  X(2, 256, 8, 512, 8, 8, 8)      \
  X(3, 256, 16, 256, 16, 16)      \
  X(4, 256, 16, 256, 8, 8, 4)     \
  X(5, 128, 8, 256, 16, 16)       \
  X(6, 128, 16, 128, 16, 8)       \
  X(7, 64, 16, 64, 8, 8)          \
  X(8, 512, 32, 256, 16, 16)      \
  X(9, 64, 8, 128, 16, 8)         \
  X(10, 64, 4, 128, 16, 8)        \
  X(11, 128, 8, 128, 16, 8)       \
  X(12, 64, 8, 64, 8, 8)          \
  X(13, 64, 4, 64, 8, 8)

#define MVD_CT_ROW_CFGS(X)      \
  X(0, 2, 4, 256, 16, 16)       \
  X(1, 4, 2, 256, 8, 8, 4)      \
  X(2, 1, 4, 256, 16, 16)       \
  X(3, 2, 1, 512, 8, 8, 8)      \
  X(4, 2, 8, 128, 16, 8)        \
  X(5, 2, 8, 64, 8, 8)          \
  X(6, 2, 16, 32, 8, 4)         \
  X(7, 4, 4, 256, 16, 16)       \
  X(8, 1, 16, 32, 8, 4)         \
  X(9, 1, 8, 64, 8, 8)          \
  X(10, 1, 8, 128, 16, 8)

static const int kCtColCfg[][3] = {
#define X(i, t, tx, l, ...) {t, tx, l},
    MVD_CT_COL_CFGS(X)
#undef X
};
static const int kCtRowCfg[][3] = {
#define X(i, wpb, rpw, m, ...) {64 * wpb, wpb * rpw, m},
    MVD_CT_ROW_CFGS(X)
#undef X
};

int mvd_ct_num_cfgs(int kind) {
  return kind == PASS_X ? (int)(sizeof(kCtRowCfg) / sizeof(kCtRowCfg[0]))
                        : (int)(sizeof(kCtColCfg) / sizeof(kCtColCfg[0]));
}
int mvd_ct_cfg(int kind, int cfg, int field) { return kind == PASS_X ? kCtRowCfg[cfg][field] : kCtColCfg[cfg][field]; }

hipError_t mvd_launch_x_ct(const LaunchArgs& a, int cfg, int mode, int v, Partial* parts, int* flags,
                           int opt) {
  switch (cfg) {
#define XM(md, wpb, rpw, m, ...)                                                                   \
  case md:                                                                                         \
    k_xpass_ct<md, wpb, rpw, m, __VA_ARGS__><<<a.grid, 64 * wpb, 0, a.stream>>>(a.jobs, a.njobs,   \
                                                                               a.plans, a.tw, v,  \
                                                                               parts, flags, opt); \
    break;
#define X(i, wpb, rpw, m, ...)          \
  case i:                               \
    switch (mode) {                     \
      XM(0, wpb, rpw, m, __VA_ARGS__)   \
      XM(1, wpb, rpw, m, __VA_ARGS__)   \
      XM(2, wpb, rpw, m, __VA_ARGS__)   \
      XM(3, wpb, rpw, m, __VA_ARGS__)   \
      XM(4, wpb, rpw, m, __VA_ARGS__)   \
      default:                          \
        return hipErrorInvalidValue;    \
    }                                   \
    break;
    MVD_CT_ROW_CFGS(X)
#undef X
#undef XM
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t mvd_launch_y_ct(const LaunchArgs& a, int cfg, int inv, int v) {
  switch (cfg) {
#define X(i, t, tx, l, ...)                                                                            \
  case i:                                                                                              \
    if (inv)                                                                                           \
      k_ypass_ct<true, t, tx, l, __VA_ARGS__><<<a.grid, t, 0, a.stream>>>(a.jobs, a.njobs, a.plans,    \
                                                                         a.tw, v);                     \
    else                                                                                               \
      k_ypass_ct<false, t, tx, l, __VA_ARGS__><<<a.grid, t, 0, a.stream>>>(a.jobs, a.njobs, a.plans,   \
                                                                          a.tw, v);                    \
    break;
    MVD_CT_COL_CFGS(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t mvd_launch_z_ct(const LaunchArgs& a, int cfg, int v, int role, int conjH, int src_saved) {
  switch (cfg) {
#define X(i, t, tx, l, ...)                                                                            \
  case i:                                                                                              \
    k_zconv_ct<t, tx, l, __VA_ARGS__><<<a.grid, t, 0, a.stream>>>(a.jobs, a.njobs, a.plans, a.tw, v,   \
                                                                   role, conjH, src_saved);            \
    break;
    MVD_CT_COL_CFGS(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
