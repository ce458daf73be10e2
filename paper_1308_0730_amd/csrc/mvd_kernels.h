// Host-side entry points of the gfx950 kernels (launch wrappers).
#pragma once
#include <hip/hip_runtime.h>

#include "mvd_types.h"

struct LaunchArgs {
  const JobDesc* jobs;   // device job table
  int njobs;
  const FftPlan* plans;  // device plan table
  const float2* tw;      // device twiddle pool
  hipStream_t stream;
  int grid;              // total tiles of the pass over all jobs
};

// Extra operands of the differentiated form's x passes (block 0 only).
struct AdjPtrs {
  float* b;            // blur stored by the forward (ratio) pass
  float* q;            // ratio stored by the forward pass
  float* c;            // back-projection stored by the forward (update) pass
  float* psi_in;       // estimate before the view-update
  const float* gbar;   // dL/dpsi' (input of the update's adjoint)
  float* part;         // direct part of dL/dpsi
  float* out;          // dL/dpsi written by the finishing pass
};

int mvd_num_cfgs(int kind);
int mvd_cfg_threads(int kind, int cfg);
int mvd_cfg_param(int kind, int cfg);   // rows (x) or lines (y, z) per tile
int mvd_cfg_maxlen(int kind, int cfg);  // largest transform length it accepts
int mvd_cfg_exact(int kind, int cfg);   // > 0: compile-time plan for exactly this length;
                                        // -1: the per-length compile-time plans (mvd_exact_cfg)
int mvd_exact_cfg(int kind);            // index of the per-length compile-time plans
int mvd_exact_param(int kind, int len); // rows (x) or lines (y, z) per tile of that plan, 0 if none

// compile-time candidates (mvd_kernels_ct.hip), indexed from 0
int mvd_ct_num_cfgs(int kind);
int mvd_ct_cfg(int kind, int cfg, int field);
hipError_t mvd_launch_x_ct(const LaunchArgs& a, int cfg, int mode, int v, Partial* parts, int* flags,
                           int opt);
hipError_t mvd_launch_y_ct(const LaunchArgs& a, int cfg, int inv, int v);
hipError_t mvd_launch_z_ct(const LaunchArgs& a, int cfg, int v, int role, int conjH, int src_saved);

// mode 0: R2C of psi; 1: blur -> ratio -> R2C; 2: back-projection -> update
// -> R2C; 3: back-projection -> fold into the combined factor; 4: the same,
// then the combined update -> R2C.  opt: XOPT_* bits.
hipError_t mvd_launch_x(const LaunchArgs& a, int cfg, int mode, int v, Partial* parts, int* flags, int opt);
hipError_t mvd_launch_y(const LaunchArgs& a, int cfg, int inv, int v);
// src_saved: read the tile from the job's saved spectrum (write to spec)
hipError_t mvd_launch_z(const LaunchArgs& a, int cfg, int v, int role, int conjH, int src_saved = 0);
hipError_t mvd_launch_reduce(const Partial* parts, int ntiles, int nviews, double* flux,
                             unsigned long long* ratio, unsigned long long* neg, hipStream_t s);
hipError_t mvd_launch_check(const float* x, int64_t n, float lo, float hi, double* psum,
                            unsigned long long* pbad, int nblocks, hipStream_t s);
hipError_t mvd_launch_fill(float* x, int64_t n, float val, hipStream_t s);
hipError_t mvd_launch_set_int(int* p, int val, hipStream_t s);

// differentiated form (mvd_adjoint.hip); cfg indexes the runtime-plan shapes
hipError_t mvd_launch_xadj(const LaunchArgs& a, int cfg, int mode, int v, Partial* parts, int* flags,
                           const AdjPtrs& ap);
// The same with the compile-time row plan of a power-of-two half-row length M
// (16 to 256); mvd_xadj_rows gives its rows per tile, 0 if M has none.
int mvd_xadj_rows(int M);
hipError_t mvd_launch_xadj_exact(const LaunchArgs& a, int M, int mode, int v, Partial* parts, int* flags,
                                 const AdjPtrs& ap);
hipError_t mvd_launch_zext(const LaunchArgs& a, int cfg, int v, int role, int conjH, float2* s_out,
                           const float2* s_in, double2* acc, int acc_mode);
hipError_t mvd_launch_idft_z(const double2* A, int M, int Mp, int ny, int nz, int wz, const double2* twz,
                             double2* T1, hipStream_t s);
// y and x stages after the z stage: out[dz][dy][dx] (FP64, no 1/V)
hipError_t mvd_launch_idft_yx(const double2* T1, int M, int nx, int ny, int wx, int wy, int wz, const double2* twx,
                              const double2* twy, double2* T2, double* out, hipStream_t s);

// compile-time plans for every 5-smooth length (mvd_exact_*.hip); a launch
// covers jobs that all have length L (y: ny, z: nz) or half-row length M (x).
// The shape queries return 0 when no plan exists for the length.
int mvd_exact_col_shape(int L, int* threads, int* lines);
int mvd_exact_row_shape(int M, int* waves, int* rows);
hipError_t mvd_launch_y_exact(const LaunchArgs& a, int L, int inv, int v);
hipError_t mvd_launch_z_exact(const LaunchArgs& a, int L, int v, int role, int conjH, int src_saved);
// Length classes of the column plans (0..4; -1 if L has no plan) and the
// launches over blocks of several lengths of one class.
int mvd_col_class(int L);
hipError_t mvd_launch_y_class(const LaunchArgs& a, int cls, int inv, int v);
hipError_t mvd_launch_z_class(const LaunchArgs& a, int cls, int v, int role, int conjH, int src_saved);
hipError_t mvd_launch_x_exact(const LaunchArgs& a, int M, int mode, int v, Partial* parts, int* flags, int opt);
hipError_t mvd_launch_x_exact_comb(const LaunchArgs& a, int M, int mode, int v, Partial* parts, int* flags,
                                   int opt);
hipError_t mvd_launch_x_exact_win(const LaunchArgs& a, int M, int mode, int v, Partial* parts, int* flags,
                                  int opt);
hipError_t mvd_launch_zext_exact(const LaunchArgs& a, int L, int v, int role, int conjH, float2* s_out,
                                 const float2* s_in, double2* acc, int acc_mode);

// weight normalisation (mvd_weights.hip), on one block's [nviews][V] weights
hipError_t mvd_launch_overlap_stats(const float* w, int nviews, int64_t V, unsigned* cmin,
                                    unsigned long long* csum, unsigned long long* ncov, hipStream_t s);
hipError_t mvd_launch_overlap_limit(float* w, int nviews, int64_t V, float m, hipStream_t s);
hipError_t mvd_launch_overlap_count(const float* w, int nviews, int64_t V, float* out, hipStream_t s);

// linear boundary (mvd_embed.hip): copy a (ux, uy, uz) volume into / out of a
// (nx, ny, nz) grid at offset off (x, y, z); the rest of the grid is untouched
hipError_t mvd_launch_embed(float* grid, const int* gdims, const float* vol, const int* udims, const int* off,
                            hipStream_t s);
hipError_t mvd_launch_extract(float* vol, const int* udims, const float* grid, const int* gdims, const int* off,
                              hipStream_t s);
// block-wise form (mvd_embed.hip): the (gx, gy, gz) window of the periodic
// volume vdims starting at start (each 0 <= start < vdims) into grid
hipError_t mvd_launch_gather(float* grid, const int* gdims, const float* vol, const int* vdims, const int* start,
                             hipStream_t s);
// every voxel of the grid outside the (ux, uy, uz) box at offset off gets val
hipError_t mvd_launch_fill_outside(float* grid, const int* gdims, const int* udims, const int* off, float val,
                                   hipStream_t s);
