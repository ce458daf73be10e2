/*
 * mvd.h -- C ABI of the MI355X (gfx950) sequential multi-view deconvolution
 * library (Preibisch et al., "Efficient Bayesian-based Multi-View
 * Deconvolution", arXiv 1308.0730).
 *
 * What the library computes.  For views phi_v, PSFs P_v, optional weights
 * w_v and a Tikhonov weight lambda, every iteration applies each view once, in
 * index order (section 7, "Alternative iteration for faster convergence"):
 *
 *   b   = psi (x) P_v                     expected view (eq. 1, eq. 51)
 *   q   = phi_v / max(b, eps)             ratio of observed to expected (eq. 15)
 *   c   = q (x) K_v                       back-projection
 *   u   = psi * max(c, 0)                 multiplicative RL step (eq. 15)
 *   t   = 2u / (1 + sqrt(1 + 4 lambda' u))  Tikhonov MAP step (solves lambda' t^2 + t = u)
 *   psi = psi + w_v (t - psi)             weights: fraction of the step applied
 *                                         (section 10, partially overlapping data)
 *
 * (x) is circular 3-D convolution on the volume grid with kernels centred at
 * (k-1)/2.  K_v is selected by the variant:
 *   MVD_RL   K_v = P_v*, the mirrored PSF (eq. 15/51; sequential = OS-EM, section 7.1)
 *   MVD_EFF  K_v = P_v* . prod_{w!=v} (P_v* (x) P_w (x) P_w*)   (eq. 220/222)
 *   MVD_OPT1 K_v = P_v* . prod_{w!=v} (P_v* (x) P_w)            (eq. 230, Optimization I)
 *   MVD_OPT2 K_v = (P_v*)^N                                     (eq. 240, Optimization II)
 * each normalised to sum one (every kernel is a probability distribution, eq. 3).
 * Scale: s = mean over all voxels of all views; psi starts flat at s (the
 * constant initial guess of eq. 15); eps = eps_scale * s (in FP32, at least
 * the smallest normal float); lambda' = lambda / s.
 *
 * Layout.  A volume of dims {nx, ny, nz} is nx*ny*nz float32, C order
 * [z][y][x], x fastest.  A PSF of dims {kx, ky, kz} is kx*ky*kz float32 in the
 * same order.  Even PSF extents are padded with one trailing zero plane.
 *
 * Ownership.  Every input is copied at create; the caller may free it on
 * return.  The handle owns all device memory (through the allocator callbacks
 * if given, else hipMalloc).  A handle is not thread-safe; separate handles
 * are independent.
 *
 * Errors.  Every function returns MVD_OK (0) or a negative code; no C++
 * exception crosses the ABI.  On failure of a create call *out stays NULL and
 * nothing leaks.  mvd_last_error() gives a message (per handle, or
 * thread-local for calls that have no handle).  Work is asynchronous on the
 * handle's stream: device-side faults (a non-finite estimate) surface as
 * MVD_ENONFINITE at the next synchronising call (mvd_get_estimate, mvd_stats,
 * mvd_synchronize).
 */
#ifndef MVD_H
#define MVD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MVD_OK 0
#define MVD_EINVAL (-1)     /* invalid argument, shape or value */
#define MVD_ENOMEM (-2)     /* device allocation failed */
#define MVD_EDEVICE (-3)    /* HIP runtime error */
#define MVD_ENONFINITE (-4) /* the estimate became NaN or Inf */
#define MVD_ESTATE (-5)     /* call out of order */

#define MVD_RL 0
#define MVD_EFF 1
#define MVD_OPT1 2
#define MVD_OPT2 3

/* How mvd_iterate_combined merges the views' factors. */
#define MVD_MEAN_GEOMETRIC 0  /* product and |V|-th root (eq. 51, normalised as in the
                                 convergence proof for multiple views) */
#define MVD_MEAN_ARITHMETIC 1 /* sum over |V| (additive ML-EM) */

#define MVD_MEM_HOST 0
#define MVD_MEM_DEVICE 1

#define MVD_MAX_VIEWS 64
#define MVD_MAX_LEN 1024    /* largest nx/2 */
#define MVD_MAX_LEN_YZ 1024 /* largest ny and nz */

typedef struct mvd_handle mvd_handle;

/* One volume to deconvolve (a block of the batched form).
 *   n_views   1..MVD_MAX_VIEWS
 *   dims      {nx, ny, nz}: nx even, every extent 5-smooth (2^a 3^b 5^c),
 *             4 <= nx <= 2*MVD_MAX_LEN, 2 <= ny, nz <= MVD_MAX_LEN_YZ (the
 *             differentiated form takes half-rows nx/2 up to 512, or powers
 *             of two up to 1024: its other adjoint x passes use runtime plans)
 *   views     n_views pointers to nx*ny*nz floats, finite and >= 0, not all
 *             zero (s scales the start and the ratio guard), registered onto
 *             the common grid (section 6: identity transformation)
 *   psfs      n_views pointers; psf_dims[3*v + {0,1,2}] = {kx, ky, kz};
 *             finite, >= 0, positive sum, each extent (after odd padding)
 *             no larger than the volume's
 *   weights   NULL (all ones) or n_views pointers to nx*ny*nz floats in [0, 1]
 *   mem_kind  MVD_MEM_HOST or MVD_MEM_DEVICE for views, psfs and weights
 */
typedef struct mvd_problem {
  int n_views;
  int dims[3];
  const float* const* views;
  const float* const* psfs;
  const int* psf_dims;
  const float* const* weights;
  int mem_kind;
} mvd_problem;

typedef void* (*mvd_alloc_fn)(size_t bytes, void* ctx);
typedef void (*mvd_free_fn)(void* ptr, void* ctx);

/* Options (NULL = all defaults).
 *   lambda     Tikhonov weight >= 0 (0 disables), dimensionless (divided by s)
 *   eps_scale  ratio guard relative to s (0 selects 1e-6)
 *   stream     hipStream_t the work is ordered on (NULL = default stream)
 *   alloc/free device allocator and its context (NULL = hipMalloc/hipFree);
 *              alloc returns NULL on failure, and must return 256-byte aligned memory
 *   use_graphs 0 = launch kernels directly, 1 = replay one HIP graph per
 *              iteration (default when options are NULL)
 *   tile_config  0 = autotuned/default pass shapes; k > 0 forces candidate k-1
 *   boundary   MVD_BOUNDARY_CIRCULAR (0): the volume is one period of a
 *              periodic grid (the convolutions wrap around);
 *              MVD_BOUNDARY_LINEAR (1): the views are known on the volume only
 *              and psi also lives on a margin of one PSF radius around it.
 *              The handle computes on the volume extended by the largest
 *              PSF radius per axis, rounded up to transform lengths (that
 *              grid must stay within the limits above: MVD_EINVAL); each
 *              view's blur is evaluated on the volume, and outside the
 *              volume, where the view has no data, its ratio is 1, so the
 *              back-projection over the grid leaves a margin voxel's step
 *              to the part of its light that reaches the volume (per voxel
 *              the restricted-matrix EM step applied as the fraction
 *              1_volume (x) K_v of a full step, as weights apply a fraction
 *              of a step: section on partially overlapping data; the volume
 *              padded by the PSF size, Supp. Table 1).  No threshold and no
 *              division by that fraction.
 *              Weights apply on the volume and are 1 in the margin.  Only
 *              the sequential scheme (mvd_iterate, mvd_view_update) runs with
 *              it; estimates are read and set on the volume (setting one
 *              resets the margin to s).
 */
typedef struct mvd_options {
  double lambda;
  double eps_scale;
  void* stream;
  mvd_alloc_fn alloc;
  mvd_free_fn free;
  void* alloc_ctx;
  int use_graphs;
  int tile_config;
  int boundary;
} mvd_options;

#define MVD_BOUNDARY_CIRCULAR 0
#define MVD_BOUNDARY_LINEAR 1

typedef struct mvd_stats_t {
  int64_t iterations;        /* iterations run since create / set_estimate */
  int n_views;
  int n_blocks;
  double scale;              /* s of block 0 */
  double flux[MVD_MAX_VIEWS]; /* sum of psi after each view-update of the last
                                 iteration, added over blocks (FP64) */
  int64_t ratio_clamps;      /* voxels with b < eps in the last iteration */
  int64_t neg_clamps;        /* voxels with c < 0 in the last iteration */
  int nonfinite;             /* 1 if psi became NaN/Inf since the last reset */
} mvd_stats_t;

/* Create a handle for one volume (the plain form).  Validates everything
 * listed at mvd_problem (MVD_EINVAL), copies the inputs, computes s, the
 * PSF spectra and sets psi to the flat start. */
int mvd_create(mvd_handle** out, const mvd_problem* p, const mvd_options* o);

/* Batched form: n_blocks independent volumes of any valid dims with the same
 * n_views, deconvolved together; every pass of an iteration covers all
 * blocks, in one launch (runtime or single-length plans) or, with the
 * per-length plans, one launch per stream lane and length (length class for
 * the column passes of blocks of several lengths); an iteration is replayed
 * from one HIP graph. */
int mvd_create_batch(mvd_handle** out, int n_blocks, const mvd_problem* blocks,
                     const mvd_options* o);

/* Block-wise form (main text: the volume is processed in blocks to reduce
 * the memory requirements; implementation section: blocks are copied out,
 * deconvolved and pasted back).  One volume of any extents >= 1 (not
 * limited by the transform lengths, not 5-smooth), taken as one period of a
 * periodic grid, is cut into near-equal blocks per axis (block k of t along
 * an axis of n voxels starts at floor(k n / t)).  Every view-update reads,
 * for each block, the window of the estimate made of the block and `halo`
 * voxels on each side (wrapping periodically), runs the view-update of
 * mvd_iterate on that window's grid (the largest block plus twice the halo,
 * rounded up to a transform length; every block uses the same grid), and
 * writes the block's own voxels back into the estimate; every block of a
 * view-update reads the estimate from before that view-update.  With halo >= twice the largest
 * PSF radius per axis the result equals the whole-volume update.
 *   p      the volume (dims any extents >= 1; views, PSFs and weights as for
 *          mvd_create; host or device memory)
 *   tiles  NULL or blocks per axis {tx, ty, tz}, each in [1, extent], or 0
 *          for the fewest blocks whose grid has nx <= 1024 and ny, nz <= 512
 *          (the fastest transform kernels), else the fewest whose grid fits
 *          the transform lengths (nx <= 2 MVD_MAX_LEN, ny, nz <=
 *          MVD_MAX_LEN_YZ)
 *   halo   NULL (twice the largest odd-padded PSF radius per axis, the
 *          exact choice; none along an axis with one block whose extent is
 *          a transform length, where the grid is the volume's period) or
 *          {hx, hy, hz} >= 0
 * MVD_EINVAL if a block's grid exceeds the transform lengths.  The handle
 * runs the sequential scheme (mvd_iterate, mvd_view_update, mvd_profile,
 * mvd_get_estimate and mvd_set_estimate of the whole volume as block 0,
 * mvd_stats with the flux of the volume; ratio clamps are counted over the
 * block grids, negativity clamps over the blocks' own voxels); the combined
 * updates, the differentiated
 * form, mvd_set_psfs and the weight normalisation return MVD_ESTATE.
 * mvd_grid_dims reports a block's grid; blocks share one set of kernel
 * planes. */
int mvd_create_blocked(mvd_handle** out, const mvd_problem* p, const mvd_options* o, const int* tiles,
                       const int* halo);

/* Blocks per axis, halo and volume extents {x, y, z} of a handle (each may be
 * NULL): {1, 1, 1}, {0, 0, 0} and the volume for handles that are not
 * block-wise (block 0's volume for batched handles). */
int mvd_blocking(const mvd_handle* h, int* tiles, int* halo, int* dims);

/* Run n >= 0 iterations of `variant` (MVD_RL..MVD_OPT2).  Asynchronous.  The
 * compound-kernel spectra of a variant are built on its first use. */
int mvd_iterate(mvd_handle* h, int n, int variant);

/* Run n >= 0 combined updates (eq. 51): per iteration every view's
 * back-projected ratio c_v = (phi_v / max(psi x P_v, eps)) x K_v is taken
 * from the same psi, and psi <- T_lambda(psi . mean_v max(c_v, 0)) with
 * `mean` MVD_MEAN_GEOMETRIC or MVD_MEAN_ARITHMETIC; `variant` picks K_v as in
 * mvd_iterate (MVD_RL with the arithmetic mean is classic ML-EM).
 * Asynchronous.  MVD_EINVAL for a handle created with weights (they apply to
 * sequential view-updates).  The first call allocates one volume and one
 * spectrum per block.  In the statistics, flux[n_views - 1] holds the sum of
 * psi after the update and the other entries are 0. */
int mvd_iterate_combined(mvd_handle* h, int n, int variant, int mean);

/* Apply one view-update (view `view`, all blocks) -- the inspection hook of
 * a single line of the sequential scheme of section 7.  Asynchronous; does
 * not advance the iteration count. */
int mvd_view_update(mvd_handle* h, int view, int variant);

/* Profiling hook: run n >= 1 iterations with every pass launched directly
 * and bracketed by HIP events on the handle's stream; avg_ms[k] and calls[k]
 * (k < MVD_PASS_KINDS) receive the mean duration and the number of launches
 * of pass kind k: 0 y forward, 1 y inverse, 2 z transform with the spectral
 * product, 3 x pass with the ratio, 4 x pass with the update.  Synchronises. */
#define MVD_PASS_KINDS 5
int mvd_profile(mvd_handle* h, int n, int variant, double* avg_ms, int* calls);

/* Differentiated form (single-block handles, any variant: for the compound
 * variants the back-projection kernels K_v are functions of every PSF and
 * their gradients are propagated through the construction, as in
 * mvd_compound_kernel_vjp).  Runs n iterations
 * from psi0 (NULL: the flat start s; psi0_kind host or device), keeping one
 * checkpoint per iteration, and returns the loss
 *   L = sum_v sum_x (psi_n (x) P_v - phi_v)^2
 * in *loss.  If grad_psf is not NULL, grad_psf[v] (host, the raw extents of
 * PSF v, may be NULL for some v) receives dL/dG_v with respect to the raw
 * PSF values G_v as given (through the normalisation P = G / sum G of eq. 3);
 * if grad_psi0 is not NULL it receives dL/dpsi0 (nx*ny*nz floats,
 * grad_kind host or device).  Gradients come from hand-written adjoint passes
 * run in reverse over each iteration recomputed from its checkpoint; the
 * PSF cross-spectra are accumulated in FP64.  The clamps max(b, eps) and
 * max(c, 0) contribute zero derivative where active.  Leaves psi at the end
 * of the run; synchronises.  MVD_ESTATE for batched handles. */
int mvd_loss_grad(mvd_handle* h, int n, int variant, const float* psi0, int psi0_kind, double* loss,
                  double* const* grad_psf, float* grad_psi0, int grad_kind);

/* Vector-Jacobian product of the same unrolled run, for any scalar loss of
 * the estimate: given grad_psi_n = dL/dpsi_n (nx*ny*nz floats, [z][y][x],
 * grad_psi_n_kind host or device; not retained), returns dL/dG_v in
 * grad_psf[v] and dL/dpsi0 in grad_psi0, exactly as mvd_loss_grad does
 * (same arguments, same checkpointed adjoint passes, same zero derivative
 * of active clamps), with the loss's own seed replaced by grad_psi_n: the
 * reverse mode of the view-update of eq. 15 with weights and Tikhonov,
 * iterated.  Recomputes the forward run from psi0 (NULL: the flat start),
 * leaves psi = psi_n; synchronises.  MVD_EINVAL if grad_psi_n is NULL,
 * MVD_ESTATE for batched, linear-boundary or block-wise handles. */
int mvd_backward(mvd_handle* h, int n, int variant, const float* psi0, int psi0_kind, const float* grad_psi_n,
                 int grad_psi_n_kind, double* const* grad_psf, float* grad_psi0, int grad_kind);

/* The recorded form of the same product, for callers that run the forward
 * themselves and differentiate later (autograd): mvd_forward_recorded runs n
 * iterations from psi0 (NULL: the flat start) keeping one checkpoint per
 * iteration, leaves psi = psi_n, synchronises and returns a token of the
 * recorded run in *token; mvd_backward_recorded(token, grad_psi_n, ...)
 * returns dL/dG_v and dL/dpsi0 as mvd_backward does, without running the
 * forward from psi0 again (the reverse sweep recomputes each iteration from
 * its checkpoint, except the last one, whose intermediates are still held).
 * The record stays valid for further backward calls until a call changes
 * the estimate, the PSFs or the weights (mvd_iterate, mvd_view_update,
 * mvd_set_estimate, mvd_set_psfs, mvd_normalize_weights, mvd_profile,
 * mvd_loss_grad, mvd_backward, another mvd_forward_recorded): then
 * MVD_ESTATE.  Same restrictions as mvd_loss_grad (single block, circular
 * boundary). */
int mvd_forward_recorded(mvd_handle* h, int n, int variant, const float* psi0, int psi0_kind, int64_t* token);
int mvd_backward_recorded(mvd_handle* h, int64_t token, const float* grad_psi_n, int grad_psi_n_kind,
                          double* const* grad_psf, float* grad_psi0, int grad_kind);

/* Replace the PSFs of a single-block handle (same count; extents may change
 * within the volume): recomputes their spectra; compound kernels are rebuilt
 * on their next use.  For PSF refinement loops. */
int mvd_set_psfs(mvd_handle* h, const float* const* psfs, const int* psf_dims, int mem_kind);

/* Launch shapes (the autotuner's knobs).  Pass kinds: 0 x (rows), 1 y,
 * 2 z (columns).  Candidate c of a kind has a thread count, a tile size
 * (rows or columns per workgroup), the longest transform it accepts and,
 * for compile-time plans, the one length it is built for (exact_len > 0;
 * usable only when every block has that length; 0 = runtime plan, any
 * 5-smooth length up to max_len; -1 = the per-length compile-time plans,
 * one shape for each 5-smooth length up to max_len, launched per group of
 * blocks of equal length, or of one length class for the column passes of
 * blocks of several lengths: threads and per_tile are reported as 0 since
 * they depend on the length).  mvd_tile_candidates lists, into
 * out[0..cap), the candidates for transforms of length max_len and returns
 * how many exist.  mvd_set_tiles selects one candidate per kind for a handle
 * (MVD_EINVAL if one does not fit its volumes); later iterations use them.
 * mvd_get_tiles reports the current choice. */
int mvd_tile_candidates(int kind, int max_len, int* out, int cap);
int mvd_tile_shape(int kind, int cfg, int* threads, int* per_tile, int* max_len, int* exact_len);
int mvd_set_tiles(mvd_handle* h, int cfg_x, int cfg_y, int cfg_z);
int mvd_get_tiles(const mvd_handle* h, int* cfg);

/* Schedule of a multi-block handle's runs (the autotuner's other knob).
 * Blocks are independent, so every schedule gives the same results; they
 * differ in what the memory-side cache holds between passes.
 *   MVD_SCHEDULE_PASS_MAJOR  each pass covers every block of a stream lane
 *                            (one launch per lane and length or length
 *                            class), one graph per iteration (the default)
 *   MVD_SCHEDULE_BLOCK_MAJOR each lane takes its blocks one at a time: a
 *                            block's view-updates of an iteration, then the
 *                            next block
 *   MVD_SCHEDULE_RUN_MAJOR   each lane takes its blocks one at a time for
 *                            the whole run: all n iterations of a block,
 *                            then the next; one graph per run
 * The block-major schedules take effect with the per-length plans for all
 * three pass kinds and two or more blocks (otherwise runs are pass-major);
 * mvd_profile always runs pass-major.  mvd_get_schedule returns the
 * current one. */
#define MVD_SCHEDULE_PASS_MAJOR 0
#define MVD_SCHEDULE_BLOCK_MAJOR 1
#define MVD_SCHEDULE_RUN_MAJOR 2
int mvd_set_schedule(mvd_handle* h, int schedule);
int mvd_get_schedule(const mvd_handle* h);

/* Overlap numbers for mvd_normalize_weights (section on partially
 * overlapping data). */
#define MVD_OVERLAP_ONE 0  /* 1: the safe choice */
#define MVD_OVERLAP_MIN 1  /* the minimal number of contributing views over the covered voxels */
#define MVD_OVERLAP_AVG 2  /* their average number */
#define MVD_OVERLAP_USER 3 /* `value` (> 0) */

/* Limit each voxel's summed weight over the views to the overlap number m
 * of its block: where the sum s exceeds m every view's weight there is
 * multiplied by m / s; weights are never increased (section on partially
 * overlapping data).  A view contributes at a voxel where its weight is > 0;
 * "covered" voxels have at least one contributing view.  Rewrites the
 * handle's weights in place (later iterations use them); m of every block is
 * written to m_out[n_blocks] when it is not NULL.  MVD_ESTATE for a handle
 * created without weights; MVD_EINVAL for a bad mode or value.  Synchronises. */
int mvd_normalize_weights(mvd_handle* h, int mode, double value, double* m_out);

/* The number of contributing views at every voxel of `block`, as floats
 * (nx*ny*nz, host or device memory): the image the paper offers for
 * choosing the overlap number.  MVD_ESTATE without weights.  Synchronises. */
int mvd_contributing_views(mvd_handle* h, float* dst, int dst_kind, int block);

/* Copy the estimate of `block` (0 for the plain form) into dst (nx*ny*nz
 * floats, host or device memory).  Synchronises; returns MVD_ENONFINITE if
 * the estimate became non-finite (the copy is still made). */
int mvd_get_estimate(mvd_handle* h, float* dst, int dst_kind, int block);

/* Replace the estimate of `block` (finite, >= 0); resets the iteration count
 * and the non-finite flag.  Use to resume from a checkpoint or to start the
 * differentiated form from a given psi_0. */
int mvd_set_estimate(mvd_handle* h, const float* src, int src_kind, int block);

/* The computation grid (nx, ny, nz) of `block` into dims[3]: the volume's
 * own dims with the circular boundary, the volume plus its PSF margin
 * rounded up to transform lengths with the linear one. */
int mvd_grid_dims(const mvd_handle* h, int block, int* dims);

/* Synchronise and report statistics of the last mvd_iterate call. */
int mvd_stats(mvd_handle* h, mvd_stats_t* s);

/* Wait for all queued work; MVD_ENONFINITE if psi became non-finite. */
int mvd_synchronize(mvd_handle* h);

/* Release everything the handle owns.  NULL is accepted. */
int mvd_destroy(mvd_handle* h);

/* Message of the last failure on h (or of this thread when h is NULL). */
const char* mvd_last_error(const mvd_handle* h);

/* ---- host utilities (no device needed) ---------------------------------
 * Compound kernel of view v (FP64, host): the same K_v the handle uses,
 * normalised, in the odd window of P_v.  out receives kx*ky*kz doubles of
 * the padded window; out_dims (may be NULL) receives its {kx, ky, kz}. */
int mvd_compound_kernel(int n_views, const float* const* psfs, const int* psf_dims, int v,
                        int variant, double* out, int* out_dims);

/* Adjoint of mvd_compound_kernel (FP64, host): given kbar = dL/dK_v on the
 * padded odd window of P_v, grad_out[w] (n_views pointers, each the padded
 * odd window of P_w, kx*ky*kz doubles) receives dL/dP_w with respect to the
 * normalised PSFs (before the normalisation's own Jacobian), for every w
 * (zero where K_v does not depend on P_w).  The back-propagation of the
 * construction of eq. 222 (EFF), eq. 230 (OPT1) and eq. 240 (OPT2). */
int mvd_compound_kernel_vjp(int n_views, const float* const* psfs, const int* psf_dims, int v, int variant,
                            const double* kbar, double* const* grad_out);

/* Spectrum of a centred odd kernel on the volume grid, as the handle stores
 * it: H[kz][ky][kx] = (1/V) sum_d K[c+d] exp(-2 pi i k.d / n) for
 * kx < nx/2 into main (complex float pairs, nz*ny*(nx/2)), and kx = nx/2 into
 * nyq (nz*ny pairs).  FP64 arithmetic, rounded once. */
int mvd_kernel_spectrum(const double* kernel, const int* kdims, const int* dims, float* main_out,
                        float* nyq_out);

/* ---- no-allocation run ---------------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * work as mvd_create, mvd_set_estimate (when psi0 is not NULL), mvd_iterate
 * and mvd_get_estimate into psi_out, on one volume, with every device buffer
 * (estimate, spectrum, views, weights, kernel planes, FFT plans and tables,
 * partial sums, flags) placed in a static array of the library of
 * MVD_NOALLOC_SCRATCH_BYTES per GPU instead of being allocated.  No
 * hipMalloc, hipFree, stream, event or graph is created; the kernels are
 * those of mvd_iterate, launched directly on o->stream (NULL: the default
 * stream), and the call returns when they are done.
 *   p        one volume as for mvd_create (host or device inputs)
 *   o        options as for mvd_create (NULL = defaults), except that alloc
 *            and free must be NULL (MVD_EINVAL) and use_graphs is ignored
 *   psi0     NULL (flat start s) or nx*ny*nz device floats, finite, >= 0
 *   n, variant  as for mvd_iterate
 *   psi_out  nx*ny*nz device floats: the estimate after the run (may be psi0)
 * Returns MVD_EINVAL with a message naming the sizes when the problem needs
 * more than the array holds (roughly 4 (2 + n_views (1 + weights)) bytes per
 * voxel plus the kernel planes, e.g. 128^3 with 4 views and no weights),
 * MVD_ENONFINITE if the estimate became non-finite.  Every call on a GPU
 * reuses that GPU's array and starts from nothing in it; calls that overlap
 * on one GPU (from several threads, or on streams the caller does not
 * order) race on the array and give wrong results. */
#define MVD_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int mvd_iterate_noalloc(const mvd_problem* p, const mvd_options* o, const float* psi0, int n, int variant,
                        float* psi_out);

/* Library version string. */
const char* mvd_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MVD_H */
