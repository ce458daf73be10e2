// Runtime behind the C ABI: validation, device buffers, plans, kernel
// spectra, pass scheduling and HIP-graph replay of one iteration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <set>
#include <stdexcept>
#include <string>
#include <type_traits>
#include <vector>

#include "mvd.h"
#include "mvd_host.h"
#include "mvd_kernels.h"
#include "mvd_types.h"

namespace {

thread_local std::string g_err;

// The no-allocation run (mvd_iterate_noalloc): every buffer it needs lives
// in this array, one copy per GPU, held from the library's load on that GPU
// until the process ends.  In host code the name only stands in for the
// symbol; its device address on the current GPU comes from
// hipGetSymbolAddress, looked up once per device (scratch_on_current_device).
static __device__ __align__(256) unsigned char scratch[MVD_NOALLOC_SCRATCH_BYTES];

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIPCHECK(expr)                                                                   \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess) {                                                              \
      if (e_ == hipErrorOutOfMemory) throw Error(MVD_ENOMEM, std::string(#expr) + ": out of memory"); \
      throw Error(MVD_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));      \
    }                                                                                    \
  } while (0)

[[noreturn]] void bad(const std::string& m) { throw Error(MVD_EINVAL, m); }

struct Block {
  int nx = 0, ny = 0, nz = 0, M = 0;
  int Mp = 0;  // row pitch of the main half spectrum and of the kernel planes: M rounded up to 16
  int64_t V = 0, spec_main = 0, spec_elems = 0;
  // common z window of the stored kernel planes (odd, centred) and the
  // per-view size of a kernel-plane array; kz_cap is the allocated window
  int kz = 0, cz = 0, kz_cap = 0;
  int64_t h_main = 0, h_elems = 0;
  float* psi = nullptr;
  float* spec = nullptr;
  float* phi = nullptr;
  float* w = nullptr;
  float* H[N_ROLES] = {nullptr, nullptr, nullptr, nullptr};
  float* acc = nullptr;    // combined-update factor [V], allocated on first use
  float* saved = nullptr;  // spectrum of psi kept over a combined iteration
  // linear boundary: the user's volume (ux, uy, uz) at offset (ox, oy, oz)
  // in the computation grid (nx, ny, nz); circular: the same box, offset 0
  int ux = 0, uy = 0, uz = 0, ox = 0, oy = 0, oz = 0;
  int64_t UV = 0;
  std::vector<mvdh::Kern> P;  // prepared PSFs
  std::vector<double> psf_sum;     // sums of the raw PSF inputs
  std::vector<std::array<int, 3>> psf_dims;  // raw extents {kx, ky, kz}
  double s = 0;
  float eps = 0, lamp = 0;
};

}  // namespace

struct mvd_handle {
  int device = 0;
  hipStream_t stream = nullptr;
  hipStream_t cap = nullptr;
  mvd_alloc_fn alloc = nullptr;
  mvd_free_fn free_fn = nullptr;
  void* actx = nullptr;
  std::vector<void*> allocs;
  std::vector<Block> blocks;
  int nviews = 0;
  double lambda = 0, eps_scale = 1e-6;
  bool use_graphs = true;
  int force_cfg = 0;
  // buffers come from a caller-owned region and no stream, event or graph
  // is created (the no-allocation entry point: one block, direct launches
  // on the caller's stream)
  bool no_alloc = false;
  // block-wise form: the volume (any extents, one period of a periodic
  // grid) is cut into near-equal blocks; each block computes on its own grid
  // (the block plus a halo on both sides, read periodically from the volume
  // by every view-update's first x pass), and its update pass writes the
  // block's own voxels into the volume
  bool blocked = false;
  struct Tiling {
    int dims[3] = {0, 0, 0};   // the volume (x, y, z)
    int tiles[3] = {1, 1, 1};  // blocks per axis
    int halo[3] = {0, 0, 0};   // grid voxels before a block's first voxel, per axis
    int64_t V = 0;
    float* psi = nullptr;      // [V] the estimate
    std::vector<std::array<int, 3>> origin, extent, start;  // per block; start = (origin - halo) mod dims
  } tl;
  // blocks of one geometry share the kernel planes of one block
  bool shared_kernels = false;
  // device tables
  JobDesc* d_jobs = nullptr;
  // per pass kind: the job table sorted by (lane, that kind's length), and
  // the groups of equal lane and length launched one by one with the
  // per-length compile-time plans
  struct Group {
    int len, first, njobs, grid, part_off;
    int lane;      // 0: the pass's stream, 1..kSide: side stream lane - 1
    int cls = -1;  // column passes over several lengths: the length class of one launch
  };
  // side streams (default priority).  Every block has a lane (longest
  // processing time first over the blocks' voxel counts), so all groups of a
  // block run on one stream in pass order: a sequential iteration forks the
  // side streams once and joins them at its end (defer_join); other
  // sequences fork and join around every pass.
  static constexpr int kSide = 15;
  int nside = 0;  // side lanes created: one per further block, at most kSide
  hipStream_t side[kSide] = {};
  hipEvent_t ev_fork = nullptr;
  hipEvent_t ev_join[kSide] = {};
  bool defer_join = false;
  std::vector<int> block_lane;
  JobDesc* d_jobs_k[3] = {nullptr, nullptr, nullptr};
  std::vector<int> order[3];
  std::vector<Group> groups[3];
  // per pass kind and block: the one-block group of that block in the
  // sorted job order (the block-major schedules), set with the per-length
  // plans of all three kinds
  std::vector<Group> bgroups[3];
  // MVD_SCHEDULE_*: the order in which a multi-block handle's lanes take the
  // passes of a run, and the graphs of whole runs (key: variant, n)
  int schedule = 0;
  std::map<std::pair<int, int>, hipGraphExec_t> run_exec;
  FftPlan* d_plans = nullptr;
  float2* d_tw = nullptr;
  Partial* d_parts = nullptr;
  int* d_flags = nullptr;
  double* d_flux = nullptr;
  unsigned long long* d_ratio = nullptr;
  unsigned long long* d_neg = nullptr;
  double* d_chk_sum = nullptr;
  unsigned long long* d_chk_bad = nullptr;
  std::vector<JobDesc> jobs;
  std::map<int, int> plan_of_len;
  std::map<int, int> pp_of_nx;
  int cfg_x = 0, cfg_y = 0, cfg_z = 0;
  int grid_x = 0, grid_y = 0, grid_z = 0;
  int max_len[3] = {0, 0, 0};
  int uniform_len[3] = {0, 0, 0};  // the common length of a pass kind, 0 if the blocks differ
  size_t parts_cap = 0;
  bool spec_valid = false;
  bool linear = false;            // MVD_BOUNDARY_LINEAR
  bool built[N_ROLES] = {true, false, false, false};
  int64_t iterations = 0;
  // one graph per (scheme, variant): scheme 0 sequential, 1 combined with
  // the geometric mean, 2 combined with the arithmetic mean
  hipGraphExec_t exec[3 * 4] = {};
  // differentiated form: runtime-plan shapes, grids and buffers (block 0)
  int rt_cfg[3] = {-1, -1, -1};
  int rt_grid[3] = {0, 0, 0};
  // the differentiated form's x passes: rows per tile of the compile-time
  // row plan (0: runtime plans) and their grid
  int gx_rows = 0, gx_grid = 0;
  bool grad_ready = false;
  // the recorded run of the differentiated form: its checkpoints are valid
  // while rec_token is non-zero (any call that changes the estimate, the
  // PSFs or the weights clears it); inter_iter is the iteration whose
  // intermediates (b, q, c, psi and the spectra per view) are stored
  int64_t rec_token = 0, rec_count = 0;
  int rec_n = 0, rec_variant = 0, inter_iter = -1;
  int grad_ckpt_cap = 0;
  float* g_ckpt = nullptr;                 // checkpoints, one volume per iteration
  float *g_b = nullptr, *g_q = nullptr, *g_c = nullptr, *g_psi = nullptr;  // [view][V]
  float2 *g_spsi = nullptr, *g_sq = nullptr, *g_sT = nullptr;  // spectra [view][spec]
  double2* g_acc = nullptr;                // PSF cross-spectra [view][spec], FP64
  double2* g_acck = nullptr;               // compound variants: back-projection kernel cross-spectra
  float *g_gbar = nullptr, *g_part = nullptr, *g_psiT = nullptr;
  Partial* g_parts = nullptr;              // [view][x tiles]
  double* g_loss = nullptr;
  double2 *g_twz = nullptr, *g_twy = nullptr, *g_twx = nullptr;  // exp(-2 pi i m / n), FP64
  double2* g_t1 = nullptr;                 // z stage of the PSF-gradient inverse DFT
  double2* g_t2 = nullptr;                 // its y stage
  double* g_gw = nullptr;                  // the windowed result
  size_t g_t1_cap = 0, g_t2_cap = 0, g_gw_cap = 0;
  unsigned long long *g_lr = nullptr, *g_ln = nullptr;
  // weight normalisation: overlap statistics, and a staging volume for the
  // count image when the caller's buffer is in host memory
  unsigned* w_cmin = nullptr;
  unsigned long long* w_cnt = nullptr;
  float* w_stage = nullptr;
  int64_t w_stage_cap = 0;
  std::string err;

  void* dalloc(size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    void* p = nullptr;
    if (alloc) {
      p = alloc(bytes, actx);
      if (!p) throw Error(MVD_ENOMEM, "allocator callback failed for " + std::to_string(bytes) + " bytes");
    } else {
      hipError_t e = hipMalloc(&p, bytes);
      if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        throw Error(MVD_ENOMEM, "hipMalloc failed for " + std::to_string(bytes) + " bytes");
      }
    }
    allocs.push_back(p);
    return p;
  }

  void release() {
    for (auto& g : exec)
      if (g) {
        (void)hipGraphExecDestroy(g);
        g = nullptr;
      }
    for (auto& kv : run_exec) (void)hipGraphExecDestroy(kv.second);
    run_exec.clear();
    if (cap) (void)hipDeviceSynchronize();
    for (void* p : allocs) {
      if (alloc && free_fn)
        free_fn(p, actx);
      else if (!alloc)
        (void)hipFree(p);
    }
    allocs.clear();
    if (cap) (void)hipStreamDestroy(cap);
    cap = nullptr;
    for (int i = 0; i < kSide; ++i) {
      if (side[i]) (void)hipStreamDestroy(side[i]);
      if (ev_join[i]) (void)hipEventDestroy(ev_join[i]);
      side[i] = nullptr;
      ev_join[i] = nullptr;
    }
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    ev_fork = nullptr;
  }
};

extern "C" int mvd_set_estimate(mvd_handle* h, const float* src, int src_kind, int block);

namespace {

int read_flag(mvd_handle* h);

int64_t vox(const int* d) { return (int64_t)d[0] * d[1] * d[2]; }

void validate_shape(const mvd_problem* p, int idx) {
  const std::string b = "block " + std::to_string(idx) + ": ";
  if (!p) bad(b + "problem is NULL");
  if (p->n_views < 1 || p->n_views > MVD_MAX_VIEWS) bad(b + "n_views must be in [1, 64]");
  const int nx = p->dims[0], ny = p->dims[1], nz = p->dims[2];
  if (nx < 4 || nx % 2 || nx / 2 > MVD_MAX_LEN) bad(b + "nx must be even, >= 4 and <= 2048");
  if (ny < 2 || ny > MVD_MAX_LEN_YZ || nz < 2 || nz > MVD_MAX_LEN_YZ) bad(b + "ny and nz must be in [2, 1024]");
  if (!mvdh::is_smooth5(nx / 2) || !mvdh::is_smooth5(ny) || !mvdh::is_smooth5(nz))
    bad(b + "every extent must be 5-smooth (2^a 3^b 5^c)");
  if (!p->views || !p->psfs || !p->psf_dims) bad(b + "views, psfs and psf_dims are required");
  if (p->mem_kind != MVD_MEM_HOST && p->mem_kind != MVD_MEM_DEVICE) bad(b + "mem_kind must be host or device");
  for (int v = 0; v < p->n_views; ++v) {
    if (!p->views[v] || !p->psfs[v]) bad(b + "view or PSF pointer " + std::to_string(v) + " is NULL");
    if (p->weights && !p->weights[v]) bad(b + "weight pointer " + std::to_string(v) + " is NULL");
    const int* k = p->psf_dims + 3 * v;
    for (int a = 0; a < 3; ++a) {
      if (k[a] < 1) bad(b + "PSF extents must be >= 1");
      if ((k[a] | 1) > p->dims[a]) bad(b + "PSF " + std::to_string(v) + " (odd-padded) is larger than the volume");
    }
  }
}

void validate_host_values(const mvd_problem* p, int idx) {
  const std::string b = "block " + std::to_string(idx) + ": ";
  const int64_t V = vox(p->dims);
  for (int v = 0; v < p->n_views; ++v) {
    if (!mvdh::all_within(p->views[v], V, 0.f, INFINITY))
      bad(b + "view " + std::to_string(v) + " has a negative or non-finite value");
    if (p->weights && !mvdh::all_within(p->weights[v], V, 0.f, 1.f))
      bad(b + "weights " + std::to_string(v) + " outside [0, 1]");
  }
}

std::vector<float> fetch_psf(const mvd_problem* p, int v) {
  const int* k = p->psf_dims + 3 * v;
  const size_t n = (size_t)k[0] * k[1] * k[2];
  std::vector<float> h(n);
  if (p->mem_kind == MVD_MEM_HOST)
    std::memcpy(h.data(), p->psfs[v], n * sizeof(float));
  else
    HIPCHECK(hipMemcpy(h.data(), p->psfs[v], n * sizeof(float), hipMemcpyDeviceToHost));
  return h;
}

// The ratio guard eps = eps_scale * s in FP32, at least the smallest normal
// float: the ratio pass takes the hardware reciprocal of max(b, eps), which
// must stay finite (only views with a mean below about 1e-32 reach it).
float ratio_guard(const mvd_handle* h, double s) {
  return std::max((float)(h->eps_scale * s), std::numeric_limits<float>::min());
}

// Device check of one array: count of values outside [lo, hi] (or
// non-finite) and the FP64 sum.
void device_check(mvd_handle* h, const float* x, int64_t n, float lo, float hi, double* sum,
                  unsigned long long* nbad) {
  const int nb = 1024;
  if (!h->d_chk_sum) {
    h->d_chk_sum = (double*)h->dalloc(nb * sizeof(double));
    h->d_chk_bad = (unsigned long long*)h->dalloc(nb * sizeof(unsigned long long));
  }
  double* ps = h->d_chk_sum;
  unsigned long long* pb = h->d_chk_bad;
  HIPCHECK(mvd_launch_check(x, n, lo, hi, ps, pb, nb, h->stream));
  std::vector<double> hs(nb);
  std::vector<unsigned long long> hb(nb);
  HIPCHECK(hipMemcpyAsync(hs.data(), ps, nb * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHECK(hipMemcpyAsync(hb.data(), pb, nb * sizeof(unsigned long long), hipMemcpyDeviceToHost, h->stream));
  HIPCHECK(hipStreamSynchronize(h->stream));
  double s = 0;
  unsigned long long c = 0;
  for (int i = 0; i < nb; ++i) {
    s += hs[i];
    c += hb[i];
  }
  *sum = s;
  *nbad = c;
}

int plan_for(mvd_handle* h, int L, std::vector<FftPlan>& plans, std::vector<float2>& tw) {
  auto it = h->plan_of_len.find(L);
  if (it != h->plan_of_len.end()) return it->second;
  FftPlan pl{};
  pl.L = L;
  const auto r = mvdh::factorize(L);
  pl.nst = (int)r.size();
  if (pl.nst > MVD_MAX_STAGES) bad("too many FFT stages");
  int ns = 1;
  for (int i = 0; i < pl.nst; ++i) {
    pl.radix[i] = r[i];
    pl.ns[i] = ns;
    pl.tws[i] = L / (ns * r[i]);
    pl.ns_magic[i] = mvd_magic((unsigned)ns);
    pl.nb_magic[i] = mvd_magic((unsigned)(L / r[i]));
    ns *= r[i];
  }
  pl.tw = (int)tw.size();
  for (const auto& c : mvdh::twiddles(L)) tw.push_back(make_float2((float)c.real(), (float)c.imag()));
  plans.push_back(pl);
  h->plan_of_len[L] = (int)plans.size() - 1;
  return (int)plans.size() - 1;
}

// Common z window of a block's kernels: the largest z extent of its
// prepared PSFs (every compound kernel lives in its PSF's window).
void set_kernel_window(Block& B) {
  int kz = 1;
  for (const auto& K : B.P) kz = std::max(kz, K.kz);
  B.kz = kz;
  B.cz = (kz - 1) / 2;
  B.h_main = (int64_t)B.Mp * B.ny * kz;
  B.h_elems = B.h_main + (int64_t)B.ny * kz;
}

// Kernel planes of a centred kernel in the stored layout: the x and y
// stages of its spectrum (FP64 on the host) on the block's z window, the
// kernel's own planes centred in it, scaled by 1/V and rounded once to
// FP32.  The z stage is done by the z pass.
void upload_kernel(mvd_handle* h, const Block& B, const mvdh::Kern& K, float* dst) {
  if (K.kz > B.kz || (B.kz - K.kz) % 2) bad("kernel does not fit the z window");
  // x and y stages in FP64, scaled by 1/V, on the common z window
  std::vector<float> hk((size_t)B.h_elems * 2, 0.f);
  mvdh::spectrum_xy_f32(K, B.nx, B.ny, 1.0 / (double)B.V, (B.kz - K.kz) / 2, B.Mp, B.h_main, hk.data());
  HIPCHECK(hipMemcpyAsync(dst, hk.data(), hk.size() * sizeof(float), hipMemcpyHostToDevice, h->stream));
  HIPCHECK(hipStreamSynchronize(h->stream));
}

bool cfg_fits(const mvd_handle* h, int kind, int c);

// Default launch shape of a pass kind: a forced candidate if it fits, else
// the first fitting entry of a preference list (compile-time plans for the
// common power-of-two lengths, then the smallest runtime-plan family).
int pick_cfg(const mvd_handle* h, int kind) {
  if (h->force_cfg > 0 && cfg_fits(h, kind, h->force_cfg - 1)) return h->force_cfg - 1;
  const int nrt = mvd_exact_cfg(kind) - mvd_ct_num_cfgs(kind);
  // compile-time candidates in order of preference
  static const int ct_x[] = {0, 3, 4, 5, 6};
  static const int ct_c[] = {0, 3, 6, 7};
  if (kind == PASS_X) {
    for (int c : ct_x)
      if (cfg_fits(h, kind, nrt + c)) return nrt + c;
    if (cfg_fits(h, kind, mvd_exact_cfg(kind))) return mvd_exact_cfg(kind);
    for (int c : {0, 1, 2, 3, 4})
      if (cfg_fits(h, kind, c)) return c;
  } else {
    for (int c : ct_c)
      if (cfg_fits(h, kind, nrt + c)) return nrt + c;
    if (cfg_fits(h, kind, mvd_exact_cfg(kind))) return mvd_exact_cfg(kind);
    for (int c : {0, 1, 2, 3})
      if (cfg_fits(h, kind, c)) return c;
  }
  bad("no launch shape holds length " + std::to_string(h->max_len[kind]));
}

int total_tiles(const mvd_handle* h, int kind, int param) {
  int64_t t = 0;
  for (const auto& j : h->jobs) t += mvd_tiles(j, kind, param);
  if (t > 0x7fffffff) bad("too many tiles");
  return (int)t;
}

// Transform length of a pass kind in a block: x the half-row nx/2, y ny, z nz.
int job_len(const Block& B, int kind) { return kind == PASS_X ? B.M : kind == PASS_Y ? B.ny : B.nz; }

void build_jobs(mvd_handle* h) {
  h->jobs.clear();
  for (auto& B : h->blocks) {
    JobDesc j{};
    j.nx = B.nx;
    j.ny = B.ny;
    j.nz = B.nz;
    j.M = B.M;
    j.Mp = B.Mp;
    j.nviews = h->nviews;
    j.plan_x = h->plan_of_len.at(B.M);
    j.plan_y = h->plan_of_len.at(B.ny);
    j.plan_z = h->plan_of_len.at(B.nz);
    j.pp = h->pp_of_nx.at(B.nx);
    j.V = B.V;
    j.spec_main = B.spec_main;
    j.spec_elems = B.spec_elems;
    j.h_main = B.h_main;
    j.h_elems = B.h_elems;
    j.kz = B.kz;
    j.cz = B.cz;
    j.psi = B.psi;
    j.spec = B.spec;
    j.phi = B.phi;
    j.w = B.w;
    for (int r = 0; r < N_ROLES; ++r) j.H[r] = B.H[r];
    j.acc = B.acc;
    j.saved = B.saved;
    j.eps = B.eps;
    j.lamp = B.lamp;
    if (h->blocked) {
      // the block's grid is a window of the volume's estimate
      const auto& T = h->tl;
      const size_t b = h->jobs.size();
      j.vol = T.psi;
      j.vnx = T.dims[0], j.vny = T.dims[1], j.vnz = T.dims[2];
      j.sx = T.start[b][0], j.sy = T.start[b][1], j.sz = T.start[b][2];
      j.ox = T.origin[b][0], j.oy = T.origin[b][1], j.oz = T.origin[b][2];
      j.hx = T.halo[0], j.hy = T.halo[1], j.hz = T.halo[2];
      j.ex = T.extent[b][0], j.ey = T.extent[b][1], j.ez = T.extent[b][2];
    }
    h->jobs.push_back(j);
  }
  HIPCHECK(hipMemcpyAsync(h->d_jobs, h->jobs.data(), h->jobs.size() * sizeof(JobDesc), hipMemcpyHostToDevice,
                          h->stream));
  // block lanes: blocks of equal dims stay together (one launch per pass
  // serves them all); the groups go largest first onto the least loaded lane
  const int nb = (int)h->blocks.size();
  h->block_lane.assign(nb, 0);
  {
    std::map<std::array<int, 3>, std::vector<int>> same;
    for (int i = 0; i < nb; ++i) same[{h->blocks[i].nx, h->blocks[i].ny, h->blocks[i].nz}].push_back(i);
    std::vector<std::pair<int64_t, const std::vector<int>*>> groups;
    for (const auto& kv : same) groups.push_back({(int64_t)kv.second.size() * h->blocks[kv.second[0]].V, &kv.second});
    std::stable_sort(groups.begin(), groups.end(), [](const auto& a, const auto& b) { return a.first > b.first; });
    int64_t load[1 + mvd_handle::kSide] = {};
    for (const auto& g : groups) {
      int best = 0;
      for (int l = 1; l <= h->nside; ++l)
        if (load[l] < load[best]) best = l;
      for (int i : *g.second) h->block_lane[i] = best;
      load[best] += g.first;
    }
  }
  for (int k = 0; k < 3; ++k) {
    auto& ord = h->order[k];
    ord.resize(h->jobs.size());
    for (size_t i = 0; i < ord.size(); ++i) ord[i] = (int)i;
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
      const int la = h->block_lane[a], lb = h->block_lane[b];
      return la != lb ? la < lb : job_len(h->blocks[a], k) < job_len(h->blocks[b], k);
    });
    std::vector<JobDesc> sorted;
    for (int i : ord) sorted.push_back(h->jobs[i]);
    HIPCHECK(hipMemcpyAsync(h->d_jobs_k[k], sorted.data(), sorted.size() * sizeof(JobDesc), hipMemcpyHostToDevice,
                            h->stream));
  }
  HIPCHECK(hipStreamSynchronize(h->stream));
}

// Drop every cached graph (launch shapes, kernel spectra or the schedule
// changed).
void drop_graphs(mvd_handle* h) {
  bool any = false;
  for (auto& g : h->exec) any |= g != nullptr;
  if (any || !h->run_exec.empty()) HIPCHECK(hipStreamSynchronize(h->stream));
  for (auto& g : h->exec)
    if (g) {
      (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
  for (auto& kv : h->run_exec) (void)hipGraphExecDestroy(kv.second);
  h->run_exec.clear();
}

// Select the launch shapes of the three pass kinds; recomputes the grids,
// grows the partials buffer and drops the cached graphs.
bool cfg_fits(const mvd_handle* h, int kind, int c) {
  if (c < 0 || c >= mvd_num_cfgs(kind)) return false;
  // the block-wise form's x passes read and write the volume in place: the
  // per-length row kernels only
  if (h->blocked && kind == PASS_X && c != mvd_exact_cfg(kind)) return false;
  if (c == mvd_exact_cfg(kind)) {
    for (const auto& B : h->blocks)
      if (mvd_exact_param(kind, job_len(B, kind)) <= 0) return false;
    return true;
  }
  const int ex = mvd_cfg_exact(kind, c);
  if (ex > 0) return h->uniform_len[kind] == ex;
  return mvd_cfg_maxlen(kind, c) >= h->max_len[kind];
}

void set_tiles(mvd_handle* h, int cx, int cy, int cz) {
  const int c[3] = {cx, cy, cz};
  for (int k = 0; k < 3; ++k) {
    if (c[k] < 0 || c[k] >= mvd_num_cfgs(k)) bad("tile configuration index out of range");
    if (!cfg_fits(h, k, c[k])) bad("tile configuration does not fit the transform lengths of this handle");
  }
  int g[3];
  for (int k = 0; k < 3; ++k) {
    h->groups[k].clear();
    if (c[k] != mvd_exact_cfg(k)) {
      g[k] = total_tiles(h, k, mvd_cfg_param(k, c[k]));
      continue;
    }
    // groups of equal lane and length in the sorted job order
    // column passes of blocks of several lengths: groups of one length
    // class (one launch serves every length of the class)
    int64_t tiles = 0;
    const auto& ord = h->order[k];
    bool several = false;
    for (size_t i = 1; i < ord.size(); ++i)
      several |= job_len(h->blocks[ord[i]], k) != job_len(h->blocks[ord[0]], k);
    const bool by_class = k != PASS_X && several;
    auto key = [&](int b) { return by_class ? mvd_col_class(job_len(h->blocks[b], k)) : job_len(h->blocks[b], k); };
    for (size_t i = 0; i < ord.size();) {
      const int len = job_len(h->blocks[ord[i]], k);
      const int kv = key(ord[i]);
      const int lane = h->block_lane[ord[i]];
      const int param = mvd_exact_param(k, len);
      mvd_handle::Group gr{len, (int)i, 0, 0, (int)tiles, lane, by_class ? kv : -1};
      int64_t gt = 0;
      for (; i < ord.size() && key(ord[i]) == kv && h->block_lane[ord[i]] == lane; ++i) {
        gt += mvd_tiles(h->jobs[ord[i]], k, param);
        ++gr.njobs;
      }
      if (gt > 0x7fffffff) bad("too many tiles");
      gr.grid = (int)gt;
      tiles += gt;
      h->groups[k].push_back(gr);
    }
    if (tiles > 0x7fffffff) bad("too many tiles");
    g[k] = (int)tiles;
  }
  for (int k = 0; k < 3; ++k) {
    h->bgroups[k].clear();
    if (c[k] != mvd_exact_cfg(k)) continue;
    h->bgroups[k].resize(h->blocks.size());
    int64_t off = 0;
    const auto& ord = h->order[k];
    for (size_t i = 0; i < ord.size(); ++i) {
      const int b = ord[i];
      const int len = job_len(h->blocks[b], k);
      const int t = mvd_tiles(h->jobs[b], k, mvd_exact_param(k, len));
      h->bgroups[k][b] = mvd_handle::Group{len, (int)i, 1, t, (int)off, h->block_lane[b], -1};
      off += t;
    }
  }
  const int gx = g[0], gy = g[1], gz = g[2];
  if ((size_t)h->nviews * gx > h->parts_cap) {
    h->d_parts = (Partial*)h->dalloc((size_t)h->nviews * gx * sizeof(Partial));
    h->parts_cap = (size_t)h->nviews * gx;
    HIPCHECK(hipMemsetAsync(h->d_parts, 0, h->parts_cap * sizeof(Partial), h->stream));
  }
  drop_graphs(h);
  h->cfg_x = cx;
  h->cfg_y = cy;
  h->cfg_z = cz;
  h->grid_x = gx;
  h->grid_y = gy;
  h->grid_z = gz;
}

// Smallest 5-smooth length >= n (even when asked).
int next_smooth5(int n, bool even) {
  for (int m = std::max(n, 1);; ++m) {
    if (even && (m & 1)) continue;
    int k = m;
    for (int q : {2, 3, 5})
      while (k % q == 0) k /= q;
    if (k == 1) return m;
  }
}

const int* grid_dims(const Block& B) {
  thread_local int d[3];
  d[0] = B.nx;
  d[1] = B.ny;
  d[2] = B.nz;
  return d;
}
const int* user_dims(const Block& B) {
  thread_local int d[3];
  d[0] = B.ux;
  d[1] = B.uy;
  d[2] = B.uz;
  return d;
}
const int* offsets(const Block& B) {
  thread_local int d[3];
  d[0] = B.ox;
  d[1] = B.oy;
  d[2] = B.oz;
  return d;
}

void parse_options(mvd_handle* h, const mvd_options* o) {
  if (o) {
    if (!(o->lambda >= 0) || !std::isfinite(o->lambda)) bad("lambda must be finite and >= 0");
    if (!(o->eps_scale >= 0) || !std::isfinite(o->eps_scale)) bad("eps_scale must be finite and >= 0");
    if ((o->alloc == nullptr) != (o->free == nullptr)) bad("alloc and free callbacks come together");
    if (o->tile_config < 0) bad("tile_config must be >= 0");
    h->lambda = o->lambda;
    h->eps_scale = o->eps_scale > 0 ? o->eps_scale : 1e-6;
    h->stream = (hipStream_t)o->stream;
    h->alloc = o->alloc;
    h->free_fn = o->free;
    h->actx = o->alloc_ctx;
    h->use_graphs = o->use_graphs != 0;
    h->force_cfg = o->tile_config;
    if (o->boundary != MVD_BOUNDARY_CIRCULAR && o->boundary != MVD_BOUNDARY_LINEAR)
      bad("boundary must be MVD_BOUNDARY_CIRCULAR or MVD_BOUNDARY_LINEAR");
    h->linear = o->boundary == MVD_BOUNDARY_LINEAR;
  }
}

void make_streams(mvd_handle* h, int nb) {
  HIPCHECK(hipGetDevice(&h->device));
  if (h->no_alloc) {
    if (nb != 1) bad("the no-allocation run takes one volume");
    h->use_graphs = false;
  } else {
    HIPCHECK(hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
    // side lanes only where blocks can use them (the block-wise form keeps
    // its blocks on one stream)
    h->nside = h->blocked ? 0 : std::min(mvd_handle::kSide, nb - 1);
    for (int i = 0; i < h->nside; ++i) {
      HIPCHECK(hipStreamCreateWithFlags(&h->side[i], hipStreamNonBlocking));
      HIPCHECK(hipEventCreateWithFlags(&h->ev_join[i], hipEventDisableTiming));
    }
    HIPCHECK(hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming));
  }
}

// Geometry of a block's grid and its buffers (psi, spectrum, views, weights).
void alloc_block(mvd_handle* h, Block& B, bool weights) {
  const int N = h->nviews;
  B.M = B.nx / 2;
  B.Mp = (B.M + 15) & ~15;
  B.V = (int64_t)B.nx * B.ny * B.nz;
  B.spec_main = (int64_t)B.Mp * B.ny * B.nz;
  B.spec_elems = B.spec_main + (int64_t)B.ny * B.nz;
  // the block-wise form keeps its estimate in the volume only
  if (!h->blocked) B.psi = (float*)h->dalloc(B.V * sizeof(float));
  B.spec = (float*)h->dalloc(B.spec_elems * 2 * sizeof(float));
  B.phi = (float*)h->dalloc((size_t)N * B.V * sizeof(float));
  if (weights) B.w = (float*)h->dalloc((size_t)N * B.V * sizeof(float));
}

// FFT plans and twiddle tables of a block's lengths.
void add_plans(mvd_handle* h, const Block& B, std::vector<FftPlan>& plans, std::vector<float2>& tw) {
  plan_for(h, B.M, plans, tw);
  plan_for(h, B.ny, plans, tw);
  plan_for(h, B.nz, plans, tw);
  if (!h->pp_of_nx.count(B.nx)) {
    h->pp_of_nx[B.nx] = (int)tw.size();
    const auto t = mvdh::twiddles(B.nx);
    for (int k = 0; k < B.M; ++k) tw.push_back(make_float2((float)t[k].real(), (float)t[k].imag()));
  }
}

// The rest of a create once every block holds its inputs and kernel planes:
// plans and tables on the device, the job tables, launch shapes and the
// statistics buffers.
void finish_create(mvd_handle* h, std::vector<FftPlan>& plans, std::vector<float2>& tw) {
  const int nb = (int)h->blocks.size(), N = h->nviews;
  h->d_plans = (FftPlan*)h->dalloc(plans.size() * sizeof(FftPlan));
  h->d_tw = (float2*)h->dalloc(tw.size() * sizeof(float2));
  HIPCHECK(hipMemcpyAsync(h->d_plans, plans.data(), plans.size() * sizeof(FftPlan), hipMemcpyHostToDevice, h->stream));
  HIPCHECK(hipMemcpyAsync(h->d_tw, tw.data(), tw.size() * sizeof(float2), hipMemcpyHostToDevice, h->stream));
  h->d_jobs = (JobDesc*)h->dalloc(nb * sizeof(JobDesc));
  for (int k = 0; k < 3; ++k) h->d_jobs_k[k] = (JobDesc*)h->dalloc(nb * sizeof(JobDesc));

  int maxM = 0, maxY = 0, maxZ = 0;
  for (auto& B : h->blocks) {
    maxM = std::max(maxM, B.M);
    maxY = std::max(maxY, B.ny);
    maxZ = std::max(maxZ, B.nz);
  }
  build_jobs(h);
  h->max_len[PASS_X] = maxM;
  h->max_len[PASS_Y] = maxY;
  h->max_len[PASS_Z] = maxZ;
  h->uniform_len[PASS_X] = maxM;
  h->uniform_len[PASS_Y] = maxY;
  h->uniform_len[PASS_Z] = maxZ;
  for (auto& B : h->blocks) {
    if (B.M != maxM) h->uniform_len[PASS_X] = 0;
    if (B.ny != maxY) h->uniform_len[PASS_Y] = 0;
    if (B.nz != maxZ) h->uniform_len[PASS_Z] = 0;
  }
  set_tiles(h, pick_cfg(h, PASS_X), pick_cfg(h, PASS_Y), pick_cfg(h, PASS_Z));
  h->d_flags = (int*)h->dalloc(sizeof(int));
  h->d_flux = (double*)h->dalloc(N * sizeof(double));
  h->d_ratio = (unsigned long long*)h->dalloc(N * sizeof(unsigned long long));
  h->d_neg = (unsigned long long*)h->dalloc(N * sizeof(unsigned long long));
  HIPCHECK(hipMemsetAsync(h->d_flux, 0, N * sizeof(double), h->stream));
  HIPCHECK(hipMemsetAsync(h->d_ratio, 0, N * sizeof(unsigned long long), h->stream));
  HIPCHECK(hipMemsetAsync(h->d_neg, 0, N * sizeof(unsigned long long), h->stream));
  HIPCHECK(mvd_launch_set_int(h->d_flags, 0, h->stream));
  HIPCHECK(hipStreamSynchronize(h->stream));
  h->spec_valid = false;
}

void create_impl(mvd_handle* h, int nb, const mvd_problem* ps, const mvd_options* o) {
  if (nb < 1) bad("n_blocks must be >= 1");
  if (!ps) bad("problem is NULL");
  for (int b = 0; b < nb; ++b) validate_shape(&ps[b], b);
  for (int b = 1; b < nb; ++b)
    if (ps[b].n_views != ps[0].n_views) bad("every block needs the same number of views");
  parse_options(h, o);
  h->nviews = ps[0].n_views;
  // host-memory values are checked before any device call
  std::vector<std::vector<mvdh::Kern>> prepared(nb);
  for (int b = 0; b < nb; ++b) {
    if (ps[b].mem_kind == MVD_MEM_HOST) {
      validate_host_values(&ps[b], b);
      for (int v = 0; v < ps[b].n_views; ++v) {
        const int* k = ps[b].psf_dims + 3 * v;
        try {
          prepared[b].push_back(mvdh::prepare_psf(ps[b].psfs[v], k[0], k[1], k[2]));
        } catch (const std::invalid_argument& e) {
          bad("block " + std::to_string(b) + " PSF " + std::to_string(v) + ": " + e.what());
        }
      }
    }
  }

  make_streams(h, nb);

  std::vector<FftPlan> plans;
  std::vector<float2> tw;
  h->blocks.resize(nb);
  const int N = h->nviews;
  for (int b = 0; b < nb; ++b) {
    const mvd_problem& p = ps[b];
    Block& B = h->blocks[b];
    B.ux = B.nx = p.dims[0];
    B.uy = B.ny = p.dims[1];
    B.uz = B.nz = p.dims[2];
    B.UV = vox(p.dims);
    if (h->linear) {
      // the largest PSF radius per axis (odd-padded extents), and the grid
      // that holds the volume plus that margin on both sides
      int r[3] = {0, 0, 0};
      for (int v = 0; v < N; ++v)
        for (int a = 0; a < 3; ++a) r[a] = std::max(r[a], (p.psf_dims[3 * v + a] | 1) / 2);
      B.ox = r[0];
      B.oy = r[1];
      B.oz = r[2];
      B.nx = next_smooth5(B.ux + 2 * r[0], true);
      B.ny = next_smooth5(B.uy + 2 * r[1], false);
      B.nz = next_smooth5(B.uz + 2 * r[2], false);
      if (B.nx / 2 > MVD_MAX_LEN || B.ny > MVD_MAX_LEN_YZ || B.nz > MVD_MAX_LEN_YZ)
        bad("block " + std::to_string(b) + ": the volume plus its PSF margin exceeds the largest transform length");
    }
    alloc_block(h, B, p.weights != nullptr);
    const hipMemcpyKind kind = p.mem_kind == MVD_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    if (!h->linear) {
      for (int v = 0; v < N; ++v) {
        HIPCHECK(hipMemcpyAsync(B.phi + (size_t)v * B.V, p.views[v], B.V * sizeof(float), kind, h->stream));
        if (p.weights)
          HIPCHECK(hipMemcpyAsync(B.w + (size_t)v * B.V, p.weights[v], B.V * sizeof(float), kind, h->stream));
      }
    } else {
      // views are zero (until the value checks below) and weights one
      // outside the volume; host inputs pass through the (not yet used)
      // estimate buffer
      HIPCHECK(mvd_launch_fill(B.phi, (int64_t)N * B.V, 0.f, h->stream));
      if (p.weights) HIPCHECK(mvd_launch_fill(B.w, (int64_t)N * B.V, 1.f, h->stream));
      auto put = [&](float* grid, const float* src) {
        const float* from = src;
        if (p.mem_kind == MVD_MEM_HOST) {
          HIPCHECK(hipMemcpyAsync(B.psi, src, B.UV * sizeof(float), hipMemcpyHostToDevice, h->stream));
          from = B.psi;
        }
        HIPCHECK(mvd_launch_embed(grid, grid_dims(B), from, user_dims(B), offsets(B), h->stream));
      };
      for (int v = 0; v < N; ++v) {
        put(B.phi + (size_t)v * B.V, p.views[v]);
        if (p.weights) put(B.w + (size_t)v * B.V, p.weights[v]);
      }
    }
    // FP64 mean over all views, plus the value checks of device inputs
    double total = 0;
    for (int v = 0; v < N; ++v) {
      double s;
      unsigned long long nbad;
      device_check(h, B.phi + (size_t)v * B.V, B.V, 0.f, INFINITY, &s, &nbad);
      if (nbad) bad("block " + std::to_string(b) + ": view " + std::to_string(v) + " has a negative or non-finite value");
      total += s;
      if (p.weights) {
        device_check(h, B.w + (size_t)v * B.V, B.V, 0.f, 1.f, &s, &nbad);
        if (nbad) bad("block " + std::to_string(b) + ": weights " + std::to_string(v) + " outside [0, 1]");
      }
    }
    B.s = total / ((double)N * (double)B.UV);
    if (!(B.s > 0)) bad("block " + std::to_string(b) + ": the views are all zero");
    // linear boundary: outside the volume a view has no data (the ratio pass
    // takes q = 1 there)
    if (h->linear)
      for (int v = 0; v < N; ++v)
        HIPCHECK(mvd_launch_fill_outside(B.phi + (size_t)v * B.V, grid_dims(B), user_dims(B), offsets(B), MVD_NO_DATA,
                                         h->stream));
    B.eps = ratio_guard(h, B.s);
    B.lamp = (float)(h->lambda / B.s);
    if (p.mem_kind == MVD_MEM_DEVICE) {
      for (int v = 0; v < N; ++v) {
        const int* k = p.psf_dims + 3 * v;
        const auto hp = fetch_psf(&p, v);
        try {
          prepared[b].push_back(mvdh::prepare_psf(hp.data(), k[0], k[1], k[2]));
        } catch (const std::invalid_argument& e) {
          bad("block " + std::to_string(b) + " PSF " + std::to_string(v) + ": " + e.what());
        }
      }
    }
    B.P = std::move(prepared[b]);
    for (int v = 0; v < N; ++v) {
      const int* k = p.psf_dims + 3 * v;
      B.psf_dims.push_back({k[0], k[1], k[2]});
    }
    if (p.mem_kind == MVD_MEM_HOST) {
      for (int v = 0; v < N; ++v) {
        const int* k = p.psf_dims + 3 * v;
        double sum = 0;
        for (size_t i = 0; i < (size_t)k[0] * k[1] * k[2]; ++i) sum += p.psfs[v][i];
        B.psf_sum.push_back(sum);
      }
    } else {
      for (int v = 0; v < N; ++v) {
        const auto hp = fetch_psf(&p, v);
        double sum = 0;
        for (float x : hp) sum += x;
        B.psf_sum.push_back(sum);
      }
    }
    set_kernel_window(B);
    B.kz_cap = B.kz;
    B.H[ROLE_P] = (float*)h->dalloc((size_t)N * B.h_elems * 2 * sizeof(float));
    for (int v = 0; v < N; ++v) upload_kernel(h, B, B.P[v], B.H[ROLE_P] + (size_t)v * B.h_elems * 2);
    add_plans(h, B, plans, tw);
    HIPCHECK(mvd_launch_fill(B.psi, B.V, (float)B.s, h->stream));
  }
  finish_create(h, plans, tw);
}

// Block-wise form (main text: processing in blocks to reduce memory; the
// implementation section's copying and pasting of blocks).  The volume may
// have any extents: only the blocks' grids are transformed.  Blocks per axis
// are near-equal (origins k n / t); every block computes on one grid of the
// largest block plus the halo on both sides, rounded up to a transform
// length.  A halo of twice the largest PSF radius (the default) leaves the
// pasted voxels equal to the whole-volume update.
void create_blocked_impl(mvd_handle* h, const mvd_problem* p, const mvd_options* o, const int* tiles,
                         const int* halo) {
  if (!p) bad("problem is NULL");
  parse_options(h, o);
  if (h->linear) bad("the block-wise form runs with the circular boundary");
  const int N = p->n_views;
  if (N < 1 || N > MVD_MAX_VIEWS) bad("n_views must be in [1, 64]");
  if (!p->views || !p->psfs || !p->psf_dims) bad("views, psfs and psf_dims are required");
  if (p->mem_kind != MVD_MEM_HOST && p->mem_kind != MVD_MEM_DEVICE) bad("mem_kind must be host or device");
  auto& T = h->tl;
  for (int a = 0; a < 3; ++a) {
    T.dims[a] = p->dims[a];
    if (T.dims[a] < 1) bad("extents must be >= 1");
  }
  T.V = vox(T.dims);
  int R[3] = {0, 0, 0}, kmax[3] = {1, 1, 1};
  for (int v = 0; v < N; ++v) {
    if (!p->views[v] || !p->psfs[v]) bad("view or PSF pointer " + std::to_string(v) + " is NULL");
    if (p->weights && !p->weights[v]) bad("weight pointer " + std::to_string(v) + " is NULL");
    const int* k = p->psf_dims + 3 * v;
    for (int a = 0; a < 3; ++a) {
      if (k[a] < 1) bad("PSF extents must be >= 1");
      R[a] = std::max(R[a], (k[a] | 1) / 2);
      kmax[a] = std::max(kmax[a], k[a] | 1);
    }
  }
  const int lim[3] = {2 * MVD_MAX_LEN, MVD_MAX_LEN_YZ, MVD_MAX_LEN_YZ};
  const int lim_fast[3] = {1024, 512, 512};
  int G[3];
  for (int a = 0; a < 3; ++a) {
    T.halo[a] = halo ? halo[a] : 2 * R[a];
    if (T.halo[a] < 0) bad("halo must be >= 0");
    const int n = T.dims[a];
    // one block along an axis whose extent is a transform length: the grid
    // is the volume's period itself, exact without a halo
    const bool period = n >= kmax[a] && n >= (a == 0 ? 8 : 2) && next_smooth5(n, a == 0) == n;
    auto halo_for = [&](int t) { return !halo && t == 1 && period ? 0 : T.halo[a]; };
    auto grid_for = [&](int t) {
      const int ext = (n + t - 1) / t;
      const int g = std::max({ext + 2 * halo_for(t), kmax[a], a == 0 ? 8 : 2});
      return next_smooth5(g, a == 0);
    };
    int t = tiles ? tiles[a] : 0;
    if (t < 0 || t > n) bad("blocks per axis must be in [0, the extent] (0: as few as the transform lengths allow)");
    if (t == 0) {
      // the fewest blocks whose grid keeps half-rows and columns within 512
      // points (the kernels with the most lines per tile), else the fewest
      // whose grid fits the transform lengths
      t = 1;
      while (t < n && grid_for(t) > lim_fast[a]) ++t;
      if (grid_for(t) > lim_fast[a]) {
        t = 1;
        while (t < n && grid_for(t) > lim[a]) ++t;
      }
    }
    T.halo[a] = halo_for(t);
    G[a] = grid_for(t);
    if (G[a] > lim[a])
      bad("a block's grid (the block plus the halo on both sides) exceeds the largest transform length along axis " +
          std::to_string(a) + ": more blocks or a thinner halo");
    T.tiles[a] = t;
  }
  const int nb = T.tiles[0] * T.tiles[1] * T.tiles[2];
  for (int bz = 0; bz < T.tiles[2]; ++bz)
    for (int by = 0; by < T.tiles[1]; ++by)
      for (int bx = 0; bx < T.tiles[0]; ++bx) {
        const int k[3] = {bx, by, bz};
        std::array<int, 3> org, ext, st;
        for (int a = 0; a < 3; ++a) {
          const int64_t n = T.dims[a], t = T.tiles[a];
          org[a] = (int)(k[a] * n / t);
          ext[a] = (int)((k[a] + 1) * n / t) - org[a];
          st[a] = (int)((((int64_t)org[a] - T.halo[a]) % n + n) % n);
        }
        T.origin.push_back(org);
        T.extent.push_back(ext);
        T.start.push_back(st);
      }
  h->blocked = true;
  h->shared_kernels = true;
  h->nviews = N;

  // host values and PSFs before any device call
  std::vector<mvdh::Kern> prepared;
  std::vector<double> psf_sum;
  if (p->mem_kind == MVD_MEM_HOST) validate_host_values(p, 0);
  make_streams(h, nb);
  for (int v = 0; v < N; ++v) {
    const int* k = p->psf_dims + 3 * v;
    const auto hp = fetch_psf(p, v);
    try {
      prepared.push_back(mvdh::prepare_psf(hp.data(), k[0], k[1], k[2]));
    } catch (const std::invalid_argument& e) {
      bad("PSF " + std::to_string(v) + ": " + e.what());
    }
    double sum = 0;
    for (float x : hp) sum += x;
    psf_sum.push_back(sum);
  }

  T.psi = (float*)h->dalloc(T.V * sizeof(float));
  h->blocks.resize(nb);
  for (auto& B : h->blocks) {
    B.nx = B.ux = G[0];
    B.ny = B.uy = G[1];
    B.nz = B.uz = G[2];
    B.UV = (int64_t)G[0] * G[1] * G[2];
    alloc_block(h, B, p->weights != nullptr);
  }
  // every view and weight volume through the staging estimate buffer (host
  // inputs) into the windows of every block; s over the volume
  double total = 0;
  for (int v = 0; v < N; ++v) {
    for (int wgt = 0; wgt < (p->weights ? 2 : 1); ++wgt) {
      const float* src = wgt ? p->weights[v] : p->views[v];
      if (p->mem_kind == MVD_MEM_HOST) {
        HIPCHECK(hipMemcpyAsync(T.psi, src, T.V * sizeof(float), hipMemcpyHostToDevice, h->stream));
        src = T.psi;
      }
      double sum;
      unsigned long long nbad;
      device_check(h, src, T.V, 0.f, wgt ? 1.f : INFINITY, &sum, &nbad);
      if (nbad)
        bad(wgt ? "weights " + std::to_string(v) + " outside [0, 1]"
                : "view " + std::to_string(v) + " has a negative or non-finite value");
      if (!wgt) total += sum;
      for (int b = 0; b < nb; ++b) {
        Block& B = h->blocks[b];
        float* dst = (wgt ? B.w : B.phi) + (size_t)v * B.V;
        HIPCHECK(mvd_launch_gather(dst, grid_dims(B), src, T.dims, T.start[b].data(), h->stream));
      }
    }
  }
  const double s = total / ((double)N * (double)T.V);
  if (!(s > 0)) bad("the views are all zero");
  std::vector<FftPlan> plans;
  std::vector<float2> tw;
  for (int b = 0; b < nb; ++b) {
    Block& B = h->blocks[b];
    B.s = s;
    B.eps = ratio_guard(h, s);
    B.lamp = (float)(h->lambda / s);
    B.P = prepared;
    B.psf_sum = psf_sum;
    for (int v = 0; v < N; ++v) {
      const int* k = p->psf_dims + 3 * v;
      B.psf_dims.push_back({k[0], k[1], k[2]});
    }
    set_kernel_window(B);
    B.kz_cap = B.kz;
    if (b == 0) {
      B.H[ROLE_P] = (float*)h->dalloc((size_t)N * B.h_elems * 2 * sizeof(float));
      for (int v = 0; v < N; ++v) upload_kernel(h, B, B.P[v], B.H[ROLE_P] + (size_t)v * B.h_elems * 2);
    } else {
      B.H[ROLE_P] = h->blocks[0].H[ROLE_P];
    }
    add_plans(h, B, plans, tw);
  }
  HIPCHECK(mvd_launch_fill(T.psi, T.V, (float)s, h->stream));
  finish_create(h, plans, tw);
}

void ensure_role(mvd_handle* h, int role) {
  if (h->built[role]) return;
  const int variant = role;  // ROLE_EFF == MVD_EFF etc.
  for (auto& B : h->blocks) {
    if (h->shared_kernels && &B != &h->blocks[0]) {
      B.H[role] = h->blocks[0].H[role];
      continue;
    }
    if (!B.H[role]) B.H[role] = (float*)h->dalloc((size_t)h->nviews * B.h_elems * 2 * sizeof(float));
    const auto K = mvdh::compound_kernels(B.P, variant);
    for (int v = 0; v < h->nviews; ++v) upload_kernel(h, B, K[v], B.H[role] + (size_t)v * B.h_elems * 2);
  }
  build_jobs(h);
  h->built[role] = true;
}

LaunchArgs args(mvd_handle* h, hipStream_t s, int grid) {
  LaunchArgs a;
  a.jobs = h->d_jobs;
  a.njobs = (int)h->jobs.size();
  a.plans = h->d_plans;
  a.tw = h->d_tw;
  a.stream = s;
  a.grid = grid;
  return a;
}

// One pass of each kind with the handle's launch shape: one launch over all
// jobs, or with the per-length compile-time plans one launch per group of
// jobs of equal length (x partials of a group start at its tile offset).
LaunchArgs group_args(mvd_handle* h, hipStream_t s, int kind, const mvd_handle::Group& g) {
  LaunchArgs a = args(h, s, g.grid);
  a.jobs = h->d_jobs_k[kind] + g.first;
  a.njobs = g.njobs;
  return a;
}

// The groups of one pass: each on its lane's stream; side lanes are forked
// from s by an event and joined back before the pass is complete, so the
// next pass on s sees every group's writes.  Under defer_join the side
// streams were forked before the sequence and are joined after it.
template <class F>
void run_groups(mvd_handle* h, hipStream_t s, int kind, F&& launch) {
  if (h->defer_join) {
    for (const auto& g : h->groups[kind]) HIPCHECK(launch(g, g.lane ? h->side[g.lane - 1] : s));
    return;
  }
  unsigned used = 0;
  for (const auto& g : h->groups[kind]) used |= 1u << g.lane;
  const bool fork = (used & ~1u) != 0;
  if (fork) {
    HIPCHECK(hipEventRecord(h->ev_fork, s));
    for (int l = 1; l <= h->nside; ++l)
      if (used & (1u << l)) HIPCHECK(hipStreamWaitEvent(h->side[l - 1], h->ev_fork, 0));
  }
  for (const auto& g : h->groups[kind]) HIPCHECK(launch(g, g.lane ? h->side[g.lane - 1] : s));
  if (fork) {
    for (int l = 1; l <= h->nside; ++l)
      if (used & (1u << l)) {
        HIPCHECK(hipEventRecord(h->ev_join[l - 1], h->side[l - 1]));
        HIPCHECK(hipStreamWaitEvent(s, h->ev_join[l - 1], 0));
      }
  }
}

void run_x(mvd_handle* h, hipStream_t s, int mode, int v, Partial* parts, int opt) {
  // the block-wise form's forward and update passes work on the volume
  if (h->blocked && (mode == 0 || mode == 2)) mode |= XMODE_WIN;
  if (h->cfg_x != mvd_exact_cfg(PASS_X)) {
    HIPCHECK(mvd_launch_x(args(h, s, h->grid_x), h->cfg_x, mode, v, parts, h->d_flags, opt));
    return;
  }
  run_groups(h, s, PASS_X, [&](const mvd_handle::Group& g, hipStream_t st) {
    return mvd_launch_x_exact(group_args(h, st, PASS_X, g), g.len, mode, v, parts ? parts + g.part_off : nullptr,
                              h->d_flags, opt);
  });
}

void run_y(mvd_handle* h, hipStream_t s, int inv, int v) {
  if (h->cfg_y != mvd_exact_cfg(PASS_Y)) {
    HIPCHECK(mvd_launch_y(args(h, s, h->grid_y), h->cfg_y, inv, v));
    return;
  }
  run_groups(h, s, PASS_Y, [&](const mvd_handle::Group& g, hipStream_t st) {
    return g.cls >= 0 ? mvd_launch_y_class(group_args(h, st, PASS_Y, g), g.cls, inv, v)
                      : mvd_launch_y_exact(group_args(h, st, PASS_Y, g), g.len, inv, v);
  });
}

void run_z(mvd_handle* h, hipStream_t s, int v, int role, int conjH, int src_saved) {
  if (h->cfg_z != mvd_exact_cfg(PASS_Z)) {
    HIPCHECK(mvd_launch_z(args(h, s, h->grid_z), h->cfg_z, v, role, conjH, src_saved));
    return;
  }
  run_groups(h, s, PASS_Z, [&](const mvd_handle::Group& g, hipStream_t st) {
    return g.cls >= 0 ? mvd_launch_z_class(group_args(h, st, PASS_Z, g), g.cls, v, role, conjH, src_saved)
                      : mvd_launch_z_exact(group_args(h, st, PASS_Z, g), g.len, v, role, conjH, src_saved);
  });
}

// Per-launch event timing of the passes (profiling hook): kinds are
// 0 y forward, 1 y inverse, 2 z product, 3 x ratio, 4 x update.
struct PassTimer {
  std::vector<hipEvent_t> ev;
  std::vector<int> kind;
  hipStream_t s = nullptr;
  void mark(int k) {
    hipEvent_t a, b;
    HIPCHECK(hipEventCreate(&a));
    HIPCHECK(hipEventCreate(&b));
    ev.push_back(a);
    ev.push_back(b);
    kind.push_back(k);
    HIPCHECK(hipEventRecord(a, s));
  }
  void done() { HIPCHECK(hipEventRecord(ev.back(), s)); }
  ~PassTimer() {
    for (auto e : ev) (void)hipEventDestroy(e);
  }
};

// One view-update of view v: two convolutions and the pointwise steps;
// spec_out: the update pass also writes the x-stage spectrum of the new psi
// (the input of the next view's blur).
void enqueue_view_passes(mvd_handle* h, hipStream_t s, int variant, int v, PassTimer* t, bool spec_out) {
  const int role = variant == MVD_RL ? ROLE_P : variant;
  const int conj_back = variant == MVD_RL ? 1 : 0;
  Partial* parts = h->d_parts + (size_t)v * h->grid_x;
  auto timed = [&](int kind, auto&& fn) {
    if (t) t->mark(kind);
    fn();
    if (t) t->done();
  };
  // b = psi (x) P_v, then q = phi_v / max(b, eps)
  timed(0, [&] { run_y(h, s, 0, v); });
  timed(2, [&] { run_z(h, s, v, ROLE_P, 0, 0); });
  timed(1, [&] { run_y(h, s, 1, v); });
  timed(3, [&] { run_x(h, s, 1, v, parts, XOPT_SPEC); });
  // c = q (x) K_v, then the update of psi
  timed(0, [&] { run_y(h, s, 0, v); });
  timed(2, [&] { run_z(h, s, v, role, conj_back, 0); });
  timed(1, [&] { run_y(h, s, 1, v); });
  timed(4, [&] { run_x(h, s, 2, v, parts, spec_out ? XOPT_SPEC : 0); });
}

// One view-update; with the block-wise form every block first transforms
// its window of the volume's estimate along x (read in place), and its
// update pass writes the block's own voxels into the volume.  Every block's
// window is read before any block writes (the x pass over all blocks
// precedes the update pass in stream order), and the own voxels of the
// blocks are disjoint.
void enqueue_view(mvd_handle* h, hipStream_t s, int variant, int v, PassTimer* t = nullptr) {
  if (!h->blocked) {
    enqueue_view_passes(h, s, variant, v, t, true);
    return;
  }
  run_x(h, s, 0, 0, nullptr, XOPT_SPEC);
  enqueue_view_passes(h, s, variant, v, t, false);
}

// One iteration: every view once, in index order (section 7).  When every
// pass kind runs in groups and blocks sit on several lanes, each lane's
// blocks go through all view-updates on their own stream, joined once at
// the end (blocks are independent; stream order keeps each block's passes
// in sequence).
void enqueue_iteration(mvd_handle* h, hipStream_t s, int variant, PassTimer* t = nullptr) {
  bool lanes = false;
  for (int l : h->block_lane) lanes |= l != 0;
  const bool grouped = h->cfg_x == mvd_exact_cfg(PASS_X) && h->cfg_y == mvd_exact_cfg(PASS_Y) &&
                       h->cfg_z == mvd_exact_cfg(PASS_Z);
  if (!lanes || !grouped || t) {
    for (int v = 0; v < h->nviews; ++v) enqueue_view(h, s, variant, v, t);
    return;
  }
  HIPCHECK(hipEventRecord(h->ev_fork, s));
  for (int l = 0; l < h->nside; ++l) HIPCHECK(hipStreamWaitEvent(h->side[l], h->ev_fork, 0));
  h->defer_join = true;
  try {
    for (int v = 0; v < h->nviews; ++v) enqueue_view(h, s, variant, v, nullptr);
  } catch (...) {
    h->defer_join = false;
    throw;
  }
  h->defer_join = false;
  for (int l = 0; l < h->nside; ++l) {
    HIPCHECK(hipEventRecord(h->ev_join[l], h->side[l]));
    HIPCHECK(hipStreamWaitEvent(s, h->ev_join[l], 0));
  }
}

// One view-update of block b alone on stream s (the block-major schedules):
// every pass launches the per-length plan over that block only.
void enqueue_view_block(mvd_handle* h, hipStream_t s, int variant, int v, int b) {
  const int role = variant == MVD_RL ? ROLE_P : variant;
  const int conj_back = variant == MVD_RL ? 1 : 0;
  Partial* parts = h->d_parts + (size_t)v * h->grid_x;
  const auto& gx = h->bgroups[PASS_X][b];
  const auto& gy = h->bgroups[PASS_Y][b];
  const auto& gz = h->bgroups[PASS_Z][b];
  auto y = [&](int inv) { HIPCHECK(mvd_launch_y_exact(group_args(h, s, PASS_Y, gy), gy.len, inv, v)); };
  auto z = [&](int r, int cj) {
    HIPCHECK(mvd_launch_z_exact(group_args(h, s, PASS_Z, gz), gz.len, v, r, cj, 0));
  };
  auto x = [&](int mode) {
    HIPCHECK(mvd_launch_x_exact(group_args(h, s, PASS_X, gx), gx.len, mode, v, parts + gx.part_off, h->d_flags,
                                XOPT_SPEC));
  };
  y(0);
  z(ROLE_P, 0);
  y(1);
  x(1);
  y(0);
  z(role, conj_back);
  y(1);
  x(2);
}

bool block_major(const mvd_handle* h) {
  if (h->schedule == MVD_SCHEDULE_PASS_MAJOR || h->blocks.size() < 2 || h->blocked || h->no_alloc) return false;
  for (int k = 0; k < 3; ++k)
    if (h->bgroups[k].size() != h->blocks.size()) return false;
  return true;
}

// n iterations with a block-major schedule: every lane's stream takes its
// blocks one at a time (MVD_SCHEDULE_BLOCK_MAJOR: each block's view-updates
// of one iteration, then the next block; MVD_SCHEDULE_RUN_MAJOR: all n
// iterations of a block, then the next), so the few blocks in flight, one
// per lane, keep their spectra, views and estimates in the memory-side
// cache from pass to pass.  Blocks are independent, so any such order gives
// the same results; the lanes are forked once and joined at the end.
void enqueue_run_blocks(mvd_handle* h, hipStream_t s, int variant, int n) {
  HIPCHECK(hipEventRecord(h->ev_fork, s));
  for (int l = 0; l < h->nside; ++l) HIPCHECK(hipStreamWaitEvent(h->side[l], h->ev_fork, 0));
  for (int l = 0; l <= h->nside; ++l) {
    hipStream_t sl = l ? h->side[l - 1] : s;
    std::vector<int> mine;
    for (int b = 0; b < (int)h->blocks.size(); ++b)
      if (h->block_lane[b] == l) mine.push_back(b);
    if (h->schedule == MVD_SCHEDULE_RUN_MAJOR) {
      for (int b : mine)
        for (int i = 0; i < n; ++i)
          for (int v = 0; v < h->nviews; ++v) enqueue_view_block(h, sl, variant, v, b);
    } else {
      for (int i = 0; i < n; ++i)
        for (int b : mine)
          for (int v = 0; v < h->nviews; ++v) enqueue_view_block(h, sl, variant, v, b);
    }
  }
  for (int l = 0; l < h->nside; ++l) {
    HIPCHECK(hipEventRecord(h->ev_join[l], h->side[l]));
    HIPCHECK(hipStreamWaitEvent(s, h->ev_join[l], 0));
  }
}

// One combined update (eq. 51): every view's back-projected ratio is taken
// from the same psi.  The x/y-stage spectrum of psi is computed once and
// saved; per view the blur's z pass reads it, the ratio and the
// back-projection follow as in a view-update, and the back-projected ratio
// is folded into the factor acc; the last view's x pass applies the update
// and leaves the x-stage spectrum of the new psi for the next iteration.
void enqueue_combined_iteration(mvd_handle* h, hipStream_t s, int variant, bool geo) {
  const int role = variant == MVD_RL ? ROLE_P : variant;
  const int conj_back = variant == MVD_RL ? 1 : 0;
  const int N = h->nviews;
  run_y(h, s, 0, 0);
  for (const auto& B : h->blocks)
    HIPCHECK(hipMemcpyAsync(B.saved, B.spec, B.spec_elems * 2 * sizeof(float), hipMemcpyDeviceToDevice, s));
  const int mean = geo ? XOPT_GEO : 0;
  for (int v = 0; v < N; ++v) {
    Partial* parts = h->d_parts + (size_t)v * h->grid_x;
    run_z(h, s, v, ROLE_P, 0, 1);
    run_y(h, s, 1, v);
    run_x(h, s, 1, v, parts, XOPT_SPEC);
    run_y(h, s, 0, v);
    run_z(h, s, v, role, conj_back, 0);
    run_y(h, s, 1, v);
    const int first = v == 0 ? XOPT_FIRST : 0;
    if (v < N - 1)
      run_x(h, s, 3, v, parts, first | mean);
    else
      run_x(h, s, 4, v, parts, first | mean | XOPT_SPEC);
  }
}

void ensure_combined(mvd_handle* h) {
  bool grown = false;
  for (auto& B : h->blocks) {
    if (!B.acc) {
      B.acc = (float*)h->dalloc(B.V * sizeof(float));
      grown = true;
    }
    if (!B.saved) {
      B.saved = (float*)h->dalloc(B.spec_elems * 2 * sizeof(float));
      grown = true;
    }
  }
  if (grown) build_jobs(h);
}

void prepare_run(mvd_handle* h, int variant) {
  if (variant < MVD_RL || variant > MVD_OPT2) bad("variant must be MVD_RL, MVD_EFF, MVD_OPT1 or MVD_OPT2");
  const int role = variant == MVD_RL ? ROLE_P : variant;
  ensure_role(h, role);
  if (!h->spec_valid && !h->blocked) {
    run_x(h, h->stream, 0, 0, nullptr, XOPT_SPEC);
    h->spec_valid = true;
  }
}

// scheme 0: sequential; 1, 2: combined with the geometric / arithmetic mean
hipGraphExec_t graph_for(mvd_handle* h, int variant, int scheme = 0) {
  hipGraphExec_t& slot = h->exec[scheme * 4 + variant];
  if (slot) return slot;
  hipGraph_t g = nullptr;
  HIPCHECK(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
  try {
    if (scheme == 0)
      enqueue_iteration(h, h->cap, variant);
    else
      enqueue_combined_iteration(h, h->cap, variant, scheme == 1);
  } catch (...) {
    (void)hipStreamEndCapture(h->cap, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  HIPCHECK(hipStreamEndCapture(h->cap, &g));
  hipGraphExec_t ex = nullptr;
  hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  HIPCHECK(e);
  slot = ex;
  return ex;
}

// Statistics of the last iteration from the partial results (the block-wise
// form's update passes count and sum the own voxels of every block).
void reduce_stats(mvd_handle* h, hipStream_t s) {
  HIPCHECK(mvd_launch_reduce(h->d_parts, h->grid_x, h->nviews, h->d_flux, h->d_ratio, h->d_neg, s));
}

// The graph of a whole block-major run of n iterations (one launch per run).
hipGraphExec_t run_graph_for(mvd_handle* h, int variant, int n) {
  const auto key = std::make_pair(variant, n);
  auto it = h->run_exec.find(key);
  if (it != h->run_exec.end()) return it->second;
  hipGraph_t g = nullptr;
  HIPCHECK(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
  try {
    enqueue_run_blocks(h, h->cap, variant, n);
  } catch (...) {
    (void)hipStreamEndCapture(h->cap, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  HIPCHECK(hipStreamEndCapture(h->cap, &g));
  hipGraphExec_t ex = nullptr;
  hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  HIPCHECK(e);
  // a few run lengths are kept (a caller stepping through n = 1, 2, ...
  // would otherwise grow the cache without bound)
  if (h->run_exec.size() >= 4) {
    HIPCHECK(hipStreamSynchronize(h->stream));
    for (auto& kv : h->run_exec) (void)hipGraphExecDestroy(kv.second);
    h->run_exec.clear();
  }
  h->run_exec[key] = ex;
  return ex;
}

void iterate_impl(mvd_handle* h, int n, int variant) {
  if (variant < MVD_RL || variant > MVD_OPT2) bad("variant must be MVD_RL, MVD_EFF, MVD_OPT1 or MVD_OPT2");
  if (n < 0) bad("n must be >= 0");
  if (n == 0) return;
  h->rec_token = 0;
  prepare_run(h, variant);
  if (block_major(h)) {
    if (h->use_graphs)
      HIPCHECK(hipGraphLaunch(run_graph_for(h, variant, n), h->stream));
    else
      enqueue_run_blocks(h, h->stream, variant, n);
  } else if (h->use_graphs) {
    hipGraphExec_t ex = graph_for(h, variant);
    for (int i = 0; i < n; ++i) HIPCHECK(hipGraphLaunch(ex, h->stream));
  } else {
    for (int i = 0; i < n; ++i) enqueue_iteration(h, h->stream, variant);
  }
  reduce_stats(h, h->stream);
  h->iterations += n;
}

void iterate_combined_impl(mvd_handle* h, int n, int variant, int mean) {
  h->rec_token = 0;
  if (variant < MVD_RL || variant > MVD_OPT2) bad("variant must be MVD_RL, MVD_EFF, MVD_OPT1 or MVD_OPT2");
  if (mean != MVD_MEAN_GEOMETRIC && mean != MVD_MEAN_ARITHMETIC) bad("mean must be MVD_MEAN_GEOMETRIC or MVD_MEAN_ARITHMETIC");
  if (n < 0) bad("n must be >= 0");
  if (h->linear) throw Error(MVD_ESTATE, "combined updates run with the circular boundary only");
  if (h->blocked) throw Error(MVD_ESTATE, "combined updates run on whole volumes only");
  for (const auto& B : h->blocks)
    if (B.w) bad("combined updates take no weights (weights apply to sequential view-updates)");
  if (n == 0) return;
  prepare_run(h, variant);
  ensure_combined(h);
  const bool geo = mean == MVD_MEAN_GEOMETRIC;
  if (h->use_graphs) {
    hipGraphExec_t ex = graph_for(h, variant, geo ? 1 : 2);
    for (int i = 0; i < n; ++i) HIPCHECK(hipGraphLaunch(ex, h->stream));
  } else {
    for (int i = 0; i < n; ++i) enqueue_combined_iteration(h, h->stream, variant, geo);
  }
  HIPCHECK(mvd_launch_reduce(h->d_parts, h->grid_x, h->nviews, h->d_flux, h->d_ratio, h->d_neg, h->stream));
  h->iterations += n;
}

// ---- differentiated form -------------------------------------------------

void grad_setup(mvd_handle* h, int n) {
  const Block& B = h->blocks[0];
  if (!h->grad_ready) {
    // runtime-plan shapes only for the passes no compile-time plan serves:
    // the adjoint x passes of half-rows that are not a power of two in
    // [16, 1024] (the y and z passes and the x transform of psi have
    // per-length plans for every supported length)
    const int lens[3] = {B.M, B.ny, B.nz};
    const int nrt[3] = {5, 4, 4};
    const bool need[3] = {mvd_xadj_rows(B.M) == 0, mvd_exact_param(PASS_Y, B.ny) <= 0,
                          mvd_exact_param(PASS_Z, B.nz) <= 0};
    for (int k = 0; k < 3; ++k) {
      if (!need[k]) continue;
      for (int c = 0; c < nrt[k]; ++c)
        if (mvd_cfg_maxlen(k, c) >= lens[k]) {
          h->rt_cfg[k] = c;
          break;
        }
      if (h->rt_cfg[k] < 0)
        bad("the differentiated form takes half-rows up to 512, or power-of-two half-rows up to 1024");
      h->rt_grid[k] = total_tiles(h, k, mvd_cfg_param(k, h->rt_cfg[k]));
    }
    const size_t N = h->nviews, V = B.V, S = B.spec_elems;
    h->g_b = (float*)h->dalloc(N * V * sizeof(float));
    h->g_q = (float*)h->dalloc(N * V * sizeof(float));
    h->g_c = (float*)h->dalloc(N * V * sizeof(float));
    h->g_psi = (float*)h->dalloc(N * V * sizeof(float));
    h->g_spsi = (float2*)h->dalloc(N * S * sizeof(float2));
    h->g_sq = (float2*)h->dalloc(N * S * sizeof(float2));
    h->g_sT = (float2*)h->dalloc(S * sizeof(float2));
    h->g_acc = (double2*)h->dalloc(N * S * sizeof(double2));
    h->g_gbar = (float*)h->dalloc(V * sizeof(float));
    h->g_part = (float*)h->dalloc(V * sizeof(float));
    h->g_psiT = (float*)h->dalloc(V * sizeof(float));
    // the x passes: the compile-time row plan for power-of-two half-rows
    h->gx_rows = mvd_xadj_rows(B.M);
    h->gx_grid = h->gx_rows > 0 ? mvd_tiles(h->jobs[0], PASS_X, h->gx_rows) : h->rt_grid[0];
    h->g_parts = (Partial*)h->dalloc(N * h->gx_grid * sizeof(Partial));
    h->g_loss = (double*)h->dalloc(N * sizeof(double));
    h->g_lr = (unsigned long long*)h->dalloc(N * sizeof(unsigned long long));
    h->g_ln = (unsigned long long*)h->dalloc(N * sizeof(unsigned long long));
    h->grad_ready = true;
  }
  if (n > h->grad_ckpt_cap) {
    h->g_ckpt = (float*)h->dalloc((size_t)n * B.V * sizeof(float));
    h->grad_ckpt_cap = n;
  }
}

AdjPtrs adj_ptrs(mvd_handle* h, int v) {
  const size_t V = h->blocks[0].V;
  AdjPtrs a{};
  a.b = h->g_b + v * V;
  a.q = h->g_q + v * V;
  a.c = h->g_c + v * V;
  a.psi_in = h->g_psi + v * V;
  a.gbar = h->g_gbar;
  a.part = h->g_part;
  a.out = h->g_gbar;
  return a;
}

// An x pass of the differentiated form (mode 3..8 of the adjoint x kernels).
void grad_x(mvd_handle* h, int mode, int v, Partial* parts, const AdjPtrs& ap) {
  const LaunchArgs ax = args(h, h->stream, h->gx_grid);
  if (h->gx_rows > 0)
    HIPCHECK(mvd_launch_xadj_exact(ax, h->blocks[0].M, mode, v, parts, h->d_flags, ap));
  else
    HIPCHECK(mvd_launch_xadj(ax, h->rt_cfg[0], mode, v, parts, h->d_flags, ap));
}

// Forward view-update v with its intermediates stored (b, q, c, the input
// psi and the spectra of psi and q).
// The differentiated form's y and z passes: the block's per-length
// compile-time plan when its length has one, else the runtime plans.
void grad_y(mvd_handle* h, int inv, int v) {
  const int ny = h->blocks[0].ny, p = mvd_exact_param(PASS_Y, ny);
  if (p > 0)
    HIPCHECK(mvd_launch_y_exact(args(h, h->stream, mvd_tiles(h->jobs[0], PASS_Y, p)), ny, inv, v));
  else
    HIPCHECK(mvd_launch_y(args(h, h->stream, h->rt_grid[1]), h->rt_cfg[1], inv, v));
}

void grad_zext(mvd_handle* h, int v, int conjH, float2* s_out, const float2* s_in, double2* acc, int acc_mode,
               int role = ROLE_P) {
  const int nz = h->blocks[0].nz, p = mvd_exact_param(PASS_Z, nz);
  if (p > 0)
    HIPCHECK(mvd_launch_zext_exact(args(h, h->stream, mvd_tiles(h->jobs[0], PASS_Z, p)), nz, v, role, conjH, s_out,
                                   s_in, acc, acc_mode));
  else
    HIPCHECK(mvd_launch_zext(args(h, h->stream, h->rt_grid[2]), h->rt_cfg[2], v, role, conjH, s_out, s_in, acc,
                             acc_mode));
}

// The back-projection kernel of a variant as the z pass applies it: RL the
// conjugated PSF spectrum (K_v = P_v*), otherwise the compound spectrum.
int back_role(int variant) { return variant == MVD_RL ? ROLE_P : variant; }
int back_conj(int variant) { return variant == MVD_RL ? 1 : 0; }

void grad_forward_view(mvd_handle* h, int v, int variant) {
  const Block& B = h->blocks[0];
  hipStream_t s = h->stream;
  const AdjPtrs ap = adj_ptrs(h, v);
  Partial* parts = h->g_parts + (size_t)v * h->gx_grid;
  grad_y(h, 0, v);
  grad_zext(h, v, 0, h->g_spsi + (size_t)v * B.spec_elems, nullptr, nullptr, 0);
  grad_y(h, 1, v);
  grad_x(h, 3, v, parts, ap);
  grad_y(h, 0, v);
  grad_zext(h, v, back_conj(variant), h->g_sq + (size_t)v * B.spec_elems, nullptr, nullptr, 0, back_role(variant));
  grad_y(h, 1, v);
  grad_x(h, 4, v, parts, ap);
}

// Adjoint of view-update v: g_gbar holds dL/dpsi' on entry and dL/dpsi on exit.
// The back-projection's kernel term conj(Cbar) Q goes to the PSF's
// cross-spectrum for RL (K_v = P_v*: the mirrored term is a PSF gradient)
// and to the kernel's own cross-spectrum for the compound variants.
void grad_adjoint_view(mvd_handle* h, int v, int variant) {
  const Block& B = h->blocks[0];
  hipStream_t s = h->stream;
  const AdjPtrs ap = adj_ptrs(h, v);
  double2* acc = h->g_acc + (size_t)v * B.spec_elems;
  double2* acck = variant == MVD_RL ? acc : h->g_acck + (size_t)v * B.spec_elems;
  // cbar and the direct part of psibar
  grad_x(h, 5, v, nullptr, ap);
  // qbar = cbar (x) K_v* (the adjoint of the back-projection), with
  // acc += conj(Cbar) Q
  grad_y(h, 0, v);
  grad_zext(h, v, 1 - back_conj(variant), nullptr, h->g_sq + (size_t)v * B.spec_elems, acck, 1,
            back_role(variant));
  grad_y(h, 1, v);
  // bbar
  grad_x(h, 6, v, nullptr, ap);
  // bbar (x) P_v*, with A_v += Bbar conj(Psi)
  grad_y(h, 0, v);
  grad_zext(h, v, 1, nullptr, h->g_spsi + (size_t)v * B.spec_elems, acc, 0);
  grad_y(h, 1, v);
  grad_x(h, 7, v, nullptr, ap);
}

// The x transform of psi that starts a run of the differentiated form.
void x_init_rt(mvd_handle* h) {
  const int M = h->blocks[0].M, p = mvd_exact_param(PASS_X, M);
  if (p > 0)
    HIPCHECK(mvd_launch_x_exact(args(h, h->stream, mvd_tiles(h->jobs[0], PASS_X, p)), M, 0, 0, nullptr, h->d_flags,
                                XOPT_SPEC));
  else
    HIPCHECK(mvd_launch_x(args(h, h->stream, h->rt_grid[0]), h->rt_cfg[0], 0, 0, nullptr, h->d_flags, XOPT_SPEC));
}

// seed == nullptr: the loss sum_v |psi_n (x) P_v - phi_v|^2 and its
// gradients; otherwise the vector-Jacobian product with seed = d/dpsi_n
// (seed_kind host or device) and no loss.
void set_estimate_impl(mvd_handle* h, const float* src, int src_kind, int block);

// Forward run of the differentiated form: n iterations from psi0 (NULL: the
// flat start) with one checkpoint per iteration; the intermediates of the
// last iteration stay stored.  Leaves psi = psi_n (also kept in g_psiT) and
// records the run.
void grad_forward_impl(mvd_handle* h, int n, int variant, const float* psi0, int psi0_kind) {
  if (h->blocks.size() != 1) throw Error(MVD_ESTATE, "the differentiated form takes a single-block handle");
  if (h->linear) throw Error(MVD_ESTATE, "the differentiated form runs with the circular boundary only");
  if (h->blocked) throw Error(MVD_ESTATE, "the block-wise form runs the sequential scheme only");
  if (variant < MVD_RL || variant > MVD_OPT2) bad("variant must be MVD_RL, MVD_EFF, MVD_OPT1 or MVD_OPT2");
  if (n < 0) bad("n must be >= 0");
  Block& B = h->blocks[0];
  const size_t V = B.V;
  hipStream_t st = h->stream;
  h->rec_token = 0;
  grad_setup(h, std::max(n, 1));
  if (variant != MVD_RL) {
    ensure_role(h, back_role(variant));
    if (!h->g_acck) h->g_acck = (double2*)h->dalloc((size_t)h->nviews * B.spec_elems * sizeof(double2));
  }
  if (psi0) {
    HIPCHECK(hipStreamSynchronize(st));
    set_estimate_impl(h, psi0, psi0_kind, 0);
  } else {
    HIPCHECK(mvd_launch_fill(B.psi, B.V, (float)B.s, st));
  }
  HIPCHECK(mvd_launch_set_int(h->d_flags, 0, st));
  x_init_rt(h);
  for (int i = 0; i < n; ++i) {
    HIPCHECK(hipMemcpyAsync(h->g_ckpt + (size_t)i * V, B.psi, V * sizeof(float), hipMemcpyDeviceToDevice, st));
    for (int v = 0; v < h->nviews; ++v) grad_forward_view(h, v, variant);
  }
  HIPCHECK(hipMemcpyAsync(h->g_psiT, B.psi, V * sizeof(float), hipMemcpyDeviceToDevice, st));
  h->inter_iter = n - 1;
  h->rec_n = n;
  h->rec_variant = variant;
  h->rec_token = ++h->rec_count;
  h->spec_valid = false;
  h->iterations = n;
}

// Reverse sweep over the recorded run: g_gbar holds dL/dpsi_n on entry and
// dL/dpsi_0 on exit; each iteration is recomputed from its checkpoint
// (unless its intermediates are the stored ones), then the adjoints of its
// view-updates run in reverse order, accumulating the PSF cross-spectra
// (g_acc must hold the loss's own contribution, or zeros).  Gradients go to
// the caller's buffers; psi is left at psi_n.
void grad_reverse_impl(mvd_handle* h, double* const* grad_psf, float* grad_psi0, int grad_kind) {
  Block& B = h->blocks[0];
  const int N = h->nviews, n = h->rec_n;
  const size_t V = B.V, S = B.spec_elems;
  hipStream_t st = h->stream;
  for (int i = n - 1; i >= 0; --i) {
    if (i != h->inter_iter) {
      HIPCHECK(hipMemcpyAsync(B.psi, h->g_ckpt + (size_t)i * V, V * sizeof(float), hipMemcpyDeviceToDevice, st));
      x_init_rt(h);
      for (int v = 0; v < N; ++v) grad_forward_view(h, v, h->rec_variant);
      h->inter_iter = i;
    }
    for (int v = N - 1; v >= 0; --v) grad_adjoint_view(h, v, h->rec_variant);
  }
  if (grad_psi0)
    HIPCHECK(hipMemcpyAsync(grad_psi0, h->g_gbar, V * sizeof(float),
                            grad_kind == MVD_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, st));
  if (grad_psf) {
    // the windowed inverse DFT of each view's cross-spectrum, on the device
    // in FP64 (z, then y, then x stage); the normalisation on the host
    auto table = [&](double2*& dst, int len) {
      if (dst) return;
      const auto t = mvdh::twiddles(len);
      dst = (double2*)h->dalloc(t.size() * sizeof(double2));
      HIPCHECK(hipMemcpyAsync(dst, t.data(), t.size() * sizeof(double2), hipMemcpyHostToDevice, st));
    };
    table(h->g_twz, B.nz);
    table(h->g_twy, B.ny);
    table(h->g_twx, B.nx);
    size_t t1n = 0, t2n = 0, gn = 0;
    for (int v = 0; v < N; ++v) {
      const mvdh::Kern& P = B.P[v];
      t1n = std::max(t1n, (size_t)(B.M + 1) * B.ny * P.kz);
      t2n = std::max(t2n, (size_t)(B.M + 1) * P.ky * P.kz);
      gn = std::max(gn, (size_t)P.kx * P.ky * P.kz);
    }
    auto grow = [&](auto*& p, size_t& cap, size_t cnt, size_t elem) {
      if (cnt <= cap) return;
      p = (std::remove_reference_t<decltype(p)>)h->dalloc(cnt * elem);
      cap = cnt;
    };
    grow(h->g_t1, h->g_t1_cap, t1n, sizeof(double2));
    grow(h->g_t2, h->g_t2_cap, t2n, sizeof(double2));
    grow(h->g_gw, h->g_gw_cap, gn, sizeof(double));
    const double invV = 1.0 / (double)B.V;
    // a cross-spectrum's windowed inverse DFT on the window of P_v
    auto window_of = [&](const double2* A, const mvdh::Kern& P) {
      HIPCHECK(mvd_launch_idft_z(A, B.M, B.Mp, B.ny, B.nz, P.kz, h->g_twz, h->g_t1, st));
      HIPCHECK(mvd_launch_idft_yx(h->g_t1, B.M, B.nx, B.ny, P.kx, P.ky, P.kz, h->g_twx, h->g_twy, h->g_t2,
                                  h->g_gw, st));
      std::vector<double> g((size_t)P.kx * P.ky * P.kz);
      HIPCHECK(hipMemcpyAsync(g.data(), h->g_gw, g.size() * sizeof(double), hipMemcpyDeviceToHost, st));
      HIPCHECK(hipStreamSynchronize(st));
      for (double& x : g) x *= invV;
      return g;
    };
    // dL/dP_v on the padded boxes: the blur terms (and for RL the mirrored
    // back-projection terms) ...
    const bool compound = h->rec_variant != MVD_RL;
    std::vector<std::vector<double>> gP(N);
    for (int v = 0; v < N; ++v)
      if (grad_psf[v] || compound) gP[v] = window_of(h->g_acc + (size_t)v * S, B.P[v]);
    // ... and for the compound variants the kernel gradients (the
    // accumulated term is the mirrored dL/dK_v) through the construction of
    // every K_v from all PSFs
    if (compound) {
      std::vector<std::vector<double>> Kbar(N);
      for (int v = 0; v < N; ++v) {
        mvdh::Kern t = B.P[v];
        t.a = window_of(h->g_acck + (size_t)v * S, B.P[v]);
        Kbar[v] = mvdh::mirror(t).a;
      }
      const auto add = mvdh::compound_kernels_vjp(B.P, h->rec_variant, Kbar);
      for (int w = 0; w < N; ++w)
        for (size_t j = 0; j < add[w].size(); ++j) gP[w][j] += add[w][j];
    }
    for (int v = 0; v < N; ++v) {
      if (!grad_psf[v]) continue;
      const mvdh::Kern& P = B.P[v];
      const std::vector<double>& g = gP[v];
      // through the normalisation P = G / sum G, then drop the odd padding
      double dot = 0;
      for (size_t j = 0; j < g.size(); ++j) dot += g[j] * P.a[j];
      const auto& d = B.psf_dims[v];
      for (int z = 0; z < d[2]; ++z)
        for (int y = 0; y < d[1]; ++y)
          for (int x = 0; x < d[0]; ++x)
            grad_psf[v][((size_t)z * d[1] + y) * d[0] + x] =
                (g[((size_t)z * P.ky + y) * P.kx + x] - dot) / B.psf_sum[v];
    }
  }
  // leave psi at the end of the run
  HIPCHECK(hipMemcpyAsync(B.psi, h->g_psiT, V * sizeof(float), hipMemcpyDeviceToDevice, st));
  HIPCHECK(hipStreamSynchronize(st));
  h->spec_valid = false;
  h->iterations = n;
  if (read_flag(h)) throw Error(MVD_ENONFINITE, "the estimate became non-finite");
}

// seed == nullptr: the loss sum_v |psi_n (x) P_v - phi_v|^2 and its
// gradients; otherwise the vector-Jacobian product with seed = d/dpsi_n
// (recomputing the forward run from psi0).
void loss_grad_impl(mvd_handle* h, int n, int variant, const float* psi0, int psi0_kind, double* loss,
                    double* const* grad_psf, float* grad_psi0, int grad_kind, const float* seed = nullptr,
                    int seed_kind = MVD_MEM_HOST) {
  if (!seed && !loss) bad("loss is NULL");
  if (seed && seed_kind != MVD_MEM_HOST && seed_kind != MVD_MEM_DEVICE) bad("grad_psi_n_kind must be host or device");
  if (grad_psi0 && grad_kind != MVD_MEM_HOST && grad_kind != MVD_MEM_DEVICE) bad("grad_kind must be host or device");
  grad_forward_impl(h, n, variant, psi0, psi0_kind);
  Block& B = h->blocks[0];
  const int N = h->nviews;
  const size_t V = B.V, S = B.spec_elems;
  hipStream_t st = h->stream;
  const bool want_grad = grad_psf || grad_psi0;
  // loss sum_v |psi_T (x) P_v - phi_v|^2 and its adjoint seed, or the
  // caller's seed
  HIPCHECK(hipMemsetAsync(h->g_acc, 0, (size_t)N * S * sizeof(double2), st));
  if (h->g_acck) HIPCHECK(hipMemsetAsync(h->g_acck, 0, (size_t)N * S * sizeof(double2), st));
  if (seed)
    HIPCHECK(hipMemcpyAsync(h->g_gbar, seed, V * sizeof(float),
                            seed_kind == MVD_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, st));
  else
    HIPCHECK(hipMemsetAsync(h->g_gbar, 0, V * sizeof(float), st));
  for (int v = 0; v < N && !seed; ++v) {
    Partial* parts = h->g_parts + (size_t)v * h->gx_grid;
    AdjPtrs ap = adj_ptrs(h, v);
    ap.part = h->g_gbar;
    x_init_rt(h);
    grad_y(h, 0, v);
    grad_zext(h, v, 0, h->g_sT, nullptr, nullptr, 0);
    grad_y(h, 1, v);
    grad_x(h, 8, v, parts, ap);
    if (want_grad) {
      grad_y(h, 0, v);
      grad_zext(h, v, 1, nullptr, h->g_sT, h->g_acc + (size_t)v * S, 0);
      grad_y(h, 1, v);
      grad_x(h, 7, v, nullptr, ap);
    }
  }
  std::vector<double> lv(N, 0.0);
  if (!seed) {
    HIPCHECK(mvd_launch_reduce(h->g_parts, h->gx_grid, N, h->g_loss, h->g_lr, h->g_ln, st));
    HIPCHECK(hipMemcpyAsync(lv.data(), h->g_loss, N * sizeof(double), hipMemcpyDeviceToHost, st));
  }
  if (want_grad) {
    const int64_t token = h->rec_token;
    grad_reverse_impl(h, grad_psf, grad_psi0, grad_kind);
    h->rec_token = token;
  } else {
    HIPCHECK(hipMemcpyAsync(B.psi, h->g_psiT, V * sizeof(float), hipMemcpyDeviceToDevice, st));
    HIPCHECK(hipStreamSynchronize(st));
    h->spec_valid = false;
    if (read_flag(h)) throw Error(MVD_ENONFINITE, "the estimate became non-finite");
  }
  double L = 0;
  for (double x : lv) L += x;
  if (loss) *loss = L;
}

// The vector-Jacobian product over the run recorded by mvd_forward_recorded
// (token), without recomputing the forward run from psi0.
void backward_recorded_impl(mvd_handle* h, int64_t token, const float* seed, int seed_kind, double* const* grad_psf,
                            float* grad_psi0, int grad_kind) {
  if (!seed) bad("grad_psi_n is NULL");
  if (seed_kind != MVD_MEM_HOST && seed_kind != MVD_MEM_DEVICE) bad("grad_psi_n_kind must be host or device");
  if (grad_psi0 && grad_kind != MVD_MEM_HOST && grad_kind != MVD_MEM_DEVICE) bad("grad_kind must be host or device");
  if (token <= 0 || token != h->rec_token)
    throw Error(MVD_ESTATE, "no recorded run with this token (a later call changed the estimate, PSFs or weights)");
  Block& B = h->blocks[0];
  const size_t V = B.V, S = B.spec_elems;
  hipStream_t st = h->stream;
  HIPCHECK(hipMemsetAsync(h->g_acc, 0, (size_t)h->nviews * S * sizeof(double2), st));
  if (h->g_acck) HIPCHECK(hipMemsetAsync(h->g_acck, 0, (size_t)h->nviews * S * sizeof(double2), st));
  HIPCHECK(hipMemcpyAsync(h->g_gbar, seed, V * sizeof(float),
                          seed_kind == MVD_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, st));
  grad_reverse_impl(h, grad_psf, grad_psi0, grad_kind);
  h->rec_token = token;
}

void set_psfs_impl(mvd_handle* h, const float* const* psfs, const int* psf_dims, int mem_kind) {
  h->rec_token = 0;
  if (h->blocks.size() != 1) throw Error(MVD_ESTATE, "mvd_set_psfs takes a single-block handle");
  if (h->linear) throw Error(MVD_ESTATE, "mvd_set_psfs runs with the circular boundary only");
  if (h->blocked) throw Error(MVD_ESTATE, "the block-wise form runs the sequential scheme only");
  if (!psfs || !psf_dims) bad("psfs and psf_dims are required");
  if (mem_kind != MVD_MEM_HOST && mem_kind != MVD_MEM_DEVICE) bad("mem_kind must be host or device");
  Block& B = h->blocks[0];
  const int N = h->nviews;
  std::vector<mvdh::Kern> P;
  std::vector<double> sums;
  std::vector<std::array<int, 3>> dims;
  for (int v = 0; v < N; ++v) {
    if (!psfs[v]) bad("PSF pointer is NULL");
    const int* k = psf_dims + 3 * v;
    const int vd[3] = {B.nx, B.ny, B.nz};
    for (int a = 0; a < 3; ++a) {
      if (k[a] < 1) bad("PSF extents must be >= 1");
      if ((k[a] | 1) > vd[a]) bad("PSF (odd-padded) is larger than the volume");
    }
    const size_t n = (size_t)k[0] * k[1] * k[2];
    std::vector<float> hp(n);
    if (mem_kind == MVD_MEM_HOST)
      std::memcpy(hp.data(), psfs[v], n * sizeof(float));
    else
      HIPCHECK(hipMemcpy(hp.data(), psfs[v], n * sizeof(float), hipMemcpyDeviceToHost));
    try {
      P.push_back(mvdh::prepare_psf(hp.data(), k[0], k[1], k[2]));
    } catch (const std::invalid_argument& e) {
      bad(std::string("PSF ") + std::to_string(v) + ": " + e.what());
    }
    double sum = 0;
    for (float x : hp) sum += x;
    sums.push_back(sum);
    dims.push_back({k[0], k[1], k[2]});
  }
  HIPCHECK(hipStreamSynchronize(h->stream));
  B.P = std::move(P);
  B.psf_sum = std::move(sums);
  B.psf_dims = std::move(dims);
  set_kernel_window(B);
  if (B.kz > B.kz_cap) {
    // a wider window: fresh kernel-plane arrays (the old ones are released
    // with the handle); the compound kernels are rebuilt on next use
    B.kz_cap = B.kz;
    for (int r = 0; r < N_ROLES; ++r) B.H[r] = nullptr;
    B.H[ROLE_P] = (float*)h->dalloc((size_t)N * B.h_elems * 2 * sizeof(float));
  }
  for (int v = 0; v < N; ++v) upload_kernel(h, B, B.P[v], B.H[ROLE_P] + (size_t)v * B.h_elems * 2);
  for (int r = 1; r < N_ROLES; ++r) h->built[r] = false;
  build_jobs(h);
}

// Limit every voxel's summed weight to the overlap number of its block (see
// mvd_weights.hip); m per block into m_out when given.
void normalize_weights_impl(mvd_handle* h, int mode, double value, double* m_out) {
  h->rec_token = 0;
  if (mode < MVD_OVERLAP_ONE || mode > MVD_OVERLAP_USER) bad("mode must be one of the MVD_OVERLAP_* values");
  if (mode == MVD_OVERLAP_USER && !(value > 0 && std::isfinite(value))) bad("the user overlap must be finite and > 0");
  for (const auto& B : h->blocks)
    if (!B.w) throw Error(MVD_ESTATE, "the handle was created without weights");
  if (h->linear) throw Error(MVD_ESTATE, "weight normalisation runs with the circular boundary only");
  if (h->blocked) throw Error(MVD_ESTATE, "the block-wise form runs the sequential scheme only");
  if (!h->w_cmin) {
    h->w_cmin = (unsigned*)h->dalloc(sizeof(unsigned));
    h->w_cnt = (unsigned long long*)h->dalloc(2 * sizeof(unsigned long long));
  }
  unsigned* cmin = h->w_cmin;
  unsigned long long* cnt = h->w_cnt;
  for (size_t b = 0; b < h->blocks.size(); ++b) {
    Block& B = h->blocks[b];
    double m = mode == MVD_OVERLAP_USER ? value : 1.0;
    if (mode == MVD_OVERLAP_MIN || mode == MVD_OVERLAP_AVG) {
      const unsigned init = 0xffffffffu;
      const unsigned long long zero[2] = {0, 0};
      HIPCHECK(hipMemcpyAsync(cmin, &init, sizeof(init), hipMemcpyHostToDevice, h->stream));
      HIPCHECK(hipMemcpyAsync(cnt, zero, sizeof(zero), hipMemcpyHostToDevice, h->stream));
      HIPCHECK(mvd_launch_overlap_stats(B.w, h->nviews, B.V, cmin, cnt, cnt + 1, h->stream));
      unsigned mn = 0;
      unsigned long long c[2] = {0, 0};
      HIPCHECK(hipMemcpyAsync(&mn, cmin, sizeof(mn), hipMemcpyDeviceToHost, h->stream));
      HIPCHECK(hipMemcpyAsync(c, cnt, sizeof(c), hipMemcpyDeviceToHost, h->stream));
      HIPCHECK(hipStreamSynchronize(h->stream));
      if (c[1] > 0) m = mode == MVD_OVERLAP_MIN ? (double)mn : (double)c[0] / (double)c[1];
    }
    HIPCHECK(mvd_launch_overlap_limit(B.w, h->nviews, B.V, (float)m, h->stream));
    if (m_out) m_out[b] = m;
  }
  HIPCHECK(hipStreamSynchronize(h->stream));
}

void contributing_views_impl(mvd_handle* h, float* dst, int dst_kind, int block) {
  if (!dst) bad("dst is NULL");
  if (dst_kind != MVD_MEM_HOST && dst_kind != MVD_MEM_DEVICE) bad("dst_kind must be host or device");
  if (block < 0 || block >= (int)h->blocks.size()) bad("block index out of range");
  const Block& B = h->blocks[block];
  if (!B.w) throw Error(MVD_ESTATE, "the handle was created without weights");
  if (h->linear) throw Error(MVD_ESTATE, "the contributing-view image needs the circular boundary");
  if (h->blocked) throw Error(MVD_ESTATE, "the block-wise form runs the sequential scheme only");
  if (dst_kind == MVD_MEM_DEVICE) {
    HIPCHECK(mvd_launch_overlap_count(B.w, h->nviews, B.V, dst, h->stream));
  } else {
    if (h->w_stage_cap < B.V) {
      int64_t cap = 0;
      for (const auto& X : h->blocks) cap = std::max(cap, X.V);
      h->w_stage = (float*)h->dalloc(cap * sizeof(float));
      h->w_stage_cap = cap;
    }
    float* tmp = h->w_stage;
    HIPCHECK(mvd_launch_overlap_count(B.w, h->nviews, B.V, tmp, h->stream));
    HIPCHECK(hipMemcpyAsync(dst, tmp, B.V * sizeof(float), hipMemcpyDeviceToHost, h->stream));
  }
  HIPCHECK(hipStreamSynchronize(h->stream));
}

int read_flag(mvd_handle* h) {
  int f = 0;
  HIPCHECK(hipMemcpyAsync(&f, h->d_flags, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIPCHECK(hipStreamSynchronize(h->stream));
  return f;
}

const Block& block_of(mvd_handle* h, int b) {
  if (b < 0 || b >= (int)h->blocks.size()) bad("block index out of range");
  return h->blocks[b];
}

// Copy the estimate of a block out (the volume of the grid with the linear
// boundary); returns the non-finite flag.  Synchronises.
int get_estimate_impl(mvd_handle* h, float* dst, int dst_kind, int block) {
  const Block& B = block_of(h, block);
  if (!dst) bad("dst is NULL");
  if (dst_kind != MVD_MEM_HOST && dst_kind != MVD_MEM_DEVICE) bad("dst_kind must be host or device");
  if (h->blocked) {
    if (block != 0) bad("the block-wise form has one estimate: block 0");
    HIPCHECK(hipMemcpyAsync(dst, h->tl.psi, h->tl.V * sizeof(float),
                            dst_kind == MVD_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, h->stream));
  } else if (!h->linear) {
    HIPCHECK(hipMemcpyAsync(dst, B.psi, B.V * sizeof(float),
                            dst_kind == MVD_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, h->stream));
  } else {
    // the volume out of the grid; host copies pass through the factor buffer
    float* to = dst;
    if (dst_kind == MVD_MEM_HOST) {
      ensure_combined(h);
      to = B.acc;
    }
    HIPCHECK(mvd_launch_extract(to, user_dims(B), B.psi, grid_dims(B), offsets(B), h->stream));
    if (dst_kind == MVD_MEM_HOST)
      HIPCHECK(hipMemcpyAsync(dst, to, B.UV * sizeof(float), hipMemcpyDeviceToHost, h->stream));
  }
  return read_flag(h);
}

// Replace the estimate of a block (checked finite and >= 0); resets the
// iteration count and the non-finite flag.  Synchronises.
void set_estimate_impl(mvd_handle* h, const float* src, int src_kind, int block) {
  h->rec_token = 0;
  h->inter_iter = -1;
  Block& B = const_cast<Block&>(block_of(h, block));
  if (!src) bad("src is NULL");
  if (src_kind != MVD_MEM_HOST && src_kind != MVD_MEM_DEVICE) bad("src_kind must be host or device");
  if (h->blocked) {
    if (block != 0) bad("the block-wise form has one estimate: block 0");
    const int64_t V = h->tl.V;
    if (src_kind == MVD_MEM_HOST) {
      for (int64_t i = 0; i < V; ++i)
        if (!(src[i] >= 0.f) || !std::isfinite(src[i])) bad("estimate has a negative or non-finite value");
      HIPCHECK(hipMemcpyAsync(h->tl.psi, src, V * sizeof(float), hipMemcpyHostToDevice, h->stream));
    } else {
      double s;
      unsigned long long nb;
      device_check(h, src, V, 0.f, INFINITY, &s, &nb);
      if (nb) bad("estimate has a negative or non-finite value");
      HIPCHECK(hipMemcpyAsync(h->tl.psi, src, V * sizeof(float), hipMemcpyDeviceToDevice, h->stream));
    }
    HIPCHECK(mvd_launch_set_int(h->d_flags, 0, h->stream));
    HIPCHECK(hipStreamSynchronize(h->stream));
    h->iterations = 0;
    return;
  }
  // with the linear boundary the volume goes into the grid (host data via
  // the factor buffer) and the margin restarts at s
  float* to = B.psi;
  if (h->linear) {
    ensure_combined(h);
    to = B.acc;
  }
  if (src_kind == MVD_MEM_HOST) {
    for (int64_t i = 0; i < B.UV; ++i)
      if (!(src[i] >= 0.f) || !std::isfinite(src[i])) bad("estimate has a negative or non-finite value");
    HIPCHECK(hipMemcpyAsync(to, src, B.UV * sizeof(float), hipMemcpyHostToDevice, h->stream));
  } else {
    double s;
    unsigned long long nb;
    device_check(h, src, B.UV, 0.f, INFINITY, &s, &nb);
    if (nb) bad("estimate has a negative or non-finite value");
    if (h->linear)
      to = const_cast<float*>(src);
    else
      HIPCHECK(hipMemcpyAsync(B.psi, src, B.V * sizeof(float), hipMemcpyDeviceToDevice, h->stream));
  }
  if (h->linear) {
    HIPCHECK(mvd_launch_fill(B.psi, B.V, (float)B.s, h->stream));
    HIPCHECK(mvd_launch_embed(B.psi, grid_dims(B), to, user_dims(B), offsets(B), h->stream));
  }
  HIPCHECK(mvd_launch_set_int(h->d_flags, 0, h->stream));
  HIPCHECK(hipStreamSynchronize(h->stream));
  h->spec_valid = false;
  h->iterations = 0;
}

template <class F>
int guard(mvd_handle* h, F&& f) {
  try {
    f();
    if (h) h->err.clear();
    return MVD_OK;
  } catch (const Error& e) {
    (h ? h->err : g_err) = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    (h ? h->err : g_err) = "host allocation failed";
    return MVD_ENOMEM;
  } catch (const std::exception& e) {
    (h ? h->err : g_err) = e.what();
    return MVD_EINVAL;
  } catch (...) {
    (h ? h->err : g_err) = "unknown failure";
    return MVD_EDEVICE;
  }
}

std::mutex g_scratch_mu;
void* g_scratch_dev[256] = {};

void* scratch_on_current_device() {
  int dev = 0;
  HIPCHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= 256) bad("device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      throw Error(MVD_EDEVICE, std::string("hipGetSymbolAddress of the scratch array: ") + hipGetErrorString(e));
    }
    g_scratch_dev[dev] = ptr;
  }
  return g_scratch_dev[dev];
}

// Bump allocation over the scratch array (the handle's allocator callbacks;
// dalloc rounds every request up to 256 bytes, so every buffer stays
// 256-byte aligned).  Nothing is freed: the region is reused by the next run.
struct ScratchArena {
  unsigned char* base;
  size_t cap, used, refused;
};

void* arena_alloc(size_t bytes, void* ctx) {
  auto* a = static_cast<ScratchArena*>(ctx);
  if (bytes > a->cap - a->used) {
    a->refused = bytes;
    return nullptr;
  }
  void* p = a->base + a->used;
  a->used += bytes;
  return p;
}

void arena_free(void*, void*) {}

void iterate_noalloc_impl(const mvd_problem* p, const mvd_options* o, const float* psi0, int n, int variant,
                          float* psi_out) {
  if (!p) bad("problem is NULL");
  if (!psi_out) bad("psi_out is NULL");
  if (variant < MVD_RL || variant > MVD_OPT2) bad("variant must be MVD_RL, MVD_EFF, MVD_OPT1 or MVD_OPT2");
  if (n < 0) bad("n must be >= 0");
  if (o && (o->alloc || o->free)) bad("the no-allocation run takes no allocator callbacks");
  mvd_options opt{};
  if (o) opt = *o;
  ScratchArena arena{static_cast<unsigned char*>(scratch_on_current_device()), MVD_NOALLOC_SCRATCH_BYTES, 0, 0};
  opt.alloc = arena_alloc;
  opt.free = arena_free;
  opt.alloc_ctx = &arena;
  opt.use_graphs = 0;
  mvd_handle h;
  h.no_alloc = true;
  try {
    create_impl(&h, 1, p, &opt);
    if (psi0) set_estimate_impl(&h, psi0, MVD_MEM_DEVICE, 0);
    iterate_impl(&h, n, variant);
    const int nonfinite = get_estimate_impl(&h, psi_out, MVD_MEM_DEVICE, 0);
    h.release();
    if (nonfinite) throw Error(MVD_ENONFINITE, "the estimate became non-finite");
  } catch (...) {
    // nothing queued may outlive the call: the next run reuses the region
    (void)hipStreamSynchronize(h.stream);
    h.release();
    if (arena.refused)
      bad("the problem needs more device memory than the no-allocation run's scratch array holds (" +
          std::to_string(MVD_NOALLOC_SCRATCH_BYTES) + " bytes; a request of " + std::to_string(arena.refused) +
          " bytes with " + std::to_string(arena.used) + " in use)");
    throw;
  }
}

}  // namespace

extern "C" {

int mvd_create_batch(mvd_handle** out, int n_blocks, const mvd_problem* blocks, const mvd_options* o) {
  if (!out) {
    g_err = "out is NULL";
    return MVD_EINVAL;
  }
  *out = nullptr;
  mvd_handle* h = new (std::nothrow) mvd_handle();
  if (!h) {
    g_err = "host allocation failed";
    return MVD_ENOMEM;
  }
  const int rc = guard(nullptr, [&] { create_impl(h, n_blocks, blocks, o); });
  if (rc != MVD_OK) {
    h->release();
    delete h;
    return rc;
  }
  *out = h;
  return MVD_OK;
}

int mvd_create(mvd_handle** out, const mvd_problem* p, const mvd_options* o) {
  return mvd_create_batch(out, 1, p, o);
}

int mvd_create_blocked(mvd_handle** out, const mvd_problem* p, const mvd_options* o, const int* tiles,
                       const int* halo) {
  if (!out) {
    g_err = "out is NULL";
    return MVD_EINVAL;
  }
  *out = nullptr;
  mvd_handle* h = new (std::nothrow) mvd_handle();
  if (!h) {
    g_err = "host allocation failed";
    return MVD_ENOMEM;
  }
  const int rc = guard(nullptr, [&] { create_blocked_impl(h, p, o, tiles, halo); });
  if (rc != MVD_OK) {
    h->release();
    delete h;
    return rc;
  }
  *out = h;
  return MVD_OK;
}

int mvd_blocking(const mvd_handle* h, int* tiles, int* halo, int* dims) {
  if (!h) {
    g_err = "handle is NULL";
    return MVD_EINVAL;
  }
  for (int a = 0; a < 3; ++a) {
    const Block& B = h->blocks[0];
    if (tiles) tiles[a] = h->blocked ? h->tl.tiles[a] : 1;
    if (halo) halo[a] = h->blocked ? h->tl.halo[a] : 0;
    if (dims) dims[a] = h->blocked ? h->tl.dims[a] : (a == 0 ? B.ux : a == 1 ? B.uy : B.uz);
  }
  return MVD_OK;
}

int mvd_iterate(mvd_handle* h, int n, int variant) {
  if (!h) {
    g_err = "handle is NULL";
    return MVD_EINVAL;
  }
  return guard(h, [&] { iterate_impl(h, n, variant); });
}

int mvd_iterate_combined(mvd_handle* h, int n, int variant, int mean) {
  if (!h) {
    g_err = "handle is NULL";
    return MVD_EINVAL;
  }
  return guard(h, [&] { iterate_combined_impl(h, n, variant, mean); });
}

int mvd_normalize_weights(mvd_handle* h, int mode, double value, double* m_out) {
  if (!h) {
    g_err = "handle is NULL";
    return MVD_EINVAL;
  }
  return guard(h, [&] { normalize_weights_impl(h, mode, value, m_out); });
}

int mvd_contributing_views(mvd_handle* h, float* dst, int dst_kind, int block) {
  if (!h) {
    g_err = "handle is NULL";
    return MVD_EINVAL;
  }
  return guard(h, [&] { contributing_views_impl(h, dst, dst_kind, block); });
}

int mvd_grid_dims(const mvd_handle* h, int block, int* dims) {
  if (!h || !dims) {
    g_err = "handle or dims is NULL";
    return MVD_EINVAL;
  }
  if (block < 0 || block >= (int)h->blocks.size()) {
    g_err = "block index out of range";
    return MVD_EINVAL;
  }
  const Block& B = h->blocks[block];
  dims[0] = B.nx;
  dims[1] = B.ny;
  dims[2] = B.nz;
  return MVD_OK;
}

int mvd_get_estimate(mvd_handle* h, float* dst, int dst_kind, int block) {
  if (!h) {
    g_err = "handle is NULL";
    return MVD_EINVAL;
  }
  int nonfinite = 0;
  int rc = guard(h, [&] { nonfinite = get_estimate_impl(h, dst, dst_kind, block); });
  if (rc == MVD_OK && nonfinite) {
    h->err = "the estimate became non-finite";
    return MVD_ENONFINITE;
  }
  return rc;
}

int mvd_set_estimate(mvd_handle* h, const float* src, int src_kind, int block) {
  if (!h) {
    g_err = "handle is NULL";
    return MVD_EINVAL;
  }
  return guard(h, [&] { set_estimate_impl(h, src, src_kind, block); });
}

int mvd_stats(mvd_handle* h, mvd_stats_t* s) {
  if (!h) {
    g_err = "handle is NULL";
    return MVD_EINVAL;
  }
  return guard(h, [&] {
    if (!s) bad("stats is NULL");
    std::memset(s, 0, sizeof(*s));
    const int N = h->nviews;
    std::vector<double> f(N);
    std::vector<unsigned long long> a(N), b(N);
    HIPCHECK(hipMemcpyAsync(f.data(), h->d_flux, N * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHECK(hipMemcpyAsync(a.data(), h->d_ratio, N * sizeof(unsigned long long), hipMemcpyDeviceToHost, h->stream));
    HIPCHECK(hipMemcpyAsync(b.data(), h->d_neg, N * sizeof(unsigned long long), hipMemcpyDeviceToHost, h->stream));
    s->nonfinite = read_flag(h);
    s->iterations = h->iterations;
    s->n_views = N;
    s->n_blocks = (int)h->blocks.size();
    s->scale = h->blocks[0].s;
    for (int v = 0; v < N; ++v) {
      s->flux[v] = f[v];
      s->ratio_clamps += (int64_t)a[v];
      s->neg_clamps += (int64_t)b[v];
    }
  });
}

int mvd_synchronize(mvd_handle* h) {
  if (!h) {
    g_err = "handle is NULL";
    return MVD_EINVAL;
  }
  int nonfinite = 0;
  int rc = guard(h, [&] { nonfinite = read_flag(h); });
  if (rc == MVD_OK && nonfinite) {
    h->err = "the estimate became non-finite";
    return MVD_ENONFINITE;
  }
  return rc;
}

int mvd_destroy(mvd_handle* h) {
  if (!h) return MVD_OK;
  h->release();
  delete h;
  return MVD_OK;
}

const char* mvd_last_error(const mvd_handle* h) { return h ? h->err.c_str() : g_err.c_str(); }

int mvd_view_update(mvd_handle* h, int view, int variant) {
  if (!h) {
    g_err = "handle is NULL";
    return MVD_EINVAL;
  }
  return guard(h, [&] {
    if (view < 0 || view >= h->nviews) bad("view index out of range");
    h->rec_token = 0;
    prepare_run(h, variant);
    enqueue_view(h, h->stream, variant, view);
  });
}

int mvd_profile(mvd_handle* h, int n, int variant, double* avg_ms, int* calls) {
  if (!h) {
    g_err = "handle is NULL";
    return MVD_EINVAL;
  }
  return guard(h, [&] {
    if (n < 1) bad("n must be >= 1");
    if (!avg_ms || !calls) bad("avg_ms and calls are required");
    h->rec_token = 0;
    prepare_run(h, variant);
    PassTimer t;
    t.s = h->stream;
    for (int i = 0; i < n; ++i) enqueue_iteration(h, h->stream, variant, &t);
    HIPCHECK(hipStreamSynchronize(h->stream));
    double tot[MVD_PASS_KINDS] = {0};
    int cnt[MVD_PASS_KINDS] = {0};
    for (size_t i = 0; i < t.kind.size(); ++i) {
      float ms = 0;
      HIPCHECK(hipEventElapsedTime(&ms, t.ev[2 * i], t.ev[2 * i + 1]));
      tot[t.kind[i]] += ms;
      cnt[t.kind[i]] += 1;
    }
    for (int k = 0; k < MVD_PASS_KINDS; ++k) {
      avg_ms[k] = cnt[k] ? tot[k] / cnt[k] : 0.0;
      calls[k] = cnt[k];
    }
    h->iterations += n;
  });
}

int mvd_loss_grad(mvd_handle* h, int n, int variant, const float* psi0, int psi0_kind, double* loss,
                  double* const* grad_psf, float* grad_psi0, int grad_kind) {
  if (!h) {
    g_err = "handle is NULL";
    return MVD_EINVAL;
  }
  return guard(h, [&] { loss_grad_impl(h, n, variant, psi0, psi0_kind, loss, grad_psf, grad_psi0, grad_kind); });
}

int mvd_backward(mvd_handle* h, int n, int variant, const float* psi0, int psi0_kind, const float* grad_psi_n,
                 int grad_psi_n_kind, double* const* grad_psf, float* grad_psi0, int grad_kind) {
  if (!h) {
    g_err = "handle is NULL";
    return MVD_EINVAL;
  }
  return guard(h, [&] {
    if (!grad_psi_n) bad("grad_psi_n is NULL");
    loss_grad_impl(h, n, variant, psi0, psi0_kind, nullptr, grad_psf, grad_psi0, grad_kind, grad_psi_n,
                   grad_psi_n_kind);
  });
}

int mvd_forward_recorded(mvd_handle* h, int n, int variant, const float* psi0, int psi0_kind, int64_t* token) {
  if (!h) {
    g_err = "handle is NULL";
    return MVD_EINVAL;
  }
  return guard(h, [&] {
    if (!token) bad("token is NULL");
    *token = 0;
    grad_forward_impl(h, n, variant, psi0, psi0_kind);
    HIPCHECK(hipStreamSynchronize(h->stream));
    if (read_flag(h)) {
      h->rec_token = 0;
      throw Error(MVD_ENONFINITE, "the estimate became non-finite");
    }
    *token = h->rec_token;
  });
}

int mvd_backward_recorded(mvd_handle* h, int64_t token, const float* grad_psi_n, int grad_psi_n_kind,
                          double* const* grad_psf, float* grad_psi0, int grad_kind) {
  if (!h) {
    g_err = "handle is NULL";
    return MVD_EINVAL;
  }
  return guard(h, [&] {
    backward_recorded_impl(h, token, grad_psi_n, grad_psi_n_kind, grad_psf, grad_psi0, grad_kind);
  });
}

int mvd_set_psfs(mvd_handle* h, const float* const* psfs, const int* psf_dims, int mem_kind) {
  if (!h) {
    g_err = "handle is NULL";
    return MVD_EINVAL;
  }
  return guard(h, [&] { set_psfs_impl(h, psfs, psf_dims, mem_kind); });
}

int mvd_set_tiles(mvd_handle* h, int cfg_x, int cfg_y, int cfg_z) {
  if (!h) {
    g_err = "handle is NULL";
    return MVD_EINVAL;
  }
  return guard(h, [&] { set_tiles(h, cfg_x, cfg_y, cfg_z); });
}

int mvd_set_schedule(mvd_handle* h, int schedule) {
  if (!h) {
    g_err = "handle is NULL";
    return MVD_EINVAL;
  }
  return guard(h, [&] {
    if (schedule < MVD_SCHEDULE_PASS_MAJOR || schedule > MVD_SCHEDULE_RUN_MAJOR) bad("unknown schedule");
    if (schedule != h->schedule) drop_graphs(h);
    h->schedule = schedule;
  });
}

int mvd_get_schedule(const mvd_handle* h) { return h ? h->schedule : MVD_EINVAL; }

int mvd_get_tiles(const mvd_handle* h, int* cfg) {
  if (!h || !cfg) {
    g_err = "NULL argument";
    return MVD_EINVAL;
  }
  cfg[0] = h->cfg_x;
  cfg[1] = h->cfg_y;
  cfg[2] = h->cfg_z;
  return MVD_OK;
}

int mvd_tile_candidates(int kind, int max_len, int* out, int cap) {
  if (kind < 0 || kind > 2) {
    g_err = "kind must be 0 (x), 1 (y) or 2 (z)";
    return MVD_EINVAL;
  }
  int n = 0;
  for (int c = 0; c < mvd_num_cfgs(kind); ++c) {
    const int ex = mvd_cfg_exact(kind, c);
    if (ex > 0 ? ex == max_len : mvd_cfg_maxlen(kind, c) >= max_len) {
      if (out && n < cap) out[n] = c;
      ++n;
    }
  }
  return n;
}

int mvd_tile_shape(int kind, int cfg, int* threads, int* per_tile, int* max_len, int* exact_len) {
  if (kind < 0 || kind > 2 || cfg < 0 || cfg >= mvd_num_cfgs(kind)) {
    g_err = "no such tile configuration";
    return MVD_EINVAL;
  }
  if (threads) *threads = mvd_cfg_threads(kind, cfg);
  if (per_tile) *per_tile = mvd_cfg_param(kind, cfg);
  if (max_len) *max_len = mvd_cfg_maxlen(kind, cfg);
  if (exact_len) *exact_len = mvd_cfg_exact(kind, cfg);
  return MVD_OK;
}

int mvd_compound_kernel(int n_views, const float* const* psfs, const int* psf_dims, int v, int variant,
                        double* out, int* out_dims) {
  return guard(nullptr, [&] {
    if (n_views < 1 || n_views > MVD_MAX_VIEWS) bad("n_views must be in [1, 64]");
    if (!psfs || !psf_dims || !out) bad("psfs, psf_dims and out are required");
    if (v < 0 || v >= n_views) bad("v out of range");
    if (variant < MVD_RL || variant > MVD_OPT2) bad("unknown variant");
    std::vector<mvdh::Kern> P;
    for (int i = 0; i < n_views; ++i) {
      if (!psfs[i]) bad("PSF pointer is NULL");
      const int* k = psf_dims + 3 * i;
      try {
        P.push_back(mvdh::prepare_psf(psfs[i], k[0], k[1], k[2]));
      } catch (const std::invalid_argument& e) {
        bad(e.what());
      }
    }
    const mvdh::Kern K = mvdh::compound_kernel(P, v, variant);
    std::memcpy(out, K.a.data(), K.a.size() * sizeof(double));
    if (out_dims) {
      out_dims[0] = K.kx;
      out_dims[1] = K.ky;
      out_dims[2] = K.kz;
    }
  });
}

int mvd_compound_kernel_vjp(int n_views, const float* const* psfs, const int* psf_dims, int v, int variant,
                            const double* kbar, double* const* grad_out) {
  return guard(nullptr, [&] {
    if (n_views < 1 || n_views > MVD_MAX_VIEWS) bad("n_views must be in [1, 64]");
    if (!psfs || !psf_dims || !kbar || !grad_out) bad("psfs, psf_dims, kbar and grad_out are required");
    if (v < 0 || v >= n_views) bad("v out of range");
    if (variant < MVD_RL || variant > MVD_OPT2) bad("unknown variant");
    std::vector<mvdh::Kern> P;
    for (int i = 0; i < n_views; ++i) {
      if (!psfs[i] || !grad_out[i]) bad("PSF or gradient pointer is NULL");
      const int* k = psf_dims + 3 * i;
      try {
        P.push_back(mvdh::prepare_psf(psfs[i], k[0], k[1], k[2]));
      } catch (const std::invalid_argument& e) {
        bad(e.what());
      }
    }
    const std::vector<double> kb(kbar, kbar + P[v].a.size());
    const auto g = mvdh::compound_kernel_vjp(P, v, variant, kb);
    for (int i = 0; i < n_views; ++i) std::memcpy(grad_out[i], g[i].data(), g[i].size() * sizeof(double));
  });
}

int mvd_kernel_spectrum(const double* kernel, const int* kdims, const int* dims, float* main_out,
                        float* nyq_out) {
  return guard(nullptr, [&] {
    if (!kernel || !kdims || !dims || !main_out || !nyq_out) bad("NULL argument");
    if (dims[0] < 4 || dims[0] % 2 || dims[1] < 2 || dims[2] < 2) bad("bad volume dims");
    mvdh::Kern K;
    K.kx = kdims[0];
    K.ky = kdims[1];
    K.kz = kdims[2];
    if (K.kx < 1 || K.ky < 1 || K.kz < 1 || !(K.kx & 1) || !(K.ky & 1) || !(K.kz & 1))
      bad("kernel extents must be odd and >= 1");
    if (K.kx > dims[0] || K.ky > dims[1] || K.kz > dims[2]) bad("kernel larger than the volume");
    K.a.assign(kernel, kernel + (size_t)K.kx * K.ky * K.kz);
    mvdh::spectrum_host(K, dims[0], dims[1], dims[2], main_out, nyq_out);
  });
}

int mvd_iterate_noalloc(const mvd_problem* p, const mvd_options* o, const float* psi0, int n, int variant,
                        float* psi_out) {
  return guard(nullptr, [&] { iterate_noalloc_impl(p, o, psi0, n, variant, psi_out); });
}

const char* mvd_version(void) { return "mvd 0.1 (gfx950)"; }

}  // extern "C"
