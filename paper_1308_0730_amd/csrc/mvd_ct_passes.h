// Pass kernels with compile-time transform plans: the length and the radix
// sequence (16, 8, 4, 2, 5, 3) are template parameters, so the index math
// folds away.
//
// They compute exactly what the runtime-plan passes of mvd_kernels.hip
// compute (same algebra, same tile mapping, same pointwise steps).  A launch
// covers jobs that all have the kernel's length.  Their fused epilogues work
// on the last transform stage's registers:
//   z pass: the kernel lines are transformed first and their last stage kept
//           in registers; the spectral product is applied to the data's last
//           forward stage outputs in the same order;
//   x pass: the ratio, the update or the combined-update fold is applied to
//           the last inverse stage's outputs, with phi, psi, w or the factor
//           prefetched in the same order.
#pragma once
#include <hip/hip_runtime.h>

#include "fft_ct.h"
#include "mvd_device.h"
#include "mvd_kernels.h"

namespace mvdk {
namespace ctp {

// Global row accessor: element pos of row `line` is the float2 pair
// (x[2 pos], x[2 pos + 1]) of row wrow0 + line.
struct GRow {
  const float* base;  // row wrow0
  int nx, nrw;
  static constexpr bool lds = false;
  __device__ __forceinline__ float2 ld(int line, int pos) const {
    return line < nrw ? ld2(base + (int64_t)line * nx + 2 * pos) : make_float2(0.f, 0.f);
  }
};

// Window row accessor (block-wise form): element pos of row `line` is the
// pair of grid voxels x = 2 pos, 2 pos + 1 of that row, read from the volume
// at (sx + x) mod vnx of the volume row whose offset the wave's table holds.
struct WinRow {
  const float* vol;
  const int64_t* rows;  // the wave's rows: offset of volume voxel x = 0 of each
  int sx, vnx, nrw;
  static constexpr bool lds = false;
  __device__ __forceinline__ float2 ld(int line, int pos) const {
    if (line >= nrw) return make_float2(0.f, 0.f);
    const float* r = vol + rows[line];
    int x = sx + 2 * pos;
    while (x >= vnx) x -= vnx;
    const int x1 = x + 1 == vnx ? 0 : x + 1;
    return make_float2(ldg(r + x), ldg(r + x1));
  }
};

// Last forward z stage: multiply by the prefetched kernel spectrum (its
// conjugate for the mirrored kernel) and store to the LDS tile.
template <int TX, int MAXB, int R>
struct MulH {
  float2* buf;
  const float2 (&h)[MAXB][R];
  int conj;
  static constexpr bool lds = true;
  __device__ __forceinline__ void st(int line, int pos, float2 v, int i, int r) {
    const float2 w = h[i][r];
    buf[pos * TX + line] = cmul(v, conj ? cconj(w) : w);
  }
};

// Global tile read with unconditional loads: a line past nl reads line
// nl - 1 (a ragged tile's extra lines are transformed but never stored, and
// their kernel lines are zero).  With no load inside a branch the compiler
// knows how many loads follow a given one, so waiting for an earlier load
// does not drain these.
struct GTileU {
  const float2* base;
  int ls, ps, nl;
  static constexpr bool lds = false;
  __device__ __forceinline__ float2 ld(int line, int pos) const {
    return ldg(base + (line < nl ? line : nl - 1) * ls + pos * ps);
  }
};

// Last forward z stage of the differentiated form's z pass: besides the
// product (as MulH) it stores the forward spectrum (s_out) and adds the FP64
// PSF cross-spectrum term a conj(s) (mode 0) or conj(a) s (mode 1) with s
// read from s_in, at the tile's spectrum index off + line + pos ps.
template <int TX, int MAXB, int R>
struct ExtMul {
  float2* buf;
  const float2 (&h)[MAXB][R];
  int conj;
  int64_t off;
  int ps, nl;
  float2* s_out;
  const float2* s_in;
  double2* acc;
  int acc_mode;
  static constexpr bool lds = true;
  __device__ __forceinline__ void st(int line, int pos, float2 a, int i, int r) {
    if (line < nl) {
      const int64_t idx = off + line + (int64_t)pos * ps;
      if (s_out) stg(s_out + idx, a);
      if (acc) {
        const float2 s = ldg(s_in + idx);
        double2 t = ldg(acc + idx);
        if (acc_mode == 0) {
          t.x += (double)a.x * s.x + (double)a.y * s.y;
          t.y += (double)a.y * s.x - (double)a.x * s.y;
        } else {
          t.x += (double)a.x * s.x + (double)a.y * s.y;
          t.y += (double)a.x * s.y - (double)a.y * s.x;
        }
        stg(acc + idx, t);
      }
    }
    const float2 w = h[i][r];
    buf[pos * TX + line] = cmul(a, conj ? cconj(w) : w);
  }
};

// Last forward z stage of the kernel lines: keep the outputs in registers,
// in the order the data's last forward stage produces its own.
template <int MAXB, int R>
struct ToRegs {
  float2 (&h)[MAXB][R];
  static constexpr bool lds = false;
  __device__ __forceinline__ void st(int, int, float2 v, int i, int r) { h[i][r] = v; }
};

// Last inverse x stage: the pointwise step of the ratio (MODE 1), of the
// update (MODE 2), of folding a view into the combined factor (MODE 3) or of
// the last fold and the combined update (MODE 4), on the two real values held
// by each complex output; the packed result goes to LDS as the input of the
// forward transform.
template <int MODE_, int PITCH, int MAXB, int R>
struct RowOp {
  static constexpr int MODE = MODE_ & 7;
  static constexpr bool WIN = (MODE_ & XMODE_WIN) != 0;
  float2* buf;
  const float2 (&pa)[MAXB][R];
  const float2 (&pb)[MAXB][R];
  float* psi_rows;  // psi at row wrow0 (MODES 2, 4)
  float* acc_rows;  // the combined factor at row wrow0 (MODES 3, 4)
  // block-wise form (MODE 2): the new psi of the own voxels, grid voxels
  // [hx, hx + ex) of the rows whose volume offset own[] holds (-1: not an
  // own row), goes to vol at own[line] + ox + x - hx; nothing else is written
  float* vol;
  const int64_t* own;
  int ox, hx, ex;
  int nx, nrw;
  bool weighted, first, geo;
  float eps, lamp, inv_n;
  double flux;
  unsigned ncr, ncn;
  bool bad;
  static constexpr bool lds = true;
  __device__ __forceinline__ void st(int line, int pos, float2 z, int i, int r) {
    if (line >= nrw) return;
    float2 o;
    if (MODE == 1) {
      o = ratio2(pa[i][r], z, eps, ncr);
    } else if (MODE == 2) {
      const float2 p = pa[i][r];
      const float ux = p.x * (z.x > 0.f ? z.x : 0.f), uy = p.y * (z.y > 0.f ? z.y : 0.f);
      const float tx = tikhonov(ux, lamp), ty = tikhonov(uy, lamp);
      if (weighted) {
        o = make_float2(p.x + pb[i][r].x * (tx - p.x), p.y + pb[i][r].y * (ty - p.y));
      } else {
        o = make_float2(tx, ty);
      }
      if (WIN) {
        const int64_t b = own[line];
        const int x = 2 * pos - hx;
        if (b >= 0 && x >= 0 && x < ex) {
          stg(vol + b + ox + x, o.x);
          ncn += z.x < 0.f;
          flux += (double)o.x;
          bad |= !isfinite(o.x);
        }
        if (b >= 0 && x + 1 >= 0 && x + 1 < ex) {
          stg(vol + b + ox + x + 1, o.y);
          ncn += z.y < 0.f;
          flux += (double)o.y;
          bad |= !isfinite(o.y);
        }
      } else {
        ncn += (z.x < 0.f) + (z.y < 0.f);
        st2(psi_rows + (int64_t)line * nx + 2 * pos, o);
        flux += (double)o.x + (double)o.y;
        bad |= !(isfinite(o.x) && isfinite(o.y));
      }
    } else {
      ncn += (z.x < 0.f) + (z.y < 0.f);
      const float cx = z.x > 0.f ? z.x : 0.f, cy = z.y > 0.f ? z.y : 0.f;
      float mx = cx, my = cy;
      if (!first) {
        mx = geo ? pa[i][r].x * cx : pa[i][r].x + cx;
        my = geo ? pa[i][r].y * cy : pa[i][r].y + cy;
      }
      if (MODE == 3) {
        o = make_float2(mx, my);
        st2(acc_rows + (int64_t)line * nx + 2 * pos, o);
      } else {
        const float gx = geo ? powf(mx, inv_n) : mx * inv_n;
        const float gy = geo ? powf(my, inv_n) : my * inv_n;
        o = make_float2(tikhonov(pb[i][r].x * gx, lamp), tikhonov(pb[i][r].y * gy, lamp));
        st2(psi_rows + (int64_t)line * nx + 2 * pos, o);
        flux += (double)o.x + (double)o.y;
        bad |= !(isfinite(o.x) && isfinite(o.y));
      }
    }
    buf[line * PITCH + pos] = o;
  }
};

}  // namespace ctp

using namespace ctp;

// ---------------------------------------------------------------------------
// y pass (see k_ypass): complex transform along y of TX adjacent columns.
template <bool INV, int T, int TX, int L, int... Rs>
__device__ __forceinline__ void ypass_tile(float2* lds, float2* s_tw, const JobDesc& J, int local,
                                           const FftPlan* __restrict__ plans, const float2* __restrict__ twp) {
  const int M = J.M, ny = J.ny, nz = J.nz;
  float2* spec = reinterpret_cast<float2*>(J.spec);
  const int nxt = mvd_cdiv(M, TX);
  GTile g;
  int xt, z, t2;
  ytile<INV>(local, mvd_tiles(J, PASS_Y, TX), nxt, nz, xt, z, t2);
  if (t2 < 0) {
    g.base = spec + (int64_t)z * ny * J.Mp + xt * TX;
    g.ls = 1;
    g.ps = J.Mp;
    g.nl = min(TX, M - xt * TX);
  } else {
    g.base = spec + J.spec_main + (int64_t)t2 * TX * ny;
    g.ls = ny;
    g.ps = 1;
    g.nl = min(TX, nz - t2 * TX);
  }
  // the table is read from the second stage on, after the first stage's barrier
  load_table<T>(s_tw, twp + plans[J.plan_y].tw, L);
  Plain<GTile> out{g};
  CtRun<INV, L, T, TX, true, SYNC_BLOCK, 1, true, Rs...>::run(threadIdx.x, s_tw, g, LdsCol<TX>{lds}, out);
}

template <bool INV, int T, int TX, int L, int... Rs>
__global__ void __launch_bounds__(T)
    k_ypass_ct(const JobDesc* __restrict__ jobs, int njobs, const FftPlan* __restrict__ plans,
               const float2* __restrict__ twp, int v) {
  __shared__ float2 lds[L * TX];
  __shared__ float2 s_tw[L];
  int local;
  const int jid = find_job(jobs, njobs, PASS_Y, TX, local);
  if (jid < 0) return;
  const JobDesc& J = jobs[jid];
  if (v >= J.nviews) return;
  ypass_tile<INV, T, TX, L, Rs...>(lds, s_tw, J, local, plans, twp);
}

// ---------------------------------------------------------------------------
// z pass with the spectral product (see k_zconv).
template <int T, int TX, int L, int... Rs>
__device__ __forceinline__ void zconv_tile(float2* lds, float2* s_tw, const JobDesc& J, int local,
                                           const FftPlan* __restrict__ plans, const float2* __restrict__ twp,
                                           int v, int role, int conjH, int src_saved) {
  constexpr int RL = LastRadix<Rs...>::value;
  using LM = LastMap<L, RL, T, TX, true>;
  const int M = J.M, ny = J.ny;
  const int nxt = mvd_cdiv(M, TX);
  int64_t off, hoff;
  int ps, nl;
  if (local < nxt * ny) {
    int xt, y;
    half_tile(local, nxt, ny, xt, y);
    off = (int64_t)y * J.Mp + xt * TX;
    hoff = off;
    ps = ny * J.Mp;
    nl = min(TX, M - xt * TX);
  } else {
    const int t2 = local - nxt * ny;
    off = J.spec_main + (int64_t)t2 * TX;
    hoff = J.h_main + (int64_t)t2 * TX;
    ps = ny;
    nl = min(TX, ny - t2 * TX);
  }
  const KLine kl{reinterpret_cast<const float2*>(J.H[role]) + (int64_t)v * J.h_elems + hoff, ps, nl, L,
                 J.kz, J.cz};
  GTile g{reinterpret_cast<float2*>(J.spec) + off, 1, ps, nl};
  const GTileU gin{reinterpret_cast<const float2*>(src_saved ? J.saved : J.spec) + off, 1, ps, nl};
  // both tiles' first-stage loads up front, the kernel taps first: the
  // kernel lines' transform then waits only for its own loads and runs while
  // the data loads are in flight
  // (the twiddle table's loads go first and its LDS stores after, so that
  // storing it waits for its own loads only)
  constexpr int R1 = FirstRadix<Rs...>::value;
  constexpr int MB1 = FirstMap<L, R1, T, TX>::MAXB;
  constexpr int NTW = (L + T - 1) / T;
  const float2* twsrc = twp + plans[J.plan_z].tw;
  float2 twv[NTW];
#pragma unroll
  for (int i = 0; i < NTW; ++i) {
    const int e = threadIdx.x + i * T;
    twv[i] = e < L ? ldg(twsrc + e) : make_float2(0.f, 0.f);
  }
  float2 kp[MB1][R1], dp[MB1][R1];
  ct_prefetch<L, R1, T, TX, true>(threadIdx.x, kl, kp);
  ct_prefetch<L, R1, T, TX, true>(threadIdx.x, gin, dp);
#pragma unroll
  for (int i = 0; i < NTW; ++i) {
    const int e = threadIdx.x + i * T;
    if (e < L) s_tw[e] = twv[i];
  }
  const LdsCol<TX> S{lds};
  // kernel spectrum of the tile's lines, in the order the last forward stage
  // produces its outputs
  float2 h[LM::MAXB][RL];
  ToRegs<LM::MAXB, RL> kreg{h};
  CtRun<false, L, T, TX, true, SYNC_BLOCK, 1, true, Rs...>::run(threadIdx.x, s_tw, RegSrc<MB1, R1>{kp}, S, kreg);
  __syncthreads();
  MulH<TX, LM::MAXB, RL> mul{lds, h, conjH};
  CtRun<false, L, T, TX, true, SYNC_BLOCK, 1, true, Rs...>::run(threadIdx.x, s_tw, RegSrc<MB1, R1>{dp}, S, mul);
  Plain<GTile> out{g};
  CtRun<true, L, T, TX, true, SYNC_BLOCK, 1, true, Rs...>::run(threadIdx.x, s_tw, S, S, out);
}

template <int T, int TX, int L, int... Rs>
__global__ void __launch_bounds__(T)
    k_zconv_ct(const JobDesc* __restrict__ jobs, int njobs, const FftPlan* __restrict__ plans,
               const float2* __restrict__ twp, int v, int role, int conjH, int src_saved) {
  __shared__ float2 lds[L * TX];
  __shared__ float2 s_tw[L];
  int local;
  const int jid = find_job(jobs, njobs, PASS_Z, TX, local);
  if (jid < 0) return;
  const JobDesc& J = jobs[jid];
  if (v >= J.nviews) return;
  zconv_tile<T, TX, L, Rs...>(lds, s_tw, J, local, plans, twp, v, role, conjH, src_saved);
}

// ---------------------------------------------------------------------------
// Column passes over blocks of several lengths in one launch: a class of
// per-length plans ColPlan<L, radices...> sharing one thread count; every
// workgroup runs the plan of its job's length (jobs sorted by length, so
// the workgroups in flight mostly share one plan's code), in LDS sized for
// the class's longest length; TX lines per tile.
template <int L, int... Rs>
struct ColPlan {};

template <class P>
struct ColRun;
template <int L, int... Rs>
struct ColRun<ColPlan<L, Rs...>> {
  template <bool INV, int T, int TX>
  static __device__ __forceinline__ bool y(int n, float2* lds, float2* s_tw, const JobDesc& J, int local,
                                           const FftPlan* __restrict__ plans, const float2* __restrict__ twp) {
    if (n != L) return false;
    ypass_tile<INV, T, TX, L, Rs...>(lds, s_tw, J, local, plans, twp);
    return true;
  }
  template <int T, int TX>
  static __device__ __forceinline__ bool z(int n, float2* lds, float2* s_tw, const JobDesc& J, int local,
                                           const FftPlan* __restrict__ plans, const float2* __restrict__ twp,
                                           int v, int role, int conjH, int src_saved) {
    if (n != L) return false;
    zconv_tile<T, TX, L, Rs...>(lds, s_tw, J, local, plans, twp, v, role, conjH, src_saved);
    return true;
  }
};

template <bool INV, int T, int TX, int LMAX, class... Ps>
__global__ void __launch_bounds__(T)
    k_ypass_class(const JobDesc* __restrict__ jobs, int njobs, const FftPlan* __restrict__ plans,
                  const float2* __restrict__ twp, int v) {
  __shared__ float2 lds[LMAX * TX];
  __shared__ float2 s_tw[LMAX];
  int local;
  const int jid = find_job(jobs, njobs, PASS_Y, TX, local);
  if (jid < 0) return;
  const JobDesc& J = jobs[jid];
  if (v >= J.nviews) return;
  (void)(ColRun<Ps>::template y<INV, T, TX>(J.ny, lds, s_tw, J, local, plans, twp) || ...);
}

template <int T, int TX, int LMAX, class... Ps>
__global__ void __launch_bounds__(T)
    k_zconv_class(const JobDesc* __restrict__ jobs, int njobs, const FftPlan* __restrict__ plans,
                  const float2* __restrict__ twp, int v, int role, int conjH, int src_saved) {
  __shared__ float2 lds[LMAX * TX];
  __shared__ float2 s_tw[LMAX];
  int local;
  const int jid = find_job(jobs, njobs, PASS_Z, TX, local);
  if (jid < 0) return;
  const JobDesc& J = jobs[jid];
  if (v >= J.nviews) return;
  (void)(ColRun<Ps>::template z<T, TX>(J.nz, lds, s_tw, J, local, plans, twp, v, role, conjH, src_saved) || ...);
}

// ---------------------------------------------------------------------------
// The differentiated form's z pass (see k_zext in mvd_adjoint.hip): the
// z pass with the product, plus the forward spectrum stored and the FP64
// PSF cross-spectrum accumulated in the product's epilogue.
template <int T, int TX, int L, int... Rs>
__global__ void __launch_bounds__(T)
    k_zext_ct(const JobDesc* __restrict__ jobs, int njobs, const FftPlan* __restrict__ plans,
              const float2* __restrict__ twp, int v, int role, int conjH, float2* __restrict__ s_out,
              const float2* __restrict__ s_in, double2* __restrict__ acc, int acc_mode) {
  constexpr int RL = LastRadix<Rs...>::value;
  using LM = LastMap<L, RL, T, TX, true>;
  __shared__ float2 lds[L * TX];
  __shared__ float2 s_tw[L];
  int local;
  const int jid = find_job(jobs, njobs, PASS_Z, TX, local);
  if (jid < 0) return;
  const JobDesc& J = jobs[jid];
  const int M = J.M, ny = J.ny;
  const int nxt = mvd_cdiv(M, TX);
  int64_t off, hoff;
  int ps, nl;
  if (local < nxt * ny) {
    const int xt = local % nxt, y = local / nxt;
    off = (int64_t)y * J.Mp + xt * TX;
    hoff = off;
    ps = ny * J.Mp;
    nl = min(TX, M - xt * TX);
  } else {
    const int t2 = local - nxt * ny;
    off = J.spec_main + (int64_t)t2 * TX;
    hoff = J.h_main + (int64_t)t2 * TX;
    ps = ny;
    nl = min(TX, ny - t2 * TX);
  }
  const KLine kl{reinterpret_cast<const float2*>(J.H[role]) + (int64_t)v * J.h_elems + hoff, ps, nl, L,
                 J.kz, J.cz};
  GTile g{reinterpret_cast<float2*>(J.spec) + off, 1, ps, nl};
  const GTileU gin{reinterpret_cast<const float2*>(J.spec) + off, 1, ps, nl};
  constexpr int R1 = FirstRadix<Rs...>::value;
  constexpr int MB1 = FirstMap<L, R1, T, TX>::MAXB;
  constexpr int NTW = (L + T - 1) / T;
  const float2* twsrc = twp + plans[J.plan_z].tw;
  float2 twv[NTW];
#pragma unroll
  for (int i = 0; i < NTW; ++i) {
    const int e = threadIdx.x + i * T;
    twv[i] = e < L ? ldg(twsrc + e) : make_float2(0.f, 0.f);
  }
  float2 kp[MB1][R1], dp[MB1][R1];
  ct_prefetch<L, R1, T, TX, true>(threadIdx.x, kl, kp);
  ct_prefetch<L, R1, T, TX, true>(threadIdx.x, gin, dp);
#pragma unroll
  for (int i = 0; i < NTW; ++i) {
    const int e = threadIdx.x + i * T;
    if (e < L) s_tw[e] = twv[i];
  }
  const LdsCol<TX> S{lds};
  float2 h[LM::MAXB][RL];
  ToRegs<LM::MAXB, RL> kreg{h};
  CtRun<false, L, T, TX, true, SYNC_BLOCK, 1, true, Rs...>::run(threadIdx.x, s_tw, RegSrc<MB1, R1>{kp}, S, kreg);
  __syncthreads();
  ExtMul<TX, LM::MAXB, RL> ext{lds, h, conjH, off, ps, nl, s_out, s_in, acc, acc_mode};
  CtRun<false, L, T, TX, true, SYNC_BLOCK, 1, true, Rs...>::run(threadIdx.x, s_tw, RegSrc<MB1, R1>{dp}, S, ext);
  Plain<GTile> out{g};
  CtRun<true, L, T, TX, true, SYNC_BLOCK, 1, true, Rs...>::run(threadIdx.x, s_tw, S, S, out);
}

// ---------------------------------------------------------------------------
// x pass (see k_xpass): MODE 0 R2C of psi, MODE 1 blur -> ratio -> R2C,
// MODE 2 back-projection -> update -> R2C.  One wave owns RPW rows.
template <int MODE_, int WPB, int RPW, int M, int... Rs>
__global__ void __launch_bounds__(64 * WPB)
    k_xpass_ct(const JobDesc* __restrict__ jobs, int njobs, const FftPlan* __restrict__ plans,
               const float2* __restrict__ twp, int v, Partial* __restrict__ parts, int* __restrict__ flags,
               int opt) {
  constexpr int T = 64 * WPB;
  constexpr int MODE = MODE_ & 7;
  // the block-wise form's modes (0 and 2 reading and writing the volume)
  constexpr bool WIN = (MODE_ & XMODE_WIN) != 0;
  constexpr bool UPD = MODE == 2 || MODE == 4;  // modes that write psi
  constexpr int RW = WPB * RPW;
  constexpr int NPAIR = M / 2 + 1;
  constexpr int NPIT = (RPW * NPAIR + 63) / 64;
  constexpr int RL = LastRadix<Rs...>::value;
  using LM = LastMap<M, RL, 64, RPW, false>;
  __shared__ float2 lds[RW * M];
  __shared__ float2 s_tw[M];
  __shared__ float2 s_pp[M];
  __shared__ double rf[WPB];
  __shared__ unsigned ra[WPB], rb[WPB];
  // block-wise form: per row of the workgroup, the volume offset of its
  // window row (MODE 0) or of its own row (MODE 2; -1 for halo rows)
  __shared__ int64_t s_rows[WIN ? RW : 1];
  int local;
  const int jid = find_job(jobs, njobs, PASS_X, RW, local, true);
  if (jid < 0) return;
  const JobDesc& J = jobs[jid];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  bool skip = MODE != 0 && v >= J.nviews;
  if (WIN && !skip) {
    int any = 0;
    for (int t = tid; t < RW; t += T) {
      const int r = local * RW + t;
      int64_t o = -1;
      if (r < J.ny * J.nz) {
        const int y = r % J.ny, z = r / J.ny;
        if (MODE == 0)
          o = ((int64_t)((J.sz + z) % J.vnz) * J.vny + (J.sy + y) % J.vny) * J.vnx;
        else if (y >= J.hy && y < J.hy + J.ey && z >= J.hz && z < J.hz + J.ez)
          o = ((int64_t)(J.oz + z - J.hz) * J.vny + (J.oy + y - J.hy)) * J.vnx;
      }
      s_rows[t] = o;
      any |= o >= 0;
    }
    // an update workgroup of halo rows only has nothing to write
    skip = !__syncthreads_or(any);
  }
  if (skip) {
    if (tid == 0 && parts) {
      if (MODE == 1) {
        parts[blockIdx.x].ratio_clamps = 0;
      } else {
        parts[blockIdx.x].flux = 0.0;
        parts[blockIdx.x].neg_clamps = 0;
      }
    }
    return;
  }
  const int nx = J.nx;
  const bool first = opt & XOPT_FIRST, geo = opt & XOPT_GEO;
  load_table<T>(s_tw, twp + plans[J.plan_x].tw, M);
  load_table<T>(s_pp, twp + J.pp, M);
  const int wrow0 = local * RW + wave * RPW;
  const int nrw = max(0, min(RPW, J.ny * J.nz - wrow0));
  const auto spec = gp(reinterpret_cast<float2*>(J.spec));
  const auto nyq = spec + J.spec_main;
  const LdsRow<M> L{lds + wave * RPW * M};
  const int64_t vo = (int64_t)v * J.V;
  const int64_t rowoff = (int64_t)wrow0 * nx;
  double flux = 0.0;
  unsigned ncr = 0, ncn = 0;
  bool bad = false;

  if (MODE == 0) {
    __syncthreads();  // twiddle tables
    Plain<LdsRow<M>> out{L};
    if (WIN) {
      const WinRow src{J.vol, s_rows + wave * RPW, J.sx, J.vnx, nrw};
      CtRun<false, M, 64, RPW, false, SYNC_WAVE, 1, true, Rs...>::run(lane, s_tw, src, L, out);
    } else {
      const GRow src{J.psi + rowoff, nx, nrw};
      CtRun<false, M, 64, RPW, false, SYNC_WAVE, 1, true, Rs...>::run(lane, s_tw, src, L, out);
    }
  } else {
    // operands of the pointwise step, in the order the last inverse stage
    // produces its outputs
    float2 pa[LM::MAXB][RL], pb[LM::MAXB][RL];
    const float* opa = MODE == 1   ? J.phi + vo + rowoff
                       : MODE == 2 ? J.psi + rowoff
                                   : (first ? nullptr : J.acc + rowoff);
    const float* opb = MODE == 2   ? (J.w ? J.w + vo + rowoff : nullptr)
                       : MODE == 4 ? J.psi + rowoff
                                   : nullptr;
#pragma unroll
    for (int i = 0; i < LM::MAXB; ++i) {
      int line, j;
      const bool ok = LM::at(lane, i, line, j) && line < nrw;
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        const int64_t g = (int64_t)line * nx + 2 * (j + r * LM::NB);
        if (MODE == 2 && WIN) {
          // psi of the own voxels from the volume
          const int64_t b = ok ? s_rows[wave * RPW + line] : -1;
          const int x = 2 * (j + r * LM::NB) - J.hx;
          const float* q = J.vol + b + J.ox + x;
          pa[i][r] = make_float2(b >= 0 && x >= 0 && x < J.ex ? ldg(q) : 0.f,
                                 b >= 0 && x + 1 >= 0 && x + 1 < J.ex ? ldg(q + 1) : 0.f);
        } else {
          pa[i][r] = (ok && opa) ? ld2(opa + g) : make_float2(0.f, 0.f);
        }
        pb[i][r] = ((MODE == 2 || MODE == 4) && ok && opb) ? ld2(opb + g) : make_float2(0.f, 0.f);
      }
    }
    // rebuild the M-point spectrum Z of these rows from their half spectrum X
    float2 xa[NPIT], xb[NPIT];
#pragma unroll
    for (int i = 0; i < NPIT; ++i) {
      const int it = lane + i * 64;
      const int r = it / NPAIR, k = it % NPAIR;
      if (r < nrw) {
        const int64_t rbase = (int64_t)(wrow0 + r) * J.Mp;
        xa[i] = spec[rbase + k];
        xb[i] = (k == 0) ? nyq[wrow0 + r] : spec[rbase + M - k];
      }
    }
    __syncthreads();  // twiddle tables
#pragma unroll
    for (int i = 0; i < NPIT; ++i) {
      const int it = lane + i * 64;
      const int r = it / NPAIR, k = it % NPAIR;
      if (r < nrw) {
        const float2 a = xa[i], b = xb[i], t = s_pp[k];
        // Z[k] = (a + conj b) + i conj(t) (a - conj b)
        const float2 s = make_float2(a.x + b.x, a.y - b.y);
        const float2 d = make_float2(a.x - b.x, a.y + b.y);
        const float2 e = cmul(cconj(t), d);
        L.st(r, k, make_float2(s.x - e.y, s.y + e.x));
        if (k != 0 && 2 * k != M) {
          // Z[M-k] = (b + conj a) - i t (b - conj a)
          const float2 s2 = make_float2(b.x + a.x, b.y - a.y);
          const float2 d2 = make_float2(b.x - a.x, b.y + a.y);
          const float2 e2 = cmul(t, d2);
          L.st(r, M - k, make_float2(s2.x + e2.y, s2.y - e2.x));
        }
      }
    }
    gsync<SYNC_WAVE>();
    RowOp<MODE_, M, LM::MAXB, RL> op{L.p,   pa,    pb,  J.psi + rowoff,
                                    (MODE == 3 || MODE == 4) ? J.acc + rowoff : nullptr,
                                    J.vol, s_rows + wave * RPW, J.ox, J.hx, J.ex,
                                    nx,    nrw,   opb != nullptr,  first, geo,
                                    J.eps, J.lamp, 1.f / (float)J.nviews, 0.0, 0u, 0u, false};
    CtRun<true, M, 64, RPW, false, SYNC_WAVE, 1, true, Rs...>::run(lane, s_tw, L, L, op);
    flux = op.flux;
    ncr = op.ncr;
    ncn = op.ncn;
    bad = op.bad;
    if (MODE == 1 || (UPD && (opt & XOPT_SPEC))) {
      Plain<LdsRow<M>> out{L};
      CtRun<false, M, 64, RPW, false, SYNC_WAVE, 1, true, Rs...>::run(lane, s_tw, L, L, out);
    }
  }

  if (MODE == 0 || MODE == 1 || (UPD && (opt & XOPT_SPEC))) {
    // half spectrum of the rows from the M-point transform
#pragma unroll
    for (int i = 0; i < NPIT; ++i) {
      const int it = lane + i * 64;
      const int r = it / NPAIR, k = it % NPAIR;
      if (r < nrw) {
        const int64_t rbase = (int64_t)(wrow0 + r) * J.Mp;
        const float2 zk = L.ld(r, k);
        if (k == 0) {
          spec[rbase] = make_float2(zk.x + zk.y, 0.f);
          nyq[wrow0 + r] = make_float2(zk.x - zk.y, 0.f);
        } else {
          const float2 zm = L.ld(r, M - k);
          const float2 t = s_pp[k];
          const float2 s = make_float2(zk.x + zm.x, zk.y - zm.y);
          const float2 d = make_float2(zk.x - zm.x, zk.y + zm.y);
          const float2 e = cmul(t, d);
          spec[rbase + k] = make_float2(0.5f * (s.x + e.y), 0.5f * (s.y - e.x));
          if (2 * k != M) {
            const float2 s2 = make_float2(zm.x + zk.x, zm.y - zk.y);
            const float2 d2 = make_float2(zm.x - zk.x, zm.y + zk.y);
            const float2 e2 = cmul(cconj(t), d2);
            spec[rbase + M - k] = make_float2(0.5f * (s2.x - e2.y), 0.5f * (s2.y + e2.x));
          }
        }
      }
    }
  }

  if (MODE != 0) {
    if (UPD && bad) atomicOr(flags, 1);
    if (parts) {
      block_reduce<T>(flux, ncr, ncn, rf, ra, rb);
      if (tid == 0) {
        if (MODE == 1) {
          parts[blockIdx.x].ratio_clamps = ncr;
        } else {
          parts[blockIdx.x].flux = flux;
          parts[blockIdx.x].neg_clamps = ncn;
        }
      }
    }
  }
}

}  // namespace mvdk
