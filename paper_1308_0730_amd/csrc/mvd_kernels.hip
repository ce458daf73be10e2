// gfx950 kernels of the sequential multi-view update.
//
// One view-update (section 7) is two circular convolutions and the pointwise
// steps of eq. 15 around them.  With the x axis transformed real-to-complex
// (half spectrum), one convolution is four passes over the volume:
//
//   y forward  ->  z forward, x H_v, z inverse  ->  y inverse  ->  x pass
//
// and the x pass of the first convolution (blur with P_v) is fused with the
// ratio phi_v / max(b, eps) and the forward x transform of the ratio; the x
// pass of the second (back-projection with K_v) is fused with the
// multiplicative update, the Tikhonov step, the weight blend, the FP64 flux
// partials and the forward x transform of the new estimate, which is the
// input of the next view's blur.  So a view-update is 8 launches and every
// voxel crosses HBM 8 times (plus the reads of phi_v, w_v and the spectra).
// The 1/V of the inverse transforms is folded into the stored spectra.
#include <hip/hip_runtime.h>

#include "fft_engine.h"
#include "mvd_device.h"
#include "mvd.h"
#include "mvd_kernels.h"

using namespace mvdk;


// ---------------------------------------------------------------------------
// x pass.  MODE 0: forward real-to-complex of psi.  MODE 1: inverse x of the
// blurred spectrum -> b, q = phi / max(b, eps), forward x of q.  MODE 2:
// inverse x of the back-projected spectrum -> c, update psi, forward x of the
// new psi (when opt has XOPT_SPEC).  Combined updates (eq. 51): MODE 3
// folds max(c, 0) of one view into the factor acc (product, or sum); MODE 4
// does the same for the last view, then psi <- T(psi . mean) with the
// |V|-th root of the product or the sum over |V|, and the forward x of the
// new psi (when opt has XOPT_SPEC).  Where the view holds MVD_NO_DATA (grid
// voxels outside the volume with the linear boundary) the ratio is 1.
//
// A row of nx reals is handled as M = nx/2 complex values z[n] = x[2n] +
// i x[2n+1]; the half spectrum follows from the M-point transform Z by
//   X[k] = (Z[k] + conj Z[M-k])/2 - i e^{-2 pi i k/nx} (Z[k] - conj Z[M-k])/2
// and the inverse rebuilds Z from X before an M-point inverse transform.
// Each wave owns RPW whole rows and its own LDS region, so after the table
// load the transforms synchronise per wave only.
template <int MODE, int WPB, int RPW, int MAXM>
__global__ void __launch_bounds__(64 * WPB)
    k_xpass(const JobDesc* __restrict__ jobs, int njobs, const FftPlan* __restrict__ plans,
            const float2* __restrict__ twp, int v, Partial* __restrict__ parts, int* __restrict__ flags,
            int opt) {
  constexpr int T = 64 * WPB;
  constexpr int RW = WPB * RPW;
  constexpr int EPT = (RPW * MAXM + 63) / 64;
  constexpr bool UPD = MODE == 2 || MODE == 4;  // modes that write psi
  constexpr int NPIT = (RPW * (MAXM / 2 + 1) + 63) / 64;
  __shared__ float2 lds[RW * MAXM];
  __shared__ float2 s_tw[MAXM];
  __shared__ float2 s_pp[MAXM];
  __shared__ double rf[WPB];
  __shared__ unsigned ra[WPB], rb[WPB];
  int local;
  const int jid = find_job(jobs, njobs, PASS_X, RW, local, true);
  if (jid < 0) return;
  const JobDesc& J = jobs[jid];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  if (MODE != 0 && v >= J.nviews) {
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
  const int M = J.M, nx = J.nx;
  const bool first = opt & XOPT_FIRST, geo = opt & XOPT_GEO;
  const float inv_n = 1.f / (float)J.nviews;
  const FftPlan* pl = plans + J.plan_x;
  load_table<T>(s_tw, twp + pl->tw, M);
  load_table<T>(s_pp, twp + J.pp, M);
  const int wrow0 = local * RW + wave * RPW;
  const int nrw = max(0, min(RPW, J.ny * J.nz - wrow0));
  const auto spec = gp(reinterpret_cast<float2*>(J.spec));
  const auto nyq = spec + J.spec_main;
  const LdsRow<MAXM> L{lds + wave * RPW * MAXM};
  const int npair = M / 2 + 1;
  const unsigned mM = mvd_magic(M), mP = mvd_magic(npair);
  const int64_t vo = (int64_t)v * J.V;
  const float eps = J.eps, lamp = J.lamp;
  const float* wv = J.w ? J.w + vo : nullptr;

  // prefetch the pointwise operands of this lane's elements
  float2 pa[EPT], pb[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int it = lane + i * 64;
    const int r = RPW == 1 ? 0 : udiv(it, mM);
    const int p = it - r * M;
    pa[i] = pb[i] = make_float2(0.f, 0.f);
    if (r < nrw && p < M) {
      const int64_t g = (int64_t)(wrow0 + r) * nx + 2 * p;
      if (MODE == 1) pa[i] = ld2(J.phi + vo + g);
      if (MODE == 0 || MODE == 2) pa[i] = ld2(J.psi + g);
      if (MODE == 2 && wv) pb[i] = ld2(wv + g);
      if ((MODE == 3 || MODE == 4) && !first) pa[i] = ld2(J.acc + g);
      if (MODE == 4) pb[i] = ld2(J.psi + g);
    }
  }

  double flux = 0.0;
  unsigned ncr = 0, ncn = 0;
  bool bad = false;
  if (MODE == 0) {
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int it = lane + i * 64;
      const int r = RPW == 1 ? 0 : udiv(it, mM);
      const int p = it - r * M;
      if (r < nrw && p < M) L.st(r, p, pa[i]);
    }
    __syncthreads();  // twiddle tables and this wave's rows
  } else {
    // rebuild the M-point spectrum Z of these rows from their half spectrum X
    float2 xa[NPIT], xb[NPIT];
#pragma unroll
    for (int i = 0; i < NPIT; ++i) {
      const int it = lane + i * 64;
      const int r = RPW == 1 ? 0 : udiv(it, mP);
      const int k = it - r * npair;
      if (r < nrw && k < npair) {
        const int64_t rbase = (int64_t)(wrow0 + r) * J.Mp;
        xa[i] = spec[rbase + k];
        xb[i] = (k == 0) ? nyq[wrow0 + r] : spec[rbase + M - k];
      }
    }
    __syncthreads();  // twiddle tables
#pragma unroll
    for (int i = 0; i < NPIT; ++i) {
      const int it = lane + i * 64;
      const int r = RPW == 1 ? 0 : udiv(it, mP);
      const int k = it - r * npair;
      if (r < nrw && k < npair) {
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
    fft_lines<true, MAXM, 64, RPW, false, SYNC_WAVE>(pl, s_tw, lane, L, L, L);

    // pointwise step on the real values held two per complex entry
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int it = lane + i * 64;
      const int r = RPW == 1 ? 0 : udiv(it, mM);
      const int p = it - r * M;
      if (r < nrw && p < M) {
        const float2 z = L.ld(r, p);
        float2 o;
        if (MODE == 1) {
          o = ratio2(pa[i], z, eps, ncr);
        } else if (MODE == 3 || MODE == 4) {
          ncn += (z.x < 0.f) + (z.y < 0.f);
          const float cx = z.x > 0.f ? z.x : 0.f, cy = z.y > 0.f ? z.y : 0.f;
          float mx = cx, my = cy;
          if (!first) {
            mx = geo ? pa[i].x * cx : pa[i].x + cx;
            my = geo ? pa[i].y * cy : pa[i].y + cy;
          }
          const int64_t g = (int64_t)(wrow0 + r) * nx + 2 * p;
          if (MODE == 3) {
            st2(J.acc + g, make_float2(mx, my));
            o = make_float2(mx, my);
          } else {
            const float gx = geo ? powf(mx, inv_n) : mx * inv_n;
            const float gy = geo ? powf(my, inv_n) : my * inv_n;
            o = make_float2(tikhonov(pb[i].x * gx, lamp), tikhonov(pb[i].y * gy, lamp));
            st2(J.psi + g, o);
            flux += (double)o.x + (double)o.y;
            bad |= !(isfinite(o.x) && isfinite(o.y));
          }
        } else {
          ncn += (z.x < 0.f) + (z.y < 0.f);
          const float ux = pa[i].x * (z.x > 0.f ? z.x : 0.f);
          const float uy = pa[i].y * (z.y > 0.f ? z.y : 0.f);
          const float tx = tikhonov(ux, lamp), ty = tikhonov(uy, lamp);
          if (wv) {
            o = make_float2(pa[i].x + pb[i].x * (tx - pa[i].x), pa[i].y + pb[i].y * (ty - pa[i].y));
          } else {
            o = make_float2(tx, ty);
          }
          st2(J.psi + (int64_t)(wrow0 + r) * nx + 2 * p, o);
          flux += (double)o.x + (double)o.y;
          bad |= !(isfinite(o.x) && isfinite(o.y));
        }
        L.st(r, p, o);
      }
    }
    gsync<SYNC_WAVE>();
  }

  if (MODE == 0 || MODE == 1 || (UPD && (opt & XOPT_SPEC))) {
    fft_lines<false, MAXM, 64, RPW, false, SYNC_WAVE>(pl, s_tw, lane, L, L, L);
    // half spectrum of the rows from the M-point transform
#pragma unroll
    for (int i = 0; i < NPIT; ++i) {
      const int it = lane + i * 64;
      const int r = RPW == 1 ? 0 : udiv(it, mP);
      const int k = it - r * npair;
      if (r < nrw && k < npair) {
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

// ---------------------------------------------------------------------------
// y pass: complex transform along y of TX adjacent kx columns (main part) or
// TX z-lines of the Nyquist plane, in place.
template <bool INV, int T, int TX, int MAXL>
__global__ void __launch_bounds__(T)
    k_ypass(const JobDesc* __restrict__ jobs, int njobs, const FftPlan* __restrict__ plans,
            const float2* __restrict__ twp, int v) {
  __shared__ float2 lds[MAXL * TX];
  __shared__ float2 s_tw[MAXL];
  int local;
  const int jid = find_job(jobs, njobs, PASS_Y, TX, local);
  if (jid < 0) return;
  const JobDesc& J = jobs[jid];
  if (v >= J.nviews) return;
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
  const FftPlan* pl = plans + J.plan_y;
  // the table is read from the second stage on, after the first stage's barrier
  load_table<T>(s_tw, twp + pl->tw, ny);
  fft_lines<INV, MAXL, T, TX, true, SYNC_BLOCK>(pl, s_tw, threadIdx.x, g, LdsCol<TX>{lds}, g);
}

// ---------------------------------------------------------------------------
// z pass with the spectral product: forward z transform of the kernel lines
// of view v (their x/y-stage planes placed on the length-nz line), forward z
// transform of the data, multiply (by the conjugate for the mirrored kernel
// P_v*), inverse z transform, all while the tile stays in LDS.  With
// src_saved the tile is read from the job's saved spectrum (combined
// updates) and written to the work spectrum.
template <int T, int TX, int MAXL>
__global__ void __launch_bounds__(T)
    k_zconv(const JobDesc* __restrict__ jobs, int njobs, const FftPlan* __restrict__ plans,
            const float2* __restrict__ twp, int v, int role, int conjH, int src_saved) {
  __shared__ float2 lds[MAXL * TX];
  __shared__ float2 s_tw[MAXL];
  int local;
  const int jid = find_job(jobs, njobs, PASS_Z, TX, local);
  if (jid < 0) return;
  const JobDesc& J = jobs[jid];
  if (v >= J.nviews) return;
  const int M = J.M, ny = J.ny, nz = J.nz;
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
  const KLine kl{reinterpret_cast<const float2*>(J.H[role]) + (int64_t)v * J.h_elems + hoff, ps, nl, nz,
                 J.kz, J.cz};
  GTile g{reinterpret_cast<float2*>(J.spec) + off, 1, ps, nl};
  const GTile gin{reinterpret_cast<float2*>(src_saved ? J.saved : J.spec) + off, 1, ps, nl};
  constexpr int EPT = (TX * MAXL + T - 1) / T;
  const int tid = threadIdx.x;
  const FftPlan* pl = plans + J.plan_z;
  load_table<T>(s_tw, twp + pl->tw, nz);
  const LdsCol<TX> S{lds};
  if (pl->nst == 1) __syncthreads();
  // kernel spectrum of the tile's lines, kept in registers
  fft_lines<false, MAXL, T, TX, true, SYNC_BLOCK>(pl, s_tw, tid, kl, S, S);
  float2 h[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = tid + i * T;
    const int line = e % TX, pos = e / TX;
    h[i] = pos < nz ? S.ld(line, pos) : make_float2(0.f, 0.f);
  }
  __syncthreads();
  fft_lines<false, MAXL, T, TX, true, SYNC_BLOCK>(pl, s_tw, tid, gin, S, S);
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = tid + i * T;
    const int line = e % TX, pos = e / TX;
    if (pos < nz) {
      const float2 a = S.ld(line, pos);
      S.st(line, pos, cmul(a, conjH ? cconj(h[i]) : h[i]));
    }
  }
  __syncthreads();
  fft_lines<true, MAXL, T, TX, true, SYNC_BLOCK>(pl, s_tw, tid, S, S, g);
}

// ---------------------------------------------------------------------------
// Sum the per-tile partials of one iteration: block v handles view v.
__global__ void __launch_bounds__(256)
    k_reduce(const Partial* __restrict__ parts, int ntiles, double* __restrict__ flux,
             unsigned long long* __restrict__ ratio, unsigned long long* __restrict__ neg) {
  __shared__ double sf[256];
  __shared__ unsigned long long sa[256], sb[256];
  const Partial* p = parts + (int64_t)blockIdx.x * ntiles;
  double f = 0.0;
  unsigned long long a = 0, b = 0;
  for (int t = threadIdx.x; t < ntiles; t += 256) {
    f += p[t].flux;
    a += p[t].ratio_clamps;
    b += p[t].neg_clamps;
  }
  sf[threadIdx.x] = f;
  sa[threadIdx.x] = a;
  sb[threadIdx.x] = b;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sf[threadIdx.x] += sf[threadIdx.x + s];
      sa[threadIdx.x] += sa[threadIdx.x + s];
      sb[threadIdx.x] += sb[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    flux[blockIdx.x] = sf[0];
    ratio[blockIdx.x] = sa[0];
    neg[blockIdx.x] = sb[0];
  }
}

// Count values that are non-finite or outside [lo, hi] and sum them in FP64,
// one partial per block (the host adds the partials in a fixed order).
__global__ void __launch_bounds__(256)
    k_check(const float* __restrict__ x, int64_t n, float lo, float hi, double* __restrict__ psum,
            unsigned long long* __restrict__ pbad) {
  __shared__ double sf[256];
  __shared__ unsigned long long sb[256];
  double f = 0.0;
  unsigned long long b = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const float a = x[i];
    if (!(a >= lo && a <= hi)) ++b;  // also catches NaN
    f += (double)a;
  }
  sf[threadIdx.x] = f;
  sb[threadIdx.x] = b;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sf[threadIdx.x] += sf[threadIdx.x + s];
      sb[threadIdx.x] += sb[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    psum[blockIdx.x] = sf[0];
    pbad[blockIdx.x] = sb[0];
  }
}

__global__ void __launch_bounds__(256) k_fill(float* __restrict__ x, int64_t n, float val) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    x[i] = val;
}

__global__ void k_set_int(int* __restrict__ p, int val) {
  if (threadIdx.x == 0) *p = val;
}

// ---------------------------------------------------------------------------
// Launch-shape candidates.  Column passes: (threads, lines per tile, max
// length).  Row passes: (threads, rows per tile, max half-row length).

#define MVD_COL_CFGS(X) \
  X(0, 64, 16, 64)      \
  X(1, 128, 16, 128)    \
  X(2, 256, 16, 256)    \
  X(3, 256, 16, 512)    \
  X(4, 256, 8, 512)     \
  X(5, 128, 8, 256)     \
  X(6, 512, 16, 512)    \
  X(7, 256, 32, 128)    \
  X(8, 256, 8, 256)

#define MVD_ROW_CFGS(X) \
  X(0, 4, 4, 32)        \
  X(1, 4, 2, 64)        \
  X(2, 4, 2, 128)       \
  X(3, 4, 1, 256)       \
  X(4, 4, 1, 512)       \
  X(5, 2, 1, 256)       \
  X(6, 8, 1, 256)       \
  X(7, 4, 1, 128)

static const int kColCfg[][3] = {
#define X(i, t, tx, l) {t, tx, l},
    MVD_COL_CFGS(X)
#undef X
};
static const int kRowCfg[][3] = {
#define X(i, wpb, rpw, m) {64 * wpb, wpb * rpw, m},
    MVD_ROW_CFGS(X)
#undef X
};

// Candidate indices: the runtime-plan shapes first, then the tuned
// compile-time ones (one exact length each), then one index for the
// compile-time plans of every 5-smooth length, launched per group of jobs of
// equal length (its shape depends on the length).
static int rt_num(int kind) {
  return kind == PASS_X ? (int)(sizeof(kRowCfg) / sizeof(kRowCfg[0]))
                        : (int)(sizeof(kColCfg) / sizeof(kColCfg[0]));
}
int mvd_exact_cfg(int kind) { return rt_num(kind) + mvd_ct_num_cfgs(kind); }
int mvd_num_cfgs(int kind) { return mvd_exact_cfg(kind) + 1; }
static int cfg_field(int kind, int cfg, int f) {
  const int n = rt_num(kind);
  if (cfg == mvd_exact_cfg(kind)) return f == 2 ? (kind == PASS_X ? MVD_MAX_LEN : MVD_MAX_LEN_YZ) : 0;
  if (cfg >= n) return mvd_ct_cfg(kind, cfg - n, f);
  return kind == PASS_X ? kRowCfg[cfg][f] : kColCfg[cfg][f];
}
int mvd_cfg_threads(int kind, int cfg) { return cfg_field(kind, cfg, 0); }
int mvd_cfg_param(int kind, int cfg) { return cfg_field(kind, cfg, 1); }
int mvd_cfg_maxlen(int kind, int cfg) { return cfg_field(kind, cfg, 2); }
int mvd_cfg_exact(int kind, int cfg) {
  if (cfg == mvd_exact_cfg(kind)) return -1;
  return cfg >= rt_num(kind) ? cfg_field(kind, cfg, 2) : 0;
}
int mvd_exact_param(int kind, int len) {
  int a = 0, b = 0;
  if (kind == PASS_X) return mvd_exact_row_shape(len, &a, &b) ? a * b : 0;
  return mvd_exact_col_shape(len, &a, &b) ? b : 0;
}

hipError_t mvd_launch_x(const LaunchArgs& a, int cfg, int mode, int v, Partial* parts, int* flags, int opt) {
  if (mode < 0 || mode > 4) return hipErrorInvalidValue;
  if (cfg >= rt_num(PASS_X)) return mvd_launch_x_ct(a, cfg - rt_num(PASS_X), mode, v, parts, flags, opt);
  switch (cfg) {
#define XM(md, wpb, rpw, m)                                                                              \
  case md:                                                                                               \
    k_xpass<md, wpb, rpw, m><<<a.grid, 64 * wpb, 0, a.stream>>>(a.jobs, a.njobs, a.plans, a.tw, v, parts, \
                                                                flags, opt);                             \
    break;
#define X(i, wpb, rpw, m)    \
  case i:                    \
    switch (mode) {          \
      XM(0, wpb, rpw, m)     \
      XM(1, wpb, rpw, m)     \
      XM(2, wpb, rpw, m)     \
      XM(3, wpb, rpw, m)     \
      XM(4, wpb, rpw, m)     \
    }                        \
    break;
    MVD_ROW_CFGS(X)
#undef X
#undef XM
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t mvd_launch_y(const LaunchArgs& a, int cfg, int inv, int v) {
  if (cfg >= rt_num(PASS_Y)) return mvd_launch_y_ct(a, cfg - rt_num(PASS_Y), inv, v);
  switch (cfg) {
#define X(i, t, tx, l)                                                                          \
  case i:                                                                                       \
    if (inv)                                                                                    \
      k_ypass<true, t, tx, l><<<a.grid, t, 0, a.stream>>>(a.jobs, a.njobs, a.plans, a.tw, v);  \
    else                                                                                        \
      k_ypass<false, t, tx, l><<<a.grid, t, 0, a.stream>>>(a.jobs, a.njobs, a.plans, a.tw, v); \
    break;
    MVD_COL_CFGS(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t mvd_launch_z(const LaunchArgs& a, int cfg, int v, int role, int conjH, int src_saved) {
  if (cfg >= rt_num(PASS_Z)) return mvd_launch_z_ct(a, cfg - rt_num(PASS_Z), v, role, conjH, src_saved);
  switch (cfg) {
#define X(i, t, tx, l)                                                                                         \
  case i:                                                                                                      \
    k_zconv<t, tx, l><<<a.grid, t, 0, a.stream>>>(a.jobs, a.njobs, a.plans, a.tw, v, role, conjH, src_saved); \
    break;
    MVD_COL_CFGS(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t mvd_launch_reduce(const Partial* parts, int ntiles, int nviews, double* flux,
                             unsigned long long* ratio, unsigned long long* neg, hipStream_t s) {
  k_reduce<<<nviews, 256, 0, s>>>(parts, ntiles, flux, ratio, neg);
  return hipGetLastError();
}

hipError_t mvd_launch_check(const float* x, int64_t n, float lo, float hi, double* psum,
                            unsigned long long* pbad, int nblocks, hipStream_t s) {
  k_check<<<nblocks, 256, 0, s>>>(x, n, lo, hi, psum, pbad);
  return hipGetLastError();
}

hipError_t mvd_launch_fill(float* x, int64_t n, float val, hipStream_t s) {
  int64_t nb = (n + 255) / 256;
  if (nb > 4096) nb = 4096;
  if (nb < 1) nb = 1;
  k_fill<<<(int)nb, 256, 0, s>>>(x, n, val);
  return hipGetLastError();
}

hipError_t mvd_launch_set_int(int* p, int val, hipStream_t s) {
  k_set_int<<<1, 64, 0, s>>>(p, val);
  return hipGetLastError();
}

