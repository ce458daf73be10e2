// Passes of the differentiated form: the forward with the intermediates
// stored, the loss, and the adjoint of every step of a view-update, in
// reverse (runtime-plan transforms for any 5-smooth size; compile-time plans
// for the x passes of power-of-two half-rows).
//
// Adjoint of one RL view-update (K_v = P_v*), given g = dL/dpsi':
//   tbar = w g;  ubar = tbar / sqrt(1 + 4 lambda' u);  cbar = ubar psi [c > 0]
//   psibar = (1 - w) g + ubar max(c, 0) + bbar (x) P_v*
//   qbar = cbar (x) P_v;  bbar = -qbar q / b [b > eps]
//   dL/dP_v[d] += sum_x bbar(x) psi(x - d) + sum_x cbar(x) q(x + d)
// The PSF terms are accumulated in the frequency domain (FP64):
//   A_v += Bbar conj(Psi) + conj(Cbar) Q
// from the spectra the z passes hold anyway; one inverse DFT per view at the
// end gives dL/dP_v on its window.
#include <hip/hip_runtime.h>

#include "fft_ct.h"
#include "fft_engine.h"
#include "mvd_device.h"
#include "mvd_exact_lengths.h"
#include "mvd_kernels.h"

using namespace mvdk;

// x pass of the differentiated form.  MODE: 3 blur -> ratio (stores b, q);
// 4 back-projection -> update (stores c and the input psi); 5 adjoint of the
// update (no inverse transform; writes the direct part of psibar, forward
// transform of cbar); 6 adjoint of the ratio (inverse -> qbar, forward of
// bbar); 7 finish (inverse -> s, out = part + s, no forward transform);
// 8 loss residual (inverse -> b, r = b - phi, FP64 sum of r^2, forward of 2r).
// Row transforms of the adjoint x passes: the runtime plan, or with radices
// Rs the compile-time plan of length MAXM (the block's M).
template <bool INV, int MAXM, int RPW, int... Rs>
__device__ __forceinline__ void xadj_lines(const FftPlan* pl, const float2* s_tw, int lane, const LdsRow<MAXM>& L) {
  if constexpr (sizeof...(Rs) == 0) {
    fft_lines<INV, MAXM, 64, RPW, false, SYNC_WAVE>(pl, s_tw, lane, L, L, L);
  } else {
    Plain<LdsRow<MAXM>> out{L};
    CtRun<INV, MAXM, 64, RPW, false, SYNC_WAVE, 1, true, Rs...>::run(lane, s_tw, L, L, out);
  }
}

template <int MODE, int WPB, int RPW, int MAXM, int... Rs>
__global__ void __launch_bounds__(64 * WPB)
    k_xadj(const JobDesc* __restrict__ jobs, int njobs, const FftPlan* __restrict__ plans,
           const float2* __restrict__ twp, int v, Partial* __restrict__ parts, int* __restrict__ flags,
           AdjPtrs ap) {
  constexpr int T = 64 * WPB;
  constexpr int RW = WPB * RPW;
  constexpr int EPT = (RPW * MAXM + 63) / 64;
  constexpr int NPIT = (RPW * (MAXM / 2 + 1) + 63) / 64;
  constexpr bool C2R = MODE != 5;
  constexpr bool R2C = MODE != 7;
  __shared__ float2 lds[RW * MAXM];
  __shared__ float2 s_tw[MAXM];
  __shared__ float2 s_pp[MAXM];
  __shared__ double rf[WPB];
  __shared__ unsigned ra[WPB], rb[WPB];
  int local;
  const int jid = find_job(jobs, njobs, PASS_X, RW, local);
  if (jid < 0) return;
  const JobDesc& J = jobs[jid];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int M = J.M, nx = J.nx;
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

  auto f2 = [](const float* p, int64_t g) { return ld2(p + g); };
  float2 pa[EPT], pb[EPT], pc[EPT], pd[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int it = lane + i * 64;
    const int r = RPW == 1 ? 0 : udiv(it, mM);
    const int p = it - r * M;
    const float2 one = make_float2(1.f, 1.f), zero = make_float2(0.f, 0.f);
    pa[i] = pb[i] = pc[i] = pd[i] = zero;
    if (r < nrw && p < M) {
      const int64_t g = (int64_t)(wrow0 + r) * nx + 2 * p;
      if (MODE == 3 || MODE == 8) pa[i] = f2(J.phi + vo, g);
      if (MODE == 4) {
        pa[i] = f2(J.psi, g);
        pb[i] = wv ? f2(wv, g) : one;
      }
      if (MODE == 5) {
        pa[i] = f2(ap.gbar, g);
        pb[i] = wv ? f2(wv, g) : one;
        pc[i] = f2(ap.psi_in, g);
        pd[i] = f2(ap.c, g);
      }
      if (MODE == 6) {
        pa[i] = f2(ap.q, g);
        pb[i] = f2(ap.b, g);
      }
      if (MODE == 7) pa[i] = f2(ap.part, g);
    }
  }

  double acc = 0.0;
  unsigned ncr = 0, ncn = 0;
  bool bad = false;
  if (C2R) {
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
        const float2 s = make_float2(a.x + b.x, a.y - b.y);
        const float2 d = make_float2(a.x - b.x, a.y + b.y);
        const float2 e = cmul(cconj(t), d);
        L.st(r, k, make_float2(s.x - e.y, s.y + e.x));
        if (k != 0 && 2 * k != M) {
          const float2 s2 = make_float2(b.x + a.x, b.y - a.y);
          const float2 d2 = make_float2(b.x - a.x, b.y + a.y);
          const float2 e2 = cmul(t, d2);
          L.st(r, M - k, make_float2(s2.x + e2.y, s2.y - e2.x));
        }
      }
    }
    gsync<SYNC_WAVE>();
    xadj_lines<true, MAXM, RPW, Rs...>(pl, s_tw, lane, L);
  } else {
    __syncthreads();  // twiddle tables
  }

#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int it = lane + i * 64;
    const int r = RPW == 1 ? 0 : udiv(it, mM);
    const int p = it - r * M;
    if (r < nrw && p < M) {
      const int64_t g = (int64_t)(wrow0 + r) * nx + 2 * p;
      const float2 z = C2R ? L.ld(r, p) : make_float2(0.f, 0.f);
      float2 o = make_float2(0.f, 0.f);
      if (MODE == 3) {
        ncr += (z.x < eps) + (z.y < eps);
        o = make_float2(pa[i].x / fmaxf(z.x, eps), pa[i].y / fmaxf(z.y, eps));
        st2(ap.b + g, z);
        st2(ap.q + g, o);
      } else if (MODE == 4) {
        ncn += (z.x < 0.f) + (z.y < 0.f);
        const float2 ps = pa[i];
        const float tx = tikhonov(ps.x * (z.x > 0.f ? z.x : 0.f), lamp);
        const float ty = tikhonov(ps.y * (z.y > 0.f ? z.y : 0.f), lamp);
        o = wv ? make_float2(ps.x + pb[i].x * (tx - ps.x), ps.y + pb[i].y * (ty - ps.y)) : make_float2(tx, ty);
        st2(ap.c + g, z);
        st2(ap.psi_in + g, ps);
        st2(J.psi + g, o);
        acc += (double)o.x + (double)o.y;
        bad |= !(isfinite(o.x) && isfinite(o.y));
      } else if (MODE == 5) {
        // g = pa, w = pb, psi = pc, c = pd
        float od[2], cb[2];
        const float gg[2] = {pa[i].x, pa[i].y}, ww[2] = {pb[i].x, pb[i].y};
        const float ps[2] = {pc[i].x, pc[i].y}, cc[2] = {pd[i].x, pd[i].y};
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const float cp = cc[e] > 0.f ? cc[e] : 0.f;
          const float u = ps[e] * cp;
          const float dT = lamp > 0.f ? 1.f / sqrtf(1.f + 4.f * lamp * u) : 1.f;
          const float ub = ww[e] * gg[e] * dT;
          od[e] = ub * cp + (wv ? (1.f - ww[e]) * gg[e] : 0.f);
          cb[e] = cc[e] > 0.f ? ub * ps[e] : 0.f;
        }
        st2(ap.part + g, make_float2(od[0], od[1]));
        o = make_float2(cb[0], cb[1]);
      } else if (MODE == 6) {
        // qbar = z, q = pa, b = pb
        o = make_float2(pb[i].x > eps ? -z.x * pa[i].x / pb[i].x : 0.f,
                        pb[i].y > eps ? -z.y * pa[i].y / pb[i].y : 0.f);
      } else if (MODE == 7) {
        st2(ap.out + g, make_float2(pa[i].x + z.x, pa[i].y + z.y));
      } else if (MODE == 8) {
        const float rx = z.x - pa[i].x, ry = z.y - pa[i].y;
        acc += (double)rx * rx + (double)ry * ry;
        o = make_float2(2.f * rx, 2.f * ry);
      }
      if (R2C) L.st(r, p, o);
    }
  }
  gsync<SYNC_WAVE>();

  if (R2C) {
    xadj_lines<false, MAXM, RPW, Rs...>(pl, s_tw, lane, L);
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

  if (MODE == 4 && bad) atomicOr(flags, 1);
  if ((MODE == 3 || MODE == 4 || MODE == 8) && parts) {
    block_reduce<T>(acc, ncr, ncn, rf, ra, rb);
    if (tid == 0) {
      if (MODE == 3) {
        parts[blockIdx.x].ratio_clamps = ncr;
      } else {
        parts[blockIdx.x].flux = acc;
        parts[blockIdx.x].neg_clamps = ncn;
      }
    }
  }
}

// z pass of the differentiated form: forward z transform; optionally store
// the spectrum (s_out) and accumulate the PSF cross-spectrum in FP64
// (acc += X conj(S) for acc_mode 0, conj(X) S for acc_mode 1); multiply by
// the kernel spectrum (conjugated if conjH); inverse z transform.
template <int T, int TX, int MAXL>
__global__ void __launch_bounds__(T)
    k_zext(const JobDesc* __restrict__ jobs, int njobs, const FftPlan* __restrict__ plans,
           const float2* __restrict__ twp, int v, int role, int conjH, float2* __restrict__ s_out,
           const float2* __restrict__ s_in, double2* __restrict__ acc, int acc_mode) {
  __shared__ float2 lds[MAXL * TX];
  __shared__ float2 s_tw[MAXL];
  int local;
  const int jid = find_job(jobs, njobs, PASS_Z, TX, local);
  if (jid < 0) return;
  const JobDesc& J = jobs[jid];
  const int M = J.M, ny = J.ny, nz = J.nz;
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
  const KLine kl{reinterpret_cast<const float2*>(J.H[role]) + (int64_t)v * J.h_elems + hoff, ps, nl, nz,
                 J.kz, J.cz};
  GTile g{reinterpret_cast<float2*>(J.spec) + off, 1, ps, nl};
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
  fft_lines<false, MAXL, T, TX, true, SYNC_BLOCK>(pl, s_tw, tid, g, S, S);
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = tid + i * T;
    const int line = e % TX, pos = e / TX;
    if (pos < nz) {
      const float2 a = S.ld(line, pos);
      if (line < nl) {
        const int64_t idx = off + line + (int64_t)pos * ps;
        if (s_out) gp(s_out)[idx] = a;
        if (acc) {
          const float2 s = gp(s_in)[idx];
          double2 t = gp(acc)[idx];
          if (acc_mode == 0) {  // a conj(s)
            t.x += (double)a.x * s.x + (double)a.y * s.y;
            t.y += (double)a.y * s.x - (double)a.x * s.y;
          } else {  // conj(a) s
            t.x += (double)a.x * s.x + (double)a.y * s.y;
            t.y += (double)a.x * s.y - (double)a.y * s.x;
          }
          gp(acc)[idx] = t;
        }
      }
      S.st(line, pos, cmul(a, conjH ? cconj(h[i]) : h[i]));
    }
  }
  __syncthreads();
  fft_lines<true, MAXL, T, TX, true, SYNC_BLOCK>(pl, s_tw, tid, S, S, g);
}

// z stage of the windowed inverse DFT of a PSF cross-spectrum (FP64):
// T1[dz][ky][kx] = sum_kz A[kz][ky][kx] exp(+2 pi i kz (dz - cz) / nz) for kx
// in [0, M] (the main part and the Nyquist plane), dz in the window.
__global__ void __launch_bounds__(256)
    k_idft_z(const double2* __restrict__ A, int M, int Mp, int ny, int nz, int wz,
             const double2* __restrict__ twz, double2* __restrict__ T1) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t total = (int64_t)(M + 1) * ny * wz;
  if (idx >= total) return;
  const int kx = (int)(idx % (M + 1));
  const int64_t rest = idx / (M + 1);
  const int ky = (int)(rest % ny);
  const int dz = (int)(rest / ny);
  const int d = dz - (wz - 1) / 2;
  const int64_t main_elems = (int64_t)Mp * ny * nz;
  double sr = 0.0, si = 0.0;
  for (int k = 0; k < nz; ++k) {
    const double2 a = kx < M ? A[((int64_t)k * ny + ky) * Mp + kx] : A[main_elems + (int64_t)k * ny + ky];
    int64_t m = ((int64_t)k * d) % nz;
    if (m < 0) m += nz;
    const double2 w = twz[m];  // exp(-2 pi i m / nz); conjugated below
    sr += a.x * w.x + a.y * w.y;
    si += a.y * w.x - a.x * w.y;
  }
  T1[idx] = make_double2(sr, si);
}

// y stage: T2[dz][dy][kx] = sum_ky T1[dz][ky][kx] exp(+2 pi i ky (dy - cy) / ny).
__global__ void __launch_bounds__(256)
    k_idft_y(const double2* __restrict__ T1, int M, int ny, int wy, int wz, const double2* __restrict__ twy,
             double2* __restrict__ T2) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t total = (int64_t)(M + 1) * wy * wz;
  if (idx >= total) return;
  const int kx = (int)(idx % (M + 1));
  const int64_t rest = idx / (M + 1);
  const int dy = (int)(rest % wy);
  const int dz = (int)(rest / wy);
  const int d = dy - (wy - 1) / 2;
  double sr = 0.0, si = 0.0;
  for (int k = 0; k < ny; ++k) {
    const double2 a = T1[((int64_t)dz * ny + k) * (M + 1) + kx];
    int64_t m = ((int64_t)k * d) % ny;
    if (m < 0) m += ny;
    const double2 w = twy[m];  // exp(-2 pi i m / ny); conjugated below
    sr += a.x * w.x + a.y * w.y;
    si += a.y * w.x - a.x * w.y;
  }
  T2[idx] = make_double2(sr, si);
}

// x stage of a real result: out[dz][dy][dx] = sum over the half spectrum kx
// in [0, M], each kx in (0, M) standing for its Hermitian mirror too, of
// Re(T2[dz][dy][kx] exp(+2 pi i kx (dx - cx) / nx)).
__global__ void __launch_bounds__(256)
    k_idft_x(const double2* __restrict__ T2, int M, int nx, int wx, int wy, int wz, const double2* __restrict__ twx,
             double* __restrict__ out) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t total = (int64_t)wx * wy * wz;
  if (idx >= total) return;
  const int dx = (int)(idx % wx);
  const int64_t zy = idx / wx;  // dz * wy + dy
  const int d = dx - (wx - 1) / 2;
  const double2* t = T2 + zy * (M + 1);
  double s = 0.0;
  for (int k = 0; k <= M; ++k) {
    const double2 a = t[k];
    int64_t m = ((int64_t)k * d) % nx;
    if (m < 0) m += nx;
    const double2 w = twx[m];
    const double re = a.x * w.x + a.y * w.y;  // Re(a conj(w))
    s += (k == 0 || k == M) ? re : 2.0 * re;
  }
  out[idx] = s;
}

hipError_t mvd_launch_idft_yx(const double2* T1, int M, int nx, int ny, int wx, int wy, int wz, const double2* twx,
                              const double2* twy, double2* T2, double* out, hipStream_t s) {
  const int64_t n2 = (int64_t)(M + 1) * wy * wz, n3 = (int64_t)wx * wy * wz;
  k_idft_y<<<(unsigned)((n2 + 255) / 256), 256, 0, s>>>(T1, M, ny, wy, wz, twy, T2);
  k_idft_x<<<(unsigned)((n3 + 255) / 256), 256, 0, s>>>(T2, M, nx, wx, wy, wz, twx, out);
  return hipGetLastError();
}

hipError_t mvd_launch_idft_z(const double2* A, int M, int Mp, int ny, int nz, int wz, const double2* twz,
                             double2* T1, hipStream_t s) {
  const int64_t total = (int64_t)(M + 1) * ny * wz;
  k_idft_z<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(A, M, Mp, ny, nz, wz, twz, T1);
  return hipGetLastError();
}

// Launch wrappers over the runtime-plan launch shapes (same candidates as
// the forward passes).
#define MVD_ADJ_ROW_CFGS(X) \
  X(0, 4, 4, 32)            \
  X(1, 4, 2, 64)            \
  X(2, 4, 2, 128)           \
  X(3, 4, 1, 256)           \
  X(4, 4, 1, 512)

#define MVD_ADJ_COL_CFGS(X) \
  X(0, 64, 16, 64)          \
  X(1, 128, 16, 128)        \
  X(2, 256, 16, 256)        \
  X(3, 256, 16, 512)

hipError_t mvd_launch_xadj(const LaunchArgs& a, int cfg, int mode, int v, Partial* parts, int* flags,
                           const AdjPtrs& ap) {
#define MODES(wpb, rpw, m)                                                                              \
  switch (mode) {                                                                                       \
    case 3: k_xadj<3, wpb, rpw, m><<<a.grid, 64 * wpb, 0, a.stream>>>(a.jobs, a.njobs, a.plans, a.tw, v, parts, flags, ap); break; \
    case 4: k_xadj<4, wpb, rpw, m><<<a.grid, 64 * wpb, 0, a.stream>>>(a.jobs, a.njobs, a.plans, a.tw, v, parts, flags, ap); break; \
    case 5: k_xadj<5, wpb, rpw, m><<<a.grid, 64 * wpb, 0, a.stream>>>(a.jobs, a.njobs, a.plans, a.tw, v, parts, flags, ap); break; \
    case 6: k_xadj<6, wpb, rpw, m><<<a.grid, 64 * wpb, 0, a.stream>>>(a.jobs, a.njobs, a.plans, a.tw, v, parts, flags, ap); break; \
    case 7: k_xadj<7, wpb, rpw, m><<<a.grid, 64 * wpb, 0, a.stream>>>(a.jobs, a.njobs, a.plans, a.tw, v, parts, flags, ap); break; \
    case 8: k_xadj<8, wpb, rpw, m><<<a.grid, 64 * wpb, 0, a.stream>>>(a.jobs, a.njobs, a.plans, a.tw, v, parts, flags, ap); break; \
    default: return hipErrorInvalidValue;                                                               \
  }
  switch (cfg) {
#define X(i, wpb, rpw, m) \
  case i:                 \
    MODES(wpb, rpw, m)    \
    break;
    MVD_ADJ_ROW_CFGS(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
#undef MODES
  return hipGetLastError();
}

// The adjoint x passes with the compile-time row plan of a power-of-two
// half-row length (the shape of the per-length row table).
template <int M, int WPB, int RPW, int... Rs>
static hipError_t xadj_ct(const LaunchArgs& a, int mode, int v, Partial* parts, int* flags, const AdjPtrs& ap) {
  if constexpr ((M & (M - 1)) == 0 && M >= 16) {
    switch (mode) {
#define XM(md)                                                                                           \
  case md:                                                                                               \
    k_xadj<md, WPB, RPW, M, Rs...><<<a.grid, 64 * WPB, 0, a.stream>>>(a.jobs, a.njobs, a.plans, a.tw, v, \
                                                                      parts, flags, ap);                 \
    break;
      XM(3) XM(4) XM(5) XM(6) XM(7) XM(8)
#undef XM
      default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

int mvd_xadj_rows(int M) {
  switch (M) {
#define X(m, wpb, rpw, ...) \
  case m:                   \
    return ((m & (m - 1)) == 0 && m >= 16) ? wpb * rpw : 0;
    MVD_EXACT_ROW(X)
#undef X
    default:
      return 0;
  }
}

hipError_t mvd_launch_xadj_exact(const LaunchArgs& a, int M, int mode, int v, Partial* parts, int* flags,
                                 const AdjPtrs& ap) {
  switch (M) {
#define X(m, wpb, rpw, ...) \
  case m:                   \
    return xadj_ct<m, wpb, rpw, __VA_ARGS__>(a, mode, v, parts, flags, ap);
    MVD_EXACT_ROW(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t mvd_launch_zext(const LaunchArgs& a, int cfg, int v, int role, int conjH, float2* s_out,
                           const float2* s_in, double2* acc, int acc_mode) {
  switch (cfg) {
#define X(i, t, tx, l)                                                                             \
  case i:                                                                                          \
    k_zext<t, tx, l><<<a.grid, t, 0, a.stream>>>(a.jobs, a.njobs, a.plans, a.tw, v, role, conjH,   \
                                                  s_out, s_in, acc, acc_mode);                     \
    break;
    MVD_ADJ_COL_CFGS(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
