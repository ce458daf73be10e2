// LDS-staged Stockham FFT engine for gfx950 (wave64).
//
// A workgroup transforms NL lines of one runtime length L (a mixed-radix plan
// of radices 2, 3, 4, 5, 8) in place.  Each stage reads R inputs per
// butterfly at stride L/R, applies twiddles, runs an R-point DFT and writes
// the outputs at the auto-sorted (Stockham) positions, so results come out
// in natural order with no bit reversal.  The first stage may read straight
// from global memory and the last may write straight back, so a tile crosses
// LDS only between stages.
//
// Line-fast mapping (column passes): consecutive lanes take consecutive lines
// at the same position, i.e. adjacent x columns: global accesses are
// contiguous runs of NL complex values and LDS is laid out [pos][line].
// Position-fast mapping (row passes): consecutive lanes take consecutive
// butterflies of one row, LDS laid out [line][pos].
//
// Synchronisation is either the whole workgroup (tiles shared by all waves)
// or one wavefront (a wave that owns its rows and its LDS region needs no
// workgroup barrier: a wave's LDS operations complete in issue order).
#pragma once
#include <hip/hip_runtime.h>

#include "mvd_gmem.h"
#include "mvd_types.h"

namespace mvdk {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
// Multiply by -i for the forward transform, +i for the inverse.
template <bool INV>
__device__ __forceinline__ float2 mul_mi(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// R-point DFT in registers, sign -1 (forward) or +1 (INV), unnormalised.
template <int R, bool INV>
struct Dft;

template <bool INV>
struct Dft<2, INV> {
  static __device__ __forceinline__ void run(float2* v) {
    const float2 t = v[0];
    v[0] = cadd(t, v[1]);
    v[1] = csub(t, v[1]);
  }
};

template <bool INV>
struct Dft<4, INV> {
  static __device__ __forceinline__ void run(float2* v) {
    const float2 a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
    const float2 c = cadd(v[1], v[3]), d = mul_mi<INV>(csub(v[1], v[3]));
    v[0] = cadd(a, c);
    v[2] = csub(a, c);
    v[1] = cadd(b, d);
    v[3] = csub(b, d);
  }
};

template <bool INV>
struct Dft<8, INV> {
  static __device__ __forceinline__ void run(float2* v) {
    const float r = 0.70710678118654752440f;
    float2 e[4] = {v[0], v[2], v[4], v[6]};
    float2 o[4] = {v[1], v[3], v[5], v[7]};
    Dft<4, INV>::run(e);
    Dft<4, INV>::run(o);
    float2 o1, o3;
    if (INV) {
      o1 = make_float2((o[1].x - o[1].y) * r, (o[1].x + o[1].y) * r);
      o3 = make_float2((-o[3].x - o[3].y) * r, (o[3].x - o[3].y) * r);
    } else {
      o1 = make_float2((o[1].x + o[1].y) * r, (o[1].y - o[1].x) * r);
      o3 = make_float2((o[3].y - o[3].x) * r, (-o[3].x - o[3].y) * r);
    }
    const float2 o2 = mul_mi<INV>(o[2]);
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
  }
};

template <bool INV>
struct Dft<3, INV> {
  static __device__ __forceinline__ void run(float2* v) {
    const float h = 0.86602540378443864676f;  // sin(2 pi / 3)
    const float2 s = cadd(v[1], v[2]);
    const float2 d = csub(v[1], v[2]);
    const float2 m = make_float2(v[0].x - 0.5f * s.x, v[0].y - 0.5f * s.y);
    const float2 t = cscale(mul_mi<INV>(d), h);
    v[0] = cadd(v[0], s);
    v[1] = cadd(m, t);
    v[2] = csub(m, t);
  }
};

template <bool INV>
struct Dft<5, INV> {
  static __device__ __forceinline__ void run(float2* v) {
    const float c1 = 0.30901699437494742410f;   // cos(2 pi / 5)
    const float c2 = -0.80901699437494742410f;  // cos(4 pi / 5)
    const float s1 = 0.95105651629515357212f;   // sin(2 pi / 5)
    const float s2 = 0.58778525229247312917f;   // sin(4 pi / 5)
    const float2 a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
    const float2 a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
    const float2 p1 = make_float2(v[0].x + c1 * a1.x + c2 * a2.x, v[0].y + c1 * a1.y + c2 * a2.y);
    const float2 p2 = make_float2(v[0].x + c2 * a1.x + c1 * a2.x, v[0].y + c2 * a1.y + c1 * a2.y);
    const float2 q1 = mul_mi<INV>(make_float2(s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y));
    const float2 q2 = mul_mi<INV>(make_float2(s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y));
    v[0] = cadd(v[0], cadd(a1, a2));
    v[1] = cadd(p1, q1);
    v[4] = csub(p1, q1);
    v[2] = cadd(p2, q2);
    v[3] = csub(p2, q2);
  }
};

// ---- element accessors ------------------------------------------------------

// LDS tile laid out [pos][line] (column passes).
template <int NL>
struct LdsCol {
  float2* p;
  static constexpr bool lds = true;
  __device__ __forceinline__ float2 ld(int line, int pos) const { return p[pos * NL + line]; }
  __device__ __forceinline__ void st(int line, int pos, float2 v) const { p[pos * NL + line] = v; }
};

// LDS tile laid out [line][pos] with a fixed row pitch (row passes).
template <int PITCH>
struct LdsRow {
  float2* p;
  static constexpr bool lds = true;
  __device__ __forceinline__ float2 ld(int line, int pos) const { return p[line * PITCH + pos]; }
  __device__ __forceinline__ void st(int line, int pos, float2 v) const { p[line * PITCH + pos] = v; }
};

// Global tile: element (line, pos) at base[line * ls + pos * ps] (32-bit
// element offsets from the tile's base); lines >= nl read as zero and are
// not written.
struct GTile {
  float2* base;
  int ls, ps;
  int nl;
  static constexpr bool lds = false;
  __device__ __forceinline__ float2 ld(int line, int pos) const {
    return line < nl ? ldg(base + line * ls + pos * ps) : make_float2(0.f, 0.f);
  }
  __device__ __forceinline__ void st(int line, int pos, float2 v) const {
    if (line < nl) stg(base + line * ls + pos * ps, v);
  }
};

// ---- synchronisation ---------------------------------------------------------

enum { SYNC_BLOCK = 0, SYNC_WAVE = 1 };

template <int SY>
__device__ __forceinline__ void gsync() {
  if (SY == SYNC_BLOCK) {
    __syncthreads();
  } else {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

__device__ __forceinline__ int udiv(int j, unsigned magic) { return (int)__umulhi((unsigned)j, magic); }

// ---- one Stockham stage ------------------------------------------------------

struct StageInfo {
  int L, Ns, tws;
  unsigned ns_magic, nb_magic;
};

// MAXL bounds L; T threads (tid in [0, T)); NL lines; LF selects the
// line-fast mapping; SY the synchronisation scope; tw is the length-L
// twiddle table (in LDS).
template <int R, bool INV, int MAXL, int T, int NL, bool LF, int SY, class S, class D>
__device__ __forceinline__ void stage(const StageInfo& si, int tid_in, const float2* tw, const S& src,
                                      const D& dst) {
  constexpr int MAXB = (NL * (MAXL / R) + T - 1) / T;
  // hide the thread index from loop-invariant code motion: otherwise the
  // per-stage index arithmetic of every radix case is hoisted out of the
  // stage loop and stays live in registers for the whole transform
  int tid = tid_in;
  asm volatile("" : "+v"(tid));
  const int nb = si.L / R;
  const int total = nb * NL;
  const int Ns = si.Ns;
  float2 v[MAXB][R];
  int ln[MAXB], jb[MAXB];
#pragma unroll
  for (int i = 0; i < MAXB; ++i) {
    const int it = tid + i * T;
    int line, j;
    if (LF) {
      line = it % NL;
      j = it / NL;
    } else if (nb == 1) {
      line = it;
      j = 0;
    } else {
      line = udiv(it, si.nb_magic);
      j = it - line * nb;
    }
    ln[i] = line;
    jb[i] = j;
    if (it < total) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = src.ld(line, j + r * nb);
    }
  }
  // in-place stages (LDS -> LDS, or a single global -> global stage) must
  // finish every read before the first write
  if (S::lds == D::lds) gsync<SY>();
#pragma unroll
  for (int i = 0; i < MAXB; ++i) {
    const int it = tid + i * T;
    if (it < total) {
      const int j = jb[i];
      const int k = Ns == 1 ? 0 : j - udiv(j, si.ns_magic) * Ns;
      if (Ns > 1) {
        const int step = k * si.tws;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          float2 w = tw[step * r];
          if (INV) w.y = -w.y;
          v[i][r] = cmul(v[i][r], w);
        }
      }
      Dft<R, INV>::run(v[i]);
      const int base = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) dst.st(ln[i], base + r * Ns, v[i][r]);
    }
  }
  if (D::lds) gsync<SY>();
}

template <bool INV, int MAXL, int T, int NL, bool LF, int SY, class S, class D>
__device__ __forceinline__ void stage_rt(int R, const StageInfo& si, int tid, const float2* tw,
                                         const S& src, const D& dst) {
  switch (R) {
    case 8: stage<8, INV, MAXL, T, NL, LF, SY>(si, tid, tw, src, dst); break;
    case 4: stage<4, INV, MAXL, T, NL, LF, SY>(si, tid, tw, src, dst); break;
    case 2: stage<2, INV, MAXL, T, NL, LF, SY>(si, tid, tw, src, dst); break;
    case 3: stage<3, INV, MAXL, T, NL, LF, SY>(si, tid, tw, src, dst); break;
    default: stage<5, INV, MAXL, T, NL, LF, SY>(si, tid, tw, src, dst); break;
  }
}

// Whole transform of NL lines: first stage src -> mid, middle stages
// mid -> mid, last stage mid -> dst (a single stage goes src -> dst).
// `mid` must be an LDS accessor; tw the plan's twiddle table in LDS.
template <bool INV, int MAXL, int T, int NL, bool LF, int SY, class S, class M, class D>
__device__ __forceinline__ void fft_lines(const FftPlan* __restrict__ pl, const float2* tw, int tid,
                                          const S& src, const M& mid, const D& dst) {
  const int nst = pl->nst;
  StageInfo si;
  si.L = pl->L;
  for (int s = 0; s < nst; ++s) {
    const int R = pl->radix[s];
    si.Ns = pl->ns[s];
    si.tws = pl->tws[s];
    si.ns_magic = pl->ns_magic[s];
    si.nb_magic = pl->nb_magic[s];
    const bool first = s == 0, last = s == nst - 1;
    if (first && last)
      stage_rt<INV, MAXL, T, NL, LF, SY>(R, si, tid, tw, src, dst);
    else if (first)
      stage_rt<INV, MAXL, T, NL, LF, SY>(R, si, tid, tw, src, mid);
    else if (last)
      stage_rt<INV, MAXL, T, NL, LF, SY>(R, si, tid, tw, mid, dst);
    else
      stage_rt<INV, MAXL, T, NL, LF, SY>(R, si, tid, tw, mid, mid);
  }
}

// Cooperative copy of n table entries into LDS (all T threads), followed by
// a workgroup barrier.
template <int T>
__device__ __forceinline__ void load_table(float2* dst, const float2* __restrict__ src, int n) {
  for (int i = threadIdx.x; i < n; i += T) dst[i] = gp(src)[i];
}

}  // namespace mvdk
