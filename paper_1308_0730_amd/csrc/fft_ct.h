// Compile-time specialised Stockham transforms for the hot power-of-two
// lengths.  Same stage algebra as the runtime engine, but the length, the
// radix sequence and the tile shape are template parameters, so every
// index, stride and twiddle offset folds to a constant, the stage loop
// unrolls, and radix 16 halves the number of LDS round trips.
//
// Accessors used as the last stage's destination receive the butterfly slot
// i and the output index r as well, so a fused epilogue (spectral product,
// ratio, update) can use operands prefetched into registers in that order.
#pragma once
#include "fft_engine.h"
#include "fft_small_tw.h"

namespace mvdk {

// Multiply by W16^M = exp(-+2 pi i M / 16) with the cheap forms spelled out.
template <bool INV, int M>
__device__ __forceinline__ float2 w16mul(float2 a) {
  constexpr int m = M & 15;
  constexpr float r = 0.70710678118654752440f;
  constexpr float c1 = 0.92387953251128675613f;  // cos(pi / 8)
  constexpr float s1 = 0.38268343236508977173f;  // sin(pi / 8)
  if constexpr (m == 0) {
    return a;
  } else if constexpr (m == 4) {
    return mul_mi<INV>(a);
  } else if constexpr (m == 8) {
    return make_float2(-a.x, -a.y);
  } else if constexpr (m == 2 || m == 6 || m == 10 || m == 14) {
    // (+-1 +- i) / sqrt 2
    constexpr float cr = (m == 2 || m == 14) ? r : -r;
    constexpr float si = (m == 2 || m == 6) ? -r : r;  // forward sign
    constexpr float sv = INV ? -si : si;
    return make_float2(cr * a.x - sv * a.y, cr * a.y + sv * a.x);
  } else {
    constexpr float cs[16] = {1.f, c1, r, s1, 0.f, -s1, -r, -c1, -1.f, -c1, -r, -s1, 0.f, s1, r, c1};
    constexpr float sn[16] = {0.f, s1, r, c1, 1.f, c1, r, s1, 0.f, -s1, -r, -c1, -1.f, -c1, -r, -s1};
    constexpr float c = cs[m];
    constexpr float s = INV ? sn[m] : -sn[m];
    return make_float2(c * a.x - s * a.y, c * a.y + s * a.x);
  }
}

template <bool INV, int N2, int K1>
__device__ __forceinline__ void tw16_apply(float2 (&a)[4][4]) {
  a[N2][K1] = w16mul<INV, N2 * K1>(a[N2][K1]);
}

// 16-point DFT as 4 x 4: X[k1 + 4 k2] = sum_n2 W16^{n2 k1} W4^{n2 k2}
// sum_n1 x[4 n1 + n2] W4^{n1 k1}.
template <bool INV>
struct Dft<16, INV> {
  static __device__ __forceinline__ void run(float2* v) {
    float2 a[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
      float2 t[4] = {v[n2], v[4 + n2], v[8 + n2], v[12 + n2]};
      Dft<4, INV>::run(t);
#pragma unroll
      for (int k1 = 0; k1 < 4; ++k1) a[n2][k1] = t[k1];
    }
    tw16_apply<INV, 1, 1>(a);
    tw16_apply<INV, 1, 2>(a);
    tw16_apply<INV, 1, 3>(a);
    tw16_apply<INV, 2, 1>(a);
    tw16_apply<INV, 2, 2>(a);
    tw16_apply<INV, 2, 3>(a);
    tw16_apply<INV, 3, 1>(a);
    tw16_apply<INV, 3, 2>(a);
    tw16_apply<INV, 3, 3>(a);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      float2 t[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
      Dft<4, INV>::run(t);
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = t[k2];
    }
  }
};

// R-point DFT of a composite radix R = R1 R2 in registers (Cooley-Tukey,
// decimation in time): X[k1 + R1 k2] = sum_n2 W_R^{n2 k1} W_R2^{n2 k2}
// sum_n1 x[R2 n1 + n2] W_R1^{n1 k1}.  The twiddles W_R^m are constants
// (m = n2 k1 mod R after unrolling); quarter turns are exact swaps.
template <int R1, int R2, bool INV>
struct DftPQ {
  static constexpr int R = R1 * R2;
  static __device__ __forceinline__ void run(float2* v) {
    float2 a[R2][R1];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) {
      float2 t[R1];
#pragma unroll
      for (int n1 = 0; n1 < R1; ++n1) t[n1] = v[R2 * n1 + n2];
      Dft<R1, INV>::run(t);
#pragma unroll
      for (int k1 = 0; k1 < R1; ++k1) {
        const int m = (n2 * k1) % R;
        float2 x = t[k1];
        if (m == 0) {
        } else if (4 * m == R) {
          x = mul_mi<INV>(x);
        } else if (2 * m == R) {
          x = make_float2(-x.x, -x.y);
        } else if (4 * m == 3 * R) {
          x = mul_mi<!INV>(x);
        } else {
          const float c = SmallTw<R>::c[m];
          const float s = INV ? SmallTw<R>::s[m] : -SmallTw<R>::s[m];
          x = make_float2(c * x.x - s * x.y, c * x.y + s * x.x);
        }
        a[n2][k1] = x;
      }
    }
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
      float2 t[R2];
#pragma unroll
      for (int n2 = 0; n2 < R2; ++n2) t[n2] = a[n2][k1];
      Dft<R2, INV>::run(t);
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) v[k1 + R1 * k2] = t[k2];
    }
  }
};

template <bool INV>
struct Dft<6, INV> : DftPQ<2, 3, INV> {};
template <bool INV>
struct Dft<9, INV> : DftPQ<3, 3, INV> {};
template <bool INV>
struct Dft<10, INV> : DftPQ<2, 5, INV> {};
template <bool INV>
struct Dft<12, INV> : DftPQ<4, 3, INV> {};
template <bool INV>
struct Dft<15, INV> : DftPQ<3, 5, INV> {};
template <bool INV>
struct Dft<20, INV> : DftPQ<4, 5, INV> {};
template <bool INV>
struct Dft<25, INV> : DftPQ<5, 5, INV> {};

// Accessor adaptors: the five-argument store used by the compile-time stages.
template <class A>
struct Plain {
  const A& a;
  static constexpr bool lds = A::lds;
  __device__ __forceinline__ float2 ld(int line, int pos) const { return a.ld(line, pos); }
  __device__ __forceinline__ void st(int line, int pos, float2 v, int, int) const { a.st(line, pos, v); }
};

// First-stage inputs already loaded into registers (by ct_prefetch), in the
// order the first stage reads them: a source that issues no loads.
template <int MAXB, int R>
struct RegSrc {
  const float2 (&v)[MAXB][R];
  static constexpr bool lds = false;
};
template <class S>
struct IsRegSrc {
  static constexpr bool value = false;
};
template <int MAXB, int R>
struct IsRegSrc<RegSrc<MAXB, R>> {
  static constexpr bool value = true;
};

// Butterfly slots of the first stage of a plan with first radix R.
template <int L, int R, int T, int NL>
struct FirstMap {
  static constexpr int MAXB = ((L / R) * NL + T - 1) / T;
};

// Issue the loads of the first stage of a plan (first radix R) into v.
template <int L, int R, int T, int NL, bool LF, class S>
__device__ __forceinline__ void ct_prefetch(int tid, const S& src, float2 (&v)[FirstMap<L, R, T, NL>::MAXB][R]) {
  constexpr int NB = L / R;
  constexpr int TOTAL = NB * NL;
  constexpr int MAXB = FirstMap<L, R, T, NL>::MAXB;
#pragma unroll
  for (int i = 0; i < MAXB; ++i) {
    const int it = tid + i * T;
    const int line = LF ? it % NL : it / NB;
    const int j = LF ? it / NL : it % NB;
    if ((TOTAL % T == 0) || it < TOTAL) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = src.ld(line, j + r * NB);
    }
  }
}

// One stage of a compile-time plan: radix R, length L, NS = product of the
// earlier radices, T threads, NL lines, line-fast (LF) or position-fast.
template <int R, bool INV, int L, int NS, int T, int NL, bool LF, int SY, class S, class D>
__device__ __forceinline__ void ct_stage(int tid_in, const float2* tw, const S& src, D& dst) {
  constexpr int NB = L / R;
  constexpr int TOTAL = NB * NL;
  constexpr int MAXB = (TOTAL + T - 1) / T;
  constexpr int TWS = L / (NS * R);
  constexpr bool FULL = TOTAL % T == 0;
  int tid = tid_in;
  asm volatile("" : "+v"(tid));
  float2 v[MAXB][R];
  int ln[MAXB], jb[MAXB];
#pragma unroll
  for (int i = 0; i < MAXB; ++i) {
    const int it = tid + i * T;
    const int line = LF ? it % NL : it / NB;
    const int j = LF ? it / NL : it % NB;
    ln[i] = line;
    jb[i] = j;
    if (FULL || it < TOTAL) {
      if constexpr (IsRegSrc<S>::value) {
#pragma unroll
        for (int r = 0; r < R; ++r) v[i][r] = src.v[i][r];
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) v[i][r] = src.ld(line, j + r * NB);
      }
    }
  }
  if (S::lds == D::lds) gsync<SY>();
#pragma unroll
  for (int i = 0; i < MAXB; ++i) {
    const int it = tid + i * T;
    if (FULL || it < TOTAL) {
      const int j = jb[i];
      const int k = j % NS;
      if (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          float2 w = tw[k * r * TWS];
          if (INV) w.y = -w.y;
          v[i][r] = cmul(v[i][r], w);
        }
      }
      Dft<R, INV>::run(v[i]);
      const int base = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) dst.st(ln[i], base + r * NS, v[i][r], i, r);
    }
  }
  if (D::lds) gsync<SY>();
}

// The radix sequence Rs... applied in order: first stage src -> mid (or dst
// when it is the only one), then mid -> mid, last stage mid -> dst.
template <bool INV, int L, int T, int NL, bool LF, int SY, int NS, bool FIRST, int R, int... Rest>
struct CtRun {
  template <class S, class M, class D>
  static __device__ __forceinline__ void run(int tid, const float2* tw, const S& src, const M& mid, D& dst) {
    if constexpr (sizeof...(Rest) == 0) {
      if constexpr (FIRST) {
        ct_stage<R, INV, L, NS, T, NL, LF, SY>(tid, tw, src, dst);
      } else {
        ct_stage<R, INV, L, NS, T, NL, LF, SY>(tid, tw, mid, dst);
      }
    } else {
      Plain<M> m{mid};
      if constexpr (FIRST) {
        ct_stage<R, INV, L, NS, T, NL, LF, SY>(tid, tw, src, m);
      } else {
        ct_stage<R, INV, L, NS, T, NL, LF, SY>(tid, tw, mid, m);
      }
      CtRun<INV, L, T, NL, LF, SY, NS * R, false, Rest...>::run(tid, tw, src, mid, dst);
    }
  }
};

template <int R, int... Rest>
struct FirstRadix {
  static constexpr int value = R;
};

template <int R, int... Rest>
struct LastRadix {
  static constexpr int value = LastRadix<Rest...>::value;
};
template <int R>
struct LastRadix<R> {
  static constexpr int value = R;
};

// Output positions of the last stage: butterfly slot i of this thread writes
// output r to position j + r * (L / RL) of line `line` (the last stage's
// butterflies have j < L / RL = NS, so k = j).
template <int L, int RL, int T, int NL, bool LF>
struct LastMap {
  static constexpr int NB = L / RL;
  static constexpr int TOTAL = NB * NL;
  static constexpr int MAXB = (TOTAL + T - 1) / T;
  static __device__ __forceinline__ bool at(int tid, int i, int& line, int& j) {
    const int it = tid + i * T;
    line = LF ? it % NL : it / NB;
    j = LF ? it / NL : it % NB;
    return (TOTAL % T == 0) || it < TOTAL;
  }
};

}  // namespace mvdk
