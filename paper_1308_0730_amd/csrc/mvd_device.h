// Device helpers shared by the pass kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "mvd_gmem.h"
#include "mvd_types.h"

namespace mvdk {

// Map this workgroup to (job, tile within the job) by walking the jobs'
// tile counts for the pass kind.  With reverse the last workgroup takes the
// first tile.  The forward x passes run reversed: the y pass before them
// writes the spectrum in ascending z and the y pass after them reads it in
// ascending z, so each reader starts on the planes written last, which are
// still held by the memory-side cache (the 256 MB Infinity Cache holds most
// of an embryo-sized spectrum).
__device__ __forceinline__ int find_job(const JobDesc* __restrict__ jobs, int njobs, int kind,
                                        int param, int& local, bool reverse = false) {
  int t = reverse ? (int)gridDim.x - 1 - (int)blockIdx.x : (int)blockIdx.x;
  for (int j = 0; j < njobs; ++j) {
    const int c = mvd_tiles(jobs[j], kind, param);
    if (t < c) {
      local = t;
      return j;
    }
    t -= c;
  }
  local = 0;
  return -1;
}

// Column tile `local` (< nxt * nl) of the z passes and the inverse y passes
// -> (kx tile xt, line l): two halves of the kx tiles, the lower first, each
// walked l-major with xt fastest.  The z pass writes the upper half last and
// the inverse y pass after it walks its tiles backwards (see ytile_local),
// so it starts on the half still held by the memory-side cache.  Halves
// keep 1 KB runs along x between workgroups in flight; narrower slabs made
// the z pass slower.
__device__ __forceinline__ void half_tile(int local, int nxt, int nl, int& xt, int& l) {
  const int sw = (nxt + 1) >> 1;
  const int per = sw * nl;
  const int s = local >= per;
  const int r = local - s * per;
  const int w = s ? nxt - sw : sw;
  l = r / w;
  xt = s * sw + r % w;
}

// Tile order of the y passes: the forward ones z-major with xt fastest (the
// x pass before them ends on the planes of low z); the inverse ones
// backwards over the half_tile order, the Nyquist-plane tiles (written last
// by the z pass) first.
template <bool INV>
__device__ __forceinline__ void ytile(int local, int ntiles, int nxt, int nz, int& xt, int& z, int& t2) {
  if (INV) local = ntiles - 1 - local;
  t2 = local - nxt * nz;
  if (t2 >= 0) return;
  if (INV) {
    half_tile(local, nxt, nz, xt, z);
  } else {
    xt = local % nxt;
    z = local / nxt;
  }
}

// Source accessor of the kernel lines of a z tile: tap d of the stored
// kernel planes sits at position (d - cz) mod nz of a length-nz line, every
// other position is zero.  base points at tap 0 of line 0; taps are ps apart.
struct KLine {
  const float2* base;
  int ps, nl, nz, kz, cz;
  static constexpr bool lds = false;
  __device__ __forceinline__ float2 ld(int line, int pos) const {
    int d = pos + cz;
    if (d >= nz) d -= nz;
    return (line < nl && d < kz) ? ldg(base + line + d * ps) : make_float2(0.f, 0.f);
  }
};

// Workgroup sum of an FP64 value and two counters; the result is valid in
// thread 0.
template <int T>
__device__ __forceinline__ void block_reduce(double& f, unsigned& a, unsigned& b, double* sf,
                                             unsigned* sa, unsigned* sb) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    f += __shfl_xor(f, o);
    a += __shfl_xor(a, o);
    b += __shfl_xor(b, o);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sf[w] = f;
    sa[w] = a;
    sb[w] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    f = 0.0;
    a = b = 0;
    for (int i = 0; i < T / 64; ++i) {
      f += sf[i];
      a += sa[i];
      b += sb[i];
    }
  }
}

// a / b for b >= 1 in magnitude or at least a normal float: the hardware
// reciprocal (within 1 ulp) times a, instead of the correctly rounded
// division's longer instruction sequence (the x passes are limited by their
// vector instructions as much as by memory).
__device__ __forceinline__ float fast_div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }

// Tikhonov MAP step: the t >= 0 solving lamp t^2 + t = u, in the form
// without cancellation (hardware square root and reciprocal, each within
// 1 ulp; the denominator is >= 1).
__device__ __forceinline__ float tikhonov(float u, float lamp) {
  return lamp > 0.f ? fast_div(2.f * u, 1.f + __builtin_amdgcn_sqrtf(1.f + 4.f * lamp * u)) : u;
}

// Ratio of observed to expected for the two real values of a packed pair:
// phi / max(b, eps), counting b < eps; 1 where the view has no data
// (MVD_NO_DATA, grid voxels outside the volume with the linear boundary).
__device__ __forceinline__ float2 ratio2(float2 phi, float2 b, float eps, unsigned& nclamp) {
  const bool dx = phi.x >= 0.f, dy = phi.y >= 0.f;
  nclamp += (dx && b.x < eps) + (dy && b.y < eps);
  return make_float2(dx ? fast_div(phi.x, fmaxf(b.x, eps)) : 1.f, dy ? fast_div(phi.y, fmaxf(b.y, eps)) : 1.f);
}

}  // namespace mvdk
