// Weight normalisation for partially overlapping views (the section on
// partially overlapping data): each voxel's summed weight over the views is
// limited to an overlap number m, scaling every view's weight by the same
// factor m / sum where the sum exceeds m (weights are never increased).
// m is 1, the minimal or the average number of contributing views over the
// covered voxels, or a user value; the count image is offered to choose it.
// Setup work on one block's [nviews][V] weights, not part of an iteration.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "mvd_gmem.h"
#include "mvd_kernels.h"

using namespace mvdk;

namespace {

__device__ __forceinline__ int count_at(const float* __restrict__ w, int nviews, int64_t V, int64_t i) {
  int c = 0;
  for (int v = 0; v < nviews; ++v) c += ldg(w + (int64_t)v * V + i) > 0.f;
  return c;
}

// Minimum of the count over covered voxels, the summed count and the number
// of covered voxels; integer atomics, one per workgroup and quantity.
__global__ void __launch_bounds__(256)
    k_overlap_stats(const float* __restrict__ w, int nviews, int64_t V, unsigned* __restrict__ cmin,
                    unsigned long long* __restrict__ csum, unsigned long long* __restrict__ ncov) {
  unsigned mn = 0xffffffffu;
  unsigned long long sm = 0, nc = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < V; i += (int64_t)gridDim.x * 256) {
    const int c = count_at(w, nviews, V, i);
    if (c > 0) {
      mn = min(mn, (unsigned)c);
      sm += (unsigned long long)c;
      nc += 1;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    mn = min(mn, (unsigned)__shfl_xor((int)mn, o));
    sm += __shfl_xor(sm, o);
    nc += __shfl_xor(nc, o);
  }
  __shared__ unsigned smn[4];
  __shared__ unsigned long long ssm[4], snc[4];
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    smn[wv] = mn;
    ssm[wv] = sm;
    snc[wv] = nc;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < 4; ++k) {
      mn = min(mn, smn[k]);
      sm += ssm[k];
      nc += snc[k];
    }
    atomicMin(cmin, mn);
    atomicAdd(csum, sm);
    atomicAdd(ncov, nc);
  }
}

__global__ void __launch_bounds__(256)
    k_overlap_limit(float* __restrict__ w, int nviews, int64_t V, float m) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < V; i += (int64_t)gridDim.x * 256) {
    float s = 0.f;
    for (int v = 0; v < nviews; ++v) s += ldg(w + (int64_t)v * V + i);
    if (s > m) {
      const float f = m / s;
      for (int v = 0; v < nviews; ++v) {
        float* p = w + (int64_t)v * V + i;
        stg(p, ldg(p) * f);
      }
    }
  }
}

__global__ void __launch_bounds__(256)
    k_overlap_count(const float* __restrict__ w, int nviews, int64_t V, float* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < V; i += (int64_t)gridDim.x * 256)
    stg(out + i, (float)count_at(w, nviews, V, i));
}

int grid_for(int64_t V) { return (int)std::min<int64_t>((V + 255) / 256, 8192); }

}  // namespace

hipError_t mvd_launch_overlap_stats(const float* w, int nviews, int64_t V, unsigned* cmin,
                                    unsigned long long* csum, unsigned long long* ncov, hipStream_t s) {
  k_overlap_stats<<<grid_for(V), 256, 0, s>>>(w, nviews, V, cmin, csum, ncov);
  return hipGetLastError();
}

hipError_t mvd_launch_overlap_limit(float* w, int nviews, int64_t V, float m, hipStream_t s) {
  k_overlap_limit<<<grid_for(V), 256, 0, s>>>(w, nviews, V, m);
  return hipGetLastError();
}

hipError_t mvd_launch_overlap_count(const float* w, int nviews, int64_t V, float* out, hipStream_t s) {
  k_overlap_count<<<grid_for(V), 256, 0, s>>>(w, nviews, V, out);
  return hipGetLastError();
}
