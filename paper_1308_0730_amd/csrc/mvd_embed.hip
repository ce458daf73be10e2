// Volumes inside computation grids.  Linear boundary: the user's volume sits
// at an offset inside a larger grid (the volume extended by the PSF radius
// and rounded up to transform lengths); setup and copy work.  Block-wise
// form: each block's grid is a window of the periodic volume (the block and
// a halo around it); its views and weights are gathered once.  Shapes are
// (nx, ny, nz) grids stored [z][y][x].
#include <hip/hip_runtime.h>

#include <algorithm>

#include "mvd_device.h"
#include "mvd_gmem.h"
#include "mvd_kernels.h"

using namespace mvdk;

namespace {

struct Box {
  int nx, ny, nz;   // grid
  int ux, uy, uz;   // user volume
  int ox, oy, oz;   // its offset in the grid
};

__device__ __forceinline__ int64_t grid_index(const Box& b, int64_t i) {
  const int x = (int)(i % b.ux);
  const int64_t r = i / b.ux;
  const int y = (int)(r % b.uy);
  const int z = (int)(r / b.uy);
  return ((int64_t)(z + b.oz) * b.ny + (y + b.oy)) * b.nx + (x + b.ox);
}

__global__ void __launch_bounds__(256) k_embed(float* __restrict__ grid, const float* __restrict__ vol, Box b) {
  const int64_t n = (int64_t)b.ux * b.uy * b.uz;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    stg(grid + grid_index(b, i), ldg(vol + i));
}

__global__ void __launch_bounds__(256) k_extract(float* __restrict__ vol, const float* __restrict__ grid, Box b) {
  const int64_t n = (int64_t)b.ux * b.uy * b.uz;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    stg(vol + i, ldg(grid + grid_index(b, i)));
}

// every grid voxel outside the box gets val
__global__ void __launch_bounds__(256) k_fill_outside(float* __restrict__ grid, Box b, float val) {
  const int64_t n = (int64_t)b.nx * b.ny * b.nz;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const int x = (int)(i % b.nx);
    const int64_t r = i / b.nx;
    const int y = (int)(r % b.ny);
    const int z = (int)(r / b.ny);
    const bool in = x >= b.ox && x < b.ox + b.ux && y >= b.oy && y < b.oy + b.uy && z >= b.oz && z < b.oz + b.uz;
    if (!in) stg(grid + i, val);
  }
}

// grid[z][y][x] = vol[(z0 + z) mod nz][(y0 + y) mod ny][(x0 + x) mod nx],
// 0 <= x0 < nx etc.; a workgroup per grid row at a time
__global__ void __launch_bounds__(256) k_gather(float* __restrict__ grid, int gx, int gy, int gz,
                                                const float* __restrict__ vol, int nx, int ny, int nz, int x0,
                                                int y0, int z0) {
  const int64_t rows = (int64_t)gy * gz;
  for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
    const int y = (int)(r % gy), z = (int)(r / gy);
    const float* src = vol + ((int64_t)((z0 + z) % nz) * ny + (y0 + y) % ny) * nx;
    float* dst = grid + r * gx;
    for (int x = threadIdx.x; x < gx; x += 256) stg(dst + x, ldg(src + (x0 + x) % nx));
  }
}

int blocks_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 8192)); }

Box box(const int* grid, const int* user, const int* off) {
  return Box{grid[0], grid[1], grid[2], user[0], user[1], user[2], off[0], off[1], off[2]};
}

}  // namespace

hipError_t mvd_launch_embed(float* grid, const int* gdims, const float* vol, const int* udims, const int* off,
                            hipStream_t s) {
  const Box b = box(gdims, udims, off);
  k_embed<<<blocks_for((int64_t)b.ux * b.uy * b.uz), 256, 0, s>>>(grid, vol, b);
  return hipGetLastError();
}

hipError_t mvd_launch_extract(float* vol, const int* udims, const float* grid, const int* gdims, const int* off,
                              hipStream_t s) {
  const Box b = box(gdims, udims, off);
  k_extract<<<blocks_for((int64_t)b.ux * b.uy * b.uz), 256, 0, s>>>(vol, grid, b);
  return hipGetLastError();
}

hipError_t mvd_launch_fill_outside(float* grid, const int* gdims, const int* udims, const int* off, float val,
                                   hipStream_t s) {
  const Box b = box(gdims, udims, off);
  k_fill_outside<<<blocks_for((int64_t)b.nx * b.ny * b.nz), 256, 0, s>>>(grid, b, val);
  return hipGetLastError();
}

hipError_t mvd_launch_gather(float* grid, const int* gdims, const float* vol, const int* vdims, const int* start,
                             hipStream_t s) {
  const int64_t rows = (int64_t)gdims[1] * gdims[2];
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(rows, 4096));
  k_gather<<<nb, 256, 0, s>>>(grid, gdims[0], gdims[1], gdims[2], vol, vdims[0], vdims[1], vdims[2], start[0],
                              start[1], start[2]);
  return hipGetLastError();
}
