// Global-memory views of generic pointers.
//
// Pointers read from the job table are generic, so plain accesses through
// them compile to flat instructions, and the hardware counts a flat access
// against the LDS wait counter as well as the vector-memory one: every wait
// for an LDS result then also waits for all outstanding HBM loads, which
// serialises the transform stages behind the memory traffic.  Accesses
// through these views compile to global instructions, counted apart.
#pragma once
#include <hip/hip_runtime.h>

namespace mvdk {

// The host pass only type-checks device code; it sees plain pointers.
#if defined(__HIP_DEVICE_COMPILE__)
template <class T>
using gmem = __attribute__((address_space(1))) T;
#else
template <class T>
using gmem = T;
#endif

template <class T>
__device__ __forceinline__ gmem<T>* gp(T* p) {
  return (gmem<T>*)p;
}
template <class T>
__device__ __forceinline__ const gmem<T>* gp(const T* p) {
  return (const gmem<T>*)p;
}

// one element at p in global memory
template <class T>
__device__ __forceinline__ T ldg(const T* p) {
  T v = *gp(p);
  return v;
}
template <class T>
__device__ __forceinline__ void stg(T* p, T v) {
  *gp(p) = v;
}

// float2 at p (8-byte aligned) in global memory
__device__ __forceinline__ float2 ld2(const float* p) { return *reinterpret_cast<const gmem<float2>*>(gp(p)); }
__device__ __forceinline__ void st2(float* p, float2 v) { *reinterpret_cast<gmem<float2>*>(gp(p)) = v; }

}  // namespace mvdk
