// Device helpers shared by the pass kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "pafc_internal.h"
#include "small_dft.h"

namespace pafc {

__device__ __forceinline__ uint32_t fdiv(uint32_t x, const FastDiv& f) {
  uint64_t t = ((uint64_t)x * f.m) >> 32;
  return (uint32_t)((t + x) >> f.l);
}

__device__ __forceinline__ uint32_t lds_phys(uint32_t x) { return x + (x >> 4); }

template <typename T>
__device__ __forceinline__ cx<T> ld_g(const void* p, int64_t idx) {
  return reinterpret_cast<const cx<T>*>(p)[idx];
}
template <typename T>
__device__ __forceinline__ void st_g(void* p, int64_t idx, cx<T> v) {
  reinterpret_cast<cx<T>*>(p)[idx] = v;
}

template <typename T>
__device__ __forceinline__ cx<T> twiddle(const PassArgs& a, uint32_t E) {
  const cx<T>* lo = reinterpret_cast<const cx<T>*>(a.tw_lo);
  if (a.tw_hi == nullptr) return lo[E];
  const cx<T>* hi = reinterpret_cast<const cx<T>*>(a.tw_hi);
  return cmul(lo[E & ((1u << a.tw_bits) - 1u)], hi[E >> a.tw_bits]);
}

}  // namespace pafc
