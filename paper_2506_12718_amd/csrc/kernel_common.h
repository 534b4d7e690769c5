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
// The same with the padding interval of a pass (PassArgs::lds_sh: one pad
// element every 2^sh, or none for sh = 31).
__device__ __forceinline__ uint32_t lds_phys(uint32_t x, uint32_t sh) { return x + (x >> sh); }

template <typename T>
__device__ __forceinline__ cx<T> ld_g(const void* p, int64_t idx) {
  return reinterpret_cast<const cx<T>*>(p)[idx];
}
template <typename T>
__device__ __forceinline__ void st_g(void* p, int64_t idx, cx<T> v) {
  reinterpret_cast<cx<T>*>(p)[idx] = v;
}

// Element `idx` of an array smaller than 4 GiB: a 32-bit byte offset from the
// uniform base pointer lets the compiler address it with one VGPR (global
// access with a scalar base) instead of a 64-bit address pair per access.
template <typename T>
__device__ __forceinline__ cx<T> ld_g32(const void* p, uint32_t idx) {
  return *reinterpret_cast<const cx<T>*>(reinterpret_cast<const char*>(p) +
                                         idx * (uint32_t)sizeof(cx<T>));
}
// A load marked non-temporal: a streamed read of data the launch uses once,
// which should not displace other lines from the caches (the global_load
// carries the nt bit).
template <typename T>
__device__ __forceinline__ cx<T> ld_nt(const cx<T>* p) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  const v2 v = __builtin_nontemporal_load(reinterpret_cast<const v2*>(p));
  return cx<T>{v.x, v.y};
}
// ld_g32, non-temporal when NT
template <typename T, bool NT>
__device__ __forceinline__ cx<T> ld_g32s(const void* p, uint32_t idx) {
  if constexpr (NT)
    return ld_nt<T>(reinterpret_cast<const cx<T>*>(reinterpret_cast<const char*>(p) +
                                                    idx * (uint32_t)sizeof(cx<T>)));
  else
    return ld_g32<T>(p, idx);
}
template <typename T>
__device__ __forceinline__ void st_g32(void* p, uint32_t idx, cx<T> v) {
  *reinterpret_cast<cx<T>*>(reinterpret_cast<char*>(p) + idx * (uint32_t)sizeof(cx<T>)) = v;
}

template <typename T>
__device__ __forceinline__ cx<T> twiddle(const PassArgs& a, uint32_t E) {
  const cx<T>* lo = reinterpret_cast<const cx<T>*>(a.tw_lo);
  if (a.tw_hi == nullptr) return lo[E];
  const cx<T>* hi = reinterpret_cast<const cx<T>*>(a.tw_hi);
  return cmul(lo[E & ((1u << a.tw_bits) - 1u)], hi[E >> a.tw_bits]);
}

}  // namespace pafc
