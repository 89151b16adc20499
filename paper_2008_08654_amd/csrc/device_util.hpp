// device_util.hpp -- small device helpers shared by the kernel translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mcs {

// A record every lane of the wave reads (a work-list entry), kept in scalar
// registers.  The record must not change during the launch: it is read
// through the constant address space, which gives scalar loads.
template <typename T>
__device__ __forceinline__ T uniform_load(const T* p) {
  static_assert(sizeof(T) % 4 == 0, "records are whole 32-bit words");
  T v;
  uint32_t* w = reinterpret_cast<uint32_t*>(&v);
  const auto* q = (const __attribute__((address_space(4))) uint32_t*)p;
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); ++i) w[i] = __builtin_amdgcn_readfirstlane(q[i]);
  return v;
}

}  // namespace mcs
