// device_util.hpp -- small device helpers shared by the kernel translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mcs {

// A record every lane of the wave reads (a work-list entry), kept in scalar
// registers.
template <typename T>
__device__ __forceinline__ T uniform_load(const T* p) {
  // all lanes read the same record; copy it through readfirstlane
  T v = *p;
  uint32_t* w = reinterpret_cast<uint32_t*>(&v);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); ++i) w[i] = __builtin_amdgcn_readfirstlane(w[i]);
  return v;
}

}  // namespace mcs
