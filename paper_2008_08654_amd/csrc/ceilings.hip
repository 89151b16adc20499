// ceilings.hip -- measured ceilings behind the rooflines (include/mcs_ceilings.h):
// issue rates of the VALU instructions the hash is made of, the HBM read
// stream, LDS atomics and device-scope global atomics.  Each probe is one
// launch; the caller times it and divides the operation count by the time.
#include <hip/hip_runtime.h>

#include "mcs.h"
#include "mcs_ceilings.h"
#include "mcs_internal.hpp"

using namespace mcs;

namespace {

constexpr int kCeilBlock = 256;
constexpr int kChains = 8;   // independent dependency chains per thread
constexpr int kUnroll = 16;  // instructions per chain per loop trip

// kChains * kUnroll instructions of one kind per trip on independent
// register chains (written in asm so that exactly that instruction runs).
template <int OP>
__global__ __launch_bounds__(kCeilBlock) void k_issue(uint32_t iters, uint64_t* __restrict__ sink) {
  uint64_t a[kChains];
  uint32_t b[kChains];
  const uint32_t x = threadIdx.x | 1u, y = threadIdx.x * 3u + 7u;
#pragma unroll
  for (int i = 0; i < kChains; ++i) {
    a[i] = (uint64_t)(threadIdx.x + i) * 0x9E3779B97F4A7C15ull;
    b[i] = threadIdx.x + 17u * i;
  }
  for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
#pragma unroll
      for (int i = 0; i < kChains; ++i) {
        if constexpr (OP == CS_CEIL_VALU_ADD32)
          asm volatile("v_add_u32 %0, %0, %1" : "+v"(b[i]) : "v"(x));
        else if constexpr (OP == CS_CEIL_MAD_U64_U32)
          asm volatile("v_mad_u64_u32 %0, vcc, %1, %2, %0" : "+v"(a[i]) : "v"(x), "v"(y) : "vcc");
        else if constexpr (OP == CS_CEIL_LSHL_ADD_U64)
          asm volatile("v_lshl_add_u64 %0, %0, 1, %1" : "+v"(a[i]) : "v"((uint64_t)y));
        else if constexpr (OP == CS_CEIL_LSHRREV_B64)
          asm volatile("v_lshrrev_b64 %0, 1, %0" : "+v"(a[i]));
        else if constexpr (OP == CS_CEIL_MOV_B32)
          asm volatile("v_mov_b32 %0, %1" : "=v"(b[i]) : "v"(b[(i + 1) % kChains]));
        else if constexpr (OP == CS_CEIL_BFE_U32)
          asm volatile("v_bfe_u32 %0, %0, %1, 16" : "+v"(b[i]) : "v"(x));
        else if constexpr (OP == CS_CEIL_AND_OR_B32)
          asm volatile("v_and_or_b32 %0, %0, %1, %2" : "+v"(b[i]) : "v"(x), "v"(y));
        else if constexpr (OP == CS_CEIL_XAD_U32)
          asm volatile("v_xad_u32 %0, %0, %1, %2" : "+v"(b[i]) : "v"(x), "v"(y));
        else if constexpr (OP == CS_CEIL_LSHLREV_B32)
          asm volatile("v_lshlrev_b32_e32 %0, %1, %0" : "+v"(b[i]) : "v"(x));
        else if constexpr (OP == CS_CEIL_AND_B32)
          asm volatile("v_and_b32_e32 %0, %1, %0" : "+v"(b[i]) : "v"(x));
        else if constexpr (OP == CS_CEIL_ADD_CO_U32) {
          if (i & 1)
            asm volatile("v_addc_co_u32_e32 %0, vcc, %1, %0, vcc" : "+v"(b[i]) : "v"(x) : "vcc");
          else
            asm volatile("v_add_co_u32_e32 %0, vcc, %1, %0" : "+v"(b[i]) : "v"(x) : "vcc");
        } else if constexpr (OP == CS_CEIL_ADD32_ONE_WAVE)
          asm volatile("v_add_u32 %0, %0, %1" : "+v"(b[i]) : "v"(x));
        else {  // CS_CEIL_MIX_MAD_ADD
          if (i & 1)
            asm volatile("v_add_u32 %0, %0, %1" : "+v"(b[i]) : "v"(x));
          else
            asm volatile("v_mad_u64_u32 %0, vcc, %1, %2, %0" : "+v"(a[i]) : "v"(x), "v"(y) : "vcc");
        }
      }
    }
  }
  uint64_t s = 0;
#pragma unroll
  for (int i = 0; i < kChains; ++i) s ^= a[i] ^ b[i];
  if (s == 0x0123456789ABCDEFull) sink[0] = s;  // keeps the chains live
}

// Reads `words` 16-byte words once (grid-stride), xor-reduces them.
__global__ __launch_bounds__(kCeilBlock) void k_read(const uint4* __restrict__ p, uint64_t words,
                                                     uint64_t* __restrict__ sink) {
  uint32_t acc = 0;
  const uint64_t stride = (uint64_t)gridDim.x * kCeilBlock;
  uint64_t i = (uint64_t)blockIdx.x * kCeilBlock + threadIdx.x;
  for (; i + 3 * stride < words; i += 4 * stride) {
    const uint4 v0 = p[i], v1 = p[i + stride], v2 = p[i + 2 * stride], v3 = p[i + 3 * stride];
    acc ^= v0.x ^ v0.y ^ v0.z ^ v0.w ^ v1.x ^ v1.y ^ v1.z ^ v1.w ^ v2.x ^ v2.y ^ v2.z ^ v2.w ^ v3.x ^ v3.y ^ v3.z ^ v3.w;
  }
  for (; i < words; i += stride) {
    const uint4 v = p[i];
    acc ^= v.x ^ v.y ^ v.z ^ v.w;
  }
  if (acc == 0x12345678u) sink[0] = acc;
}

// iters LDS atomics per thread at pseudo-random addresses of a 64 KiB table.
template <int OP>
__global__ __launch_bounds__(kCeilBlock) void k_lds_atomic(uint32_t iters, uint64_t* __restrict__ sink) {
  __shared__ unsigned long long t[8192];
  for (uint32_t i = threadIdx.x; i < 8192; i += kCeilBlock) t[i] = 0;
  __syncthreads();
  uint32_t h = threadIdx.x * 0x9E3779B1u + blockIdx.x, acc = 0;
  for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      h = h * 1664525u + 1013904223u;
      if constexpr (OP == CS_CEIL_LDS_ADD_U64)
        atomicAdd(&t[h >> 19], 1ull);
      else
        acc += atomicAdd((uint32_t*)t + (h >> 18), 1u);
    }
  }
  __syncthreads();
  if (acc == 0x12345678u || t[threadIdx.x] == 0x123456789ull) sink[0] = acc;
}

// iters device-scope int64 atomics per thread into `cells` counters: at
// pseudo-random cells, or coalesced (a wave's lanes on consecutive cells).
template <int OP>
__global__ __launch_bounds__(kCeilBlock) void k_global_atomic(unsigned long long* __restrict__ c, uint64_t cells,
                                                              uint32_t iters) {
  const uint64_t tid = (uint64_t)blockIdx.x * kCeilBlock + threadIdx.x;
  uint64_t h = tid * 0x9E3779B97F4A7C15ull + 1;
  const uint64_t nthreads = (uint64_t)gridDim.x * kCeilBlock;
  for (uint32_t it = 0; it < iters; ++it) {
    uint64_t i;
    if constexpr (OP == CS_CEIL_GLOBAL_ATOMIC_RANDOM) {
      h ^= h >> 33;
      h *= 0xFF51AFD7ED558CCDull;
      h ^= h >> 29;
      i = h % cells;
    } else {
      i = (tid + (uint64_t)it * nthreads) % cells;
    }
    atomicAdd(&c[i], 1ull);
  }
}

}  // namespace

extern "C" cs_status cs_ceiling_run(int probe, void* buffer, uint64_t bytes, uint32_t iters, uint64_t* ops,
                                    hipStream_t stream) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  const uint32_t cus = (uint32_t)device_info(dev).cus;
  const uint32_t grid = cus * 8;  // 8 blocks of 4 waves per CU: 8 waves per SIMD
  uint64_t count = 0;
  switch (probe) {
    case CS_CEIL_VALU_ADD32:
    case CS_CEIL_MAD_U64_U32:
    case CS_CEIL_LSHL_ADD_U64:
    case CS_CEIL_LSHRREV_B64:
    case CS_CEIL_MOV_B32:
    case CS_CEIL_BFE_U32:
    case CS_CEIL_AND_OR_B32:
    case CS_CEIL_XAD_U32:
    case CS_CEIL_LSHLREV_B32:
    case CS_CEIL_AND_B32:
    case CS_CEIL_ADD_CO_U32:
    case CS_CEIL_ADD32_ONE_WAVE:
    case CS_CEIL_MIX_MAD_ADD: {
      if (iters == 0) return fail(CS_EINVAL, "iters must be positive");
      uint64_t* sink = (uint64_t*)buffer;
      if (!sink || bytes < 8) return fail(CS_EINVAL, "the issue probes need an 8-byte device buffer");
      if (probe == CS_CEIL_VALU_ADD32)
        hipLaunchKernelGGL(k_issue<CS_CEIL_VALU_ADD32>, dim3(grid), dim3(kCeilBlock), 0, stream, iters, sink);
      else if (probe == CS_CEIL_MAD_U64_U32)
        hipLaunchKernelGGL(k_issue<CS_CEIL_MAD_U64_U32>, dim3(grid), dim3(kCeilBlock), 0, stream, iters, sink);
      else if (probe == CS_CEIL_LSHL_ADD_U64)
        hipLaunchKernelGGL(k_issue<CS_CEIL_LSHL_ADD_U64>, dim3(grid), dim3(kCeilBlock), 0, stream, iters, sink);
      else if (probe == CS_CEIL_LSHRREV_B64)
        hipLaunchKernelGGL(k_issue<CS_CEIL_LSHRREV_B64>, dim3(grid), dim3(kCeilBlock), 0, stream, iters, sink);
      else if (probe == CS_CEIL_MOV_B32)
        hipLaunchKernelGGL(k_issue<CS_CEIL_MOV_B32>, dim3(grid), dim3(kCeilBlock), 0, stream, iters, sink);
      else if (probe == CS_CEIL_BFE_U32)
        hipLaunchKernelGGL(k_issue<CS_CEIL_BFE_U32>, dim3(grid), dim3(kCeilBlock), 0, stream, iters, sink);
      else if (probe == CS_CEIL_AND_OR_B32)
        hipLaunchKernelGGL(k_issue<CS_CEIL_AND_OR_B32>, dim3(grid), dim3(kCeilBlock), 0, stream, iters, sink);
      else if (probe == CS_CEIL_XAD_U32)
        hipLaunchKernelGGL(k_issue<CS_CEIL_XAD_U32>, dim3(grid), dim3(kCeilBlock), 0, stream, iters, sink);
      else if (probe == CS_CEIL_LSHLREV_B32)
        hipLaunchKernelGGL(k_issue<CS_CEIL_LSHLREV_B32>, dim3(grid), dim3(kCeilBlock), 0, stream, iters, sink);
      else if (probe == CS_CEIL_AND_B32)
        hipLaunchKernelGGL(k_issue<CS_CEIL_AND_B32>, dim3(grid), dim3(kCeilBlock), 0, stream, iters, sink);
      else if (probe == CS_CEIL_ADD_CO_U32)
        hipLaunchKernelGGL(k_issue<CS_CEIL_ADD_CO_U32>, dim3(grid), dim3(kCeilBlock), 0, stream, iters, sink);
      else if (probe == CS_CEIL_ADD32_ONE_WAVE)
        hipLaunchKernelGGL(k_issue<CS_CEIL_ADD32_ONE_WAVE>, dim3(cus), dim3(kCeilBlock), 0, stream, iters, sink);
      else
        hipLaunchKernelGGL(k_issue<CS_CEIL_MIX_MAD_ADD>, dim3(grid), dim3(kCeilBlock), 0, stream, iters, sink);
      count = (uint64_t)(probe == CS_CEIL_ADD32_ONE_WAVE ? cus : grid) * kCeilBlock * iters * kChains *
              kUnroll;  // lane-instructions
      break;
    }
    case CS_CEIL_HBM_READ: {
      // the first 8 bytes are the sink; the rest is read
      if (!buffer || bytes < (1u << 20)) return fail(CS_EINVAL, "the read probe needs at least 1 MiB");
      const uint64_t words = (bytes - 256) / 16;
      hipLaunchKernelGGL(k_read, dim3(grid), dim3(kCeilBlock), 0, stream, (const uint4*)((char*)buffer + 256), words,
                         (uint64_t*)buffer);
      count = words * 16;  // bytes
      break;
    }
    case CS_CEIL_LDS_ADD_U64:
    case CS_CEIL_LDS_ADD_RTN_U32: {
      if (iters == 0 || !buffer || bytes < 8) return fail(CS_EINVAL, "the LDS probes need iters and a sink");
      if (probe == CS_CEIL_LDS_ADD_U64)
        hipLaunchKernelGGL(k_lds_atomic<CS_CEIL_LDS_ADD_U64>, dim3(grid), dim3(kCeilBlock), 0, stream, iters,
                           (uint64_t*)buffer);
      else
        hipLaunchKernelGGL(k_lds_atomic<CS_CEIL_LDS_ADD_RTN_U32>, dim3(grid), dim3(kCeilBlock), 0, stream, iters,
                           (uint64_t*)buffer);
      count = (uint64_t)grid * kCeilBlock * iters * 8;  // atomics
      break;
    }
    case CS_CEIL_GLOBAL_ATOMIC_RANDOM:
    case CS_CEIL_GLOBAL_ATOMIC_COALESCED: {
      const uint64_t cells = bytes / 8;
      if (iters == 0 || !buffer || cells == 0) return fail(CS_EINVAL, "the atomic probes need iters and counters");
      if (probe == CS_CEIL_GLOBAL_ATOMIC_RANDOM)
        hipLaunchKernelGGL(k_global_atomic<CS_CEIL_GLOBAL_ATOMIC_RANDOM>, dim3(grid), dim3(kCeilBlock), 0, stream,
                           (unsigned long long*)buffer, cells, iters);
      else
        hipLaunchKernelGGL(k_global_atomic<CS_CEIL_GLOBAL_ATOMIC_COALESCED>, dim3(grid), dim3(kCeilBlock), 0, stream,
                           (unsigned long long*)buffer, cells, iters);
      count = (uint64_t)grid * kCeilBlock * iters;  // atomics
      break;
    }
    default:
      return fail(CS_EINVAL, "unknown probe %d", probe);
  }
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "ceiling probe launch");
  if (ops) *ops = count;
  return CS_OK;
}
