// divmod_kernels.hip -- batched quotient and remainder by Mersenne and
// pseudo-Mersenne primes (Section 1.5 and Section 4 of Ahle, Knudsen, Thorup).
// Streaming, HBM-bound: each thread handles kUnroll independent values per
// iteration so several loads are in flight; the arithmetic is field.hpp's.
#include <algorithm>

#include "sketch_kernels.hpp"

namespace mcs {

constexpr int kUnroll = 4;

// prime 1 (2^61-1, Algorithm 4) and prime 3 (2^64-59, Algorithms 5 and 6):
// x is n x 2 limbs, quot and rem n x 1 limb.
template <int PRIME, bool Q, bool R>
__global__ __launch_bounds__(kBlock) void k_divmod2(const ulonglong2* __restrict__ x, uint64_t n,
                                                    uint64_t* __restrict__ quot, uint64_t* __restrict__ rem,
                                                    uint32_t* flags) {
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  uint32_t bad = 0;
  for (uint64_t base = (uint64_t)blockIdx.x * kBlock + threadIdx.x; base < n; base += stride * kUnroll) {
    ulonglong2 v[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      uint64_t i = base + u * stride;
      v[u] = i < n ? x[i] : make_ulonglong2(0, 0);
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      uint64_t i = base + u * stride;
      uint64_t q, r;
      if (PRIME == kPrime61) {
        bad |= (uint32_t)(v[u].y >> 58 != 0);
        p61_divmod(v[u].x, v[u].y, q, r);
      } else {
        bad |= (uint32_t)(v[u].y >= 0xFFFFFFFFFFFFFFFFull - 58);
        p64c_divmod(v[u].x, v[u].y, q, r);
      }
      if (i < n) {
        if (Q) quot[i] = q;
        if (R) rem[i] = r;
      }
    }
  }
  if (__any(bad)) {
    if (bad) atomicOr(flags, kFlagDomain);
  }
}

// prime 2 (2^89-1, Algorithm 4): x is n x 3 limbs, quot and rem n x 2 limbs.
template <bool Q, bool R>
__global__ __launch_bounds__(kBlock) void k_divmod89(const uint64_t* __restrict__ x, uint64_t n,
                                                     ulonglong2* __restrict__ quot, ulonglong2* __restrict__ rem,
                                                     uint32_t* flags) {
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  uint32_t bad = 0;
  for (uint64_t base = (uint64_t)blockIdx.x * kBlock + threadIdx.x; base < n; base += stride * kUnroll) {
    uint64_t v0[kUnroll], v1[kUnroll], v2[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      uint64_t i = base + u * stride;
      if (i < n) {
        v0[u] = x[3 * i];
        v1[u] = x[3 * i + 1];
        v2[u] = x[3 * i + 2];
      } else {
        v0[u] = v1[u] = v2[u] = 0;
      }
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      uint64_t i = base + u * stride;
      uint64_t q0, q1, r0, r1;
      bad |= (uint32_t)(v2[u] >> 50 != 0);
      p89_divmod(v0[u], v1[u], v2[u], q0, q1, r0, r1);
      if (i < n) {
        if (Q) quot[i] = make_ulonglong2(q0, q1);
        if (R) rem[i] = make_ulonglong2(r0, r1);
      }
    }
  }
  if (bad) atomicOr(flags, kFlagDomain);
}

// ---------------------------------------------------------------------------
// Comparator: the compiler's 128-bit `/` and `%` (primes 1 and 3) and a
// shift-and-subtract long division for prime 2.
// ---------------------------------------------------------------------------
template <int PRIME>
__global__ __launch_bounds__(kBlock) void k_divmod2_naive(const ulonglong2* __restrict__ x, uint64_t n,
                                                          uint64_t* __restrict__ quot, uint64_t* __restrict__ rem,
                                                          uint32_t* flags) {
  typedef unsigned __int128 u128;
  const u128 p = PRIME == kPrime61 ? (u128)kP61 : (u128)(0xFFFFFFFFFFFFFFFFull - 58);
  uint32_t bad = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kBlock) {
    ulonglong2 v = x[i];
    bad |= PRIME == kPrime61 ? (uint32_t)(v.y >> 58 != 0) : (uint32_t)(v.y >= (uint64_t)p);
    u128 w = ((u128)v.y << 64) | v.x;
    if (quot) quot[i] = (uint64_t)(w / p);
    if (rem) rem[i] = (uint64_t)(w % p);
  }
  if (bad) atomicOr(flags, kFlagDomain);
}

__global__ __launch_bounds__(kBlock) void k_divmod89_naive(const uint64_t* __restrict__ x, uint64_t n,
                                                           ulonglong2* __restrict__ quot, ulonglong2* __restrict__ rem,
                                                           uint32_t* flags) {
  typedef unsigned __int128 u128;
  const u128 p = (((u128)1) << 89) - 1;
  uint32_t bad = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kBlock) {
    uint64_t limb[3] = {x[3 * i], x[3 * i + 1], x[3 * i + 2]};
    bad |= (uint32_t)(limb[2] >> 50 != 0);
    u128 r = 0, q = 0;
    for (int bit = 177; bit >= 0; --bit) {
      r = (r << 1) | ((limb[bit >> 6] >> (bit & 63)) & 1);
      q <<= 1;
      if (r >= p) {
        r -= p;
        q |= 1;
      }
    }
    if (quot) quot[i] = make_ulonglong2((uint64_t)q, (uint64_t)(q >> 64));
    if (rem) rem[i] = make_ulonglong2((uint64_t)r, (uint64_t)(r >> 64));
  }
  if (bad) atomicOr(flags, kFlagDomain);
}

static uint32_t grid_for(uint64_t n, uint64_t per_thread) {
  uint64_t blocks = (n + (uint64_t)kBlock * per_thread - 1) / ((uint64_t)kBlock * per_thread);
  if (blocks > 65536) blocks = 65536;
  if (blocks == 0) blocks = 1;
  return (uint32_t)blocks;
}

// Most uniform maps of hash values v in [p] to [r] buckets (Section 1.4 and
// Section 1.5):
//   exact     floor(v r / p): the quotient of the product v r (< p 2^32, inside
//             every divmod domain) by Algorithm 4 or Algorithms 5 and 6
//   mersenne  ((v + 1) r) >> b (eq. most-uniform)
// v >= p sets the domain flag (its bucket is unspecified).
template <int PRIME, bool FAST>
__global__ __launch_bounds__(kBlock) void k_bucket_map(const uint64_t* __restrict__ v, uint64_t n, uint32_t r,
                                                       uint32_t* __restrict__ out, uint32_t* flags) {
  typedef unsigned __int128 u128;
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  uint32_t bad = 0;
  for (uint64_t base = (uint64_t)blockIdx.x * kBlock + threadIdx.x; base < n; base += stride * kUnroll) {
    uint64_t lo[kUnroll], hi[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const uint64_t i = base + u * stride;
      lo[u] = hi[u] = 0;
      if (i < n) {
        if (PRIME == kPrime89) {
          const ulonglong2 w = reinterpret_cast<const ulonglong2*>(v)[i];
          lo[u] = w.x;
          hi[u] = w.y;
        } else {
          lo[u] = v[i];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const uint64_t i = base + u * stride;
      uint32_t b;
      if (PRIME == kPrime61) {
        bad |= (uint32_t)(lo[u] >= (1ull << 61) - 1);
        if (FAST) {
          b = (uint32_t)((((u128)(lo[u] + 1)) * r) >> 61);
        } else {
          const u128 x = (u128)lo[u] * r;
          uint64_t q, rem;
          p61_divmod((uint64_t)x, (uint64_t)(x >> 64), q, rem);
          b = (uint32_t)q;
        }
      } else if (PRIME == kPrime64c) {
        bad |= (uint32_t)(lo[u] >= 0xFFFFFFFFFFFFFFFFull - 58);
        const u128 x = (u128)lo[u] * r;
        uint64_t q, rem;
        p64c_divmod((uint64_t)x, (uint64_t)(x >> 64), q, rem);
        b = (uint32_t)q;
      } else {
        bad |= (uint32_t)(hi[u] > (1ull << 25) - 1 || (hi[u] == (1ull << 25) - 1 && lo[u] == ~0ull));
        const u128 vv = ((u128)hi[u] << 64) | lo[u];
        if (FAST) {
          b = (uint32_t)(((vv + 1) * r) >> 89);
        } else {
          const u128 x = vv * r;  // < 2^121
          uint64_t q0, q1, r0, r1;
          p89_divmod((uint64_t)x, (uint64_t)(x >> 64), 0, q0, q1, r0, r1);
          b = (uint32_t)q0;
        }
      }
      if (i < n) out[i] = b;
    }
  }
  if (__any(bad)) {
    if (bad) atomicOr(flags, kFlagDomain);
  }
}

hipError_t launch_bucket_map(int prime, bool fast, const uint64_t* v, uint64_t n, uint32_t r, uint32_t* out,
                             uint32_t* flags, uint32_t cus, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const uint64_t want = (n + (uint64_t)kBlock * kUnroll - 1) / ((uint64_t)kBlock * kUnroll);
  const uint32_t g = (uint32_t)std::min<uint64_t>(want, (uint64_t)cus * 16);
  if (prime == kPrime61) {
    if (fast) hipLaunchKernelGGL((k_bucket_map<kPrime61, true>), dim3(g), dim3(kBlock), 0, st, v, n, r, out, flags);
    else hipLaunchKernelGGL((k_bucket_map<kPrime61, false>), dim3(g), dim3(kBlock), 0, st, v, n, r, out, flags);
  } else if (prime == kPrime89) {
    if (fast) hipLaunchKernelGGL((k_bucket_map<kPrime89, true>), dim3(g), dim3(kBlock), 0, st, v, n, r, out, flags);
    else hipLaunchKernelGGL((k_bucket_map<kPrime89, false>), dim3(g), dim3(kBlock), 0, st, v, n, r, out, flags);
  } else {
    hipLaunchKernelGGL((k_bucket_map<kPrime64c, false>), dim3(g), dim3(kBlock), 0, st, v, n, r, out, flags);
  }
  return hipGetLastError();
}

hipError_t launch_divmod(int prime, bool naive, const uint64_t* x, uint64_t n, uint64_t* quot, uint64_t* rem,
                         uint32_t* flags, hipStream_t st) {
  if (n == 0) return hipSuccess;
  if (naive) {
    uint32_t g = grid_for(n, 1);
    if (prime == kPrime89)
      hipLaunchKernelGGL(k_divmod89_naive, dim3(g), dim3(kBlock), 0, st, x, n, (ulonglong2*)quot, (ulonglong2*)rem,
                         flags);
    else if (prime == kPrime61)
      hipLaunchKernelGGL(k_divmod2_naive<kPrime61>, dim3(g), dim3(kBlock), 0, st, (const ulonglong2*)x, n, quot, rem,
                         flags);
    else
      hipLaunchKernelGGL(k_divmod2_naive<kPrime64c>, dim3(g), dim3(kBlock), 0, st, (const ulonglong2*)x, n, quot,
                         rem, flags);
    return hipGetLastError();
  }
  uint32_t g = grid_for(n, kUnroll * 4);
  const bool Q = quot != nullptr, R = rem != nullptr;
  if (prime == kPrime89) {
    if (Q && R) hipLaunchKernelGGL((k_divmod89<true, true>), dim3(g), dim3(kBlock), 0, st, x, n, (ulonglong2*)quot, (ulonglong2*)rem, flags);
    else if (Q) hipLaunchKernelGGL((k_divmod89<true, false>), dim3(g), dim3(kBlock), 0, st, x, n, (ulonglong2*)quot, (ulonglong2*)rem, flags);
    else hipLaunchKernelGGL((k_divmod89<false, true>), dim3(g), dim3(kBlock), 0, st, x, n, (ulonglong2*)quot, (ulonglong2*)rem, flags);
  } else if (prime == kPrime61) {
    const ulonglong2* xv = (const ulonglong2*)x;
    if (Q && R) hipLaunchKernelGGL((k_divmod2<kPrime61, true, true>), dim3(g), dim3(kBlock), 0, st, xv, n, quot, rem, flags);
    else if (Q) hipLaunchKernelGGL((k_divmod2<kPrime61, true, false>), dim3(g), dim3(kBlock), 0, st, xv, n, quot, rem, flags);
    else hipLaunchKernelGGL((k_divmod2<kPrime61, false, true>), dim3(g), dim3(kBlock), 0, st, xv, n, quot, rem, flags);
  } else {
    const ulonglong2* xv = (const ulonglong2*)x;
    if (Q && R) hipLaunchKernelGGL((k_divmod2<kPrime64c, true, true>), dim3(g), dim3(kBlock), 0, st, xv, n, quot, rem, flags);
    else if (Q) hipLaunchKernelGGL((k_divmod2<kPrime64c, true, false>), dim3(g), dim3(kBlock), 0, st, xv, n, quot, rem, flags);
    else hipLaunchKernelGGL((k_divmod2<kPrime64c, false, true>), dim3(g), dim3(kBlock), 0, st, xv, n, quot, rem, flags);
  }
  return hipGetLastError();
}

}  // namespace mcs
