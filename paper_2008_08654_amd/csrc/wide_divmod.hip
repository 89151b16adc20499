// wide_divmod.hip -- quotient and remainder of 2b-bit numbers by p = 2^b - c
// for b = 32 W, W in {1, 2, 4, 8, 16, 32}: the division experiment of
// Section 5 (b from 32 to 1024) on the GPU.
//
//   Algorithm 5 (+ Algorithm 6 for the remainder), m steps:
//     v' = v + c; z = v' >> b; m-1 times z = (z c + v') >> b; r = (v + z c) mod 2^b
//   Algorithm 10 (Crandall, Chung and Hasan), the paper's comparator:
//     q = x >> b, r = x mod 2^b; while the last quotient q_i > 0 add the high and
//     low parts of q_i c into q and r; then subtract p from r while r >= p.
//
// Values are limb planes (limb j of value i at x[j n + i]), so the lanes of a
// wave read consecutive words of each plane.  One thread per value; the limb
// loops are unrolled for each W, with 64-bit accumulators for the carries.
#include "sketch_kernels.hpp"

namespace mcs {

// Limb j of z c for a multi-limb z and a 32-bit c, with the product's running
// carry `mc` (for c = 1 the limb itself).
template <bool C1>
__device__ __forceinline__ uint32_t zc_limb(uint32_t zj, uint32_t c, uint64_t& mc) {
  if (C1) return zj;
  const uint64_t p = (uint64_t)zj * c + mc;
  mc = p >> 32;
  return (uint32_t)p;
}

template <int W, bool C1>
__global__ __launch_bounds__(kBlock, 2) void k_wide_alg5(const uint32_t* __restrict__ x, uint64_t n, uint32_t c,
                                                      uint32_t m, uint32_t* __restrict__ quot,
                                                      uint32_t* __restrict__ rem) {
  const uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  uint32_t vp[2 * W + 1], z[W + 1];
  // all limbs are loaded before the carry chain uses any, so the loads are in
  // flight together
  const uint32_t* px = x + i;
#pragma unroll
  for (int j = 0; j < 2 * W; ++j, px += n) vp[j] = *px;
  // v' = v + c (one more limb for the carry)
  uint64_t s = (uint64_t)vp[0] + c;
  vp[0] = (uint32_t)s;
#pragma unroll
  for (int j = 1; j < 2 * W; ++j) {
    s = (uint64_t)vp[j] + (s >> 32);
    vp[j] = (uint32_t)s;
  }
  vp[2 * W] = (uint32_t)(s >> 32);
  // z = v' >> b
#pragma unroll
  for (int j = 0; j <= W; ++j) z[j] = vp[W + j];
  for (uint32_t step = 1; step < m; ++step) {
    // z = (z c + v') >> b, in place: limb j - W of the new z is written at limb j
    // of the sum, after the old limb j - W has been used
    uint64_t carry = 0, mc = 0;
#pragma unroll
    for (int j = 0; j <= 2 * W; ++j) {
      uint32_t zc = 0;
      if (j <= W) zc = zc_limb<C1>(z[j], c, mc);
      else if (j == W + 1 && !C1) zc = (uint32_t)mc;
      const uint64_t a = (uint64_t)vp[j] + zc + carry;
      carry = a >> 32;
      if (j >= W) z[j - W] = (uint32_t)a;
    }
  }
  if (quot) {
#pragma unroll
    for (int j = 0; j <= W; ++j) quot[(size_t)j * n + i] = z[j];
  }
  if (rem) {
    // Algorithm 6: r = (v + z c) mod 2^b = (v' + z c - c) mod 2^b
    uint64_t carry = 0, mc = 0;
    int64_t borrow = -(int64_t)c;
#pragma unroll
    for (int j = 0; j < W; ++j) {
      const uint64_t a = (uint64_t)vp[j] + zc_limb<C1>(z[j], c, mc) + carry;
      carry = a >> 32;
      const int64_t d = (int64_t)(uint32_t)a + borrow;
      borrow = d >> 32;  // 0 or -1 after the first limb
      rem[(size_t)j * n + i] = (uint32_t)d;
    }
  }
}

template <int W, bool C1>
__global__ __launch_bounds__(kBlock, 2) void k_wide_cch(const uint32_t* __restrict__ x, uint64_t n, uint32_t c,
                                                     uint32_t* __restrict__ quot, uint32_t* __restrict__ rem) {
  const uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  // q = q_0 = x >> b, r = r_0 = x mod 2^b (one spare limb each for the sums)
  uint32_t q[W + 1], r[W + 1];
  const uint32_t* px = x + i;
#pragma unroll
  for (int j = 0; j < W; ++j, px += n) r[j] = *px;
#pragma unroll
  for (int j = 0; j < W; ++j, px += n) q[j] = *px;
  q[W] = r[W] = 0;
  // first pass of the loop, t = q_0 c: r += t mod 2^b, q_1 = t >> b (one limb)
  uint32_t any = 0;
#pragma unroll
  for (int j = 0; j < W; ++j) any |= q[j];
  uint32_t qi = 0;
  if (any) {
    uint64_t mc = 0, cr = 0;
#pragma unroll
    for (int j = 0; j < W; ++j) {
      const uint32_t lo = zc_limb<C1>(q[j], c, mc);
      const uint64_t a = (uint64_t)r[j] + lo + cr;
      r[j] = (uint32_t)a;
      cr = a >> 32;
    }
    r[W] += (uint32_t)cr;
    qi = (uint32_t)mc;
  }
  // later passes: q_i has one limb, t = q_i c has two
  while (qi) {
    uint64_t a = (uint64_t)q[0] + qi;  // q += q_i
    q[0] = (uint32_t)a;
#pragma unroll
    for (int j = 1; j <= W; ++j) {
      a = (uint64_t)q[j] + (a >> 32);
      q[j] = (uint32_t)a;
    }
    const uint64_t t = (uint64_t)qi * c;
    uint32_t lo0, lo1, hi;
    if (W == 1) {
      lo0 = (uint32_t)t;
      lo1 = 0;
      hi = (uint32_t)(t >> 32);
    } else {
      lo0 = (uint32_t)t;
      lo1 = (uint32_t)(t >> 32);
      hi = 0;
    }
    uint64_t cr = (uint64_t)r[0] + lo0;
    r[0] = (uint32_t)cr;
#pragma unroll
    for (int j = 1; j <= W; ++j) {
      cr = (uint64_t)r[j] + (j == 1 ? lo1 : 0u) + (cr >> 32);
      r[j] = (uint32_t)cr;
    }
    qi = hi;
  }
  // clean up: while r >= p = 2^b - c (i.e. r + c >= 2^b), r -= p and q += 1
  for (;;) {
    uint64_t a = (uint64_t)r[0] + c;
#pragma unroll
    for (int j = 1; j < W; ++j) a = (uint64_t)r[j] + (a >> 32);
    if (r[W] + (uint32_t)(a >> 32) == 0) break;
    a = (uint64_t)r[0] + c;
    r[0] = (uint32_t)a;
#pragma unroll
    for (int j = 1; j < W; ++j) {
      a = (uint64_t)r[j] + (a >> 32);
      r[j] = (uint32_t)a;
    }
    r[W] = r[W] + (uint32_t)(a >> 32) - 1;
    uint64_t b = (uint64_t)q[0] + 1;
    q[0] = (uint32_t)b;
#pragma unroll
    for (int j = 1; j <= W; ++j) {
      b = (uint64_t)q[j] + (b >> 32);
      q[j] = (uint32_t)b;
    }
  }
  if (quot) {
#pragma unroll
    for (int j = 0; j <= W; ++j) quot[(size_t)j * n + i] = q[j];
  }
  if (rem) {
#pragma unroll
    for (int j = 0; j < W; ++j) rem[(size_t)j * n + i] = r[j];
  }
}

template <int W>
static hipError_t launch_wide_w(int method, uint32_t c, uint32_t m, const uint32_t* x, uint64_t n, uint32_t* quot,
                                uint32_t* rem, hipStream_t st) {
  const uint32_t blocks = (uint32_t)((n + kBlock - 1) / kBlock);
  if (method == 1 && c == 1)
    hipLaunchKernelGGL((k_wide_cch<W, true>), dim3(blocks), dim3(kBlock), 0, st, x, n, c, quot, rem);
  else if (method == 1)
    hipLaunchKernelGGL((k_wide_cch<W, false>), dim3(blocks), dim3(kBlock), 0, st, x, n, c, quot, rem);
  else if (c == 1)
    hipLaunchKernelGGL((k_wide_alg5<W, true>), dim3(blocks), dim3(kBlock), 0, st, x, n, c, m, quot, rem);
  else
    hipLaunchKernelGGL((k_wide_alg5<W, false>), dim3(blocks), dim3(kBlock), 0, st, x, n, c, m, quot, rem);
  return hipGetLastError();
}

hipError_t launch_wide_divmod(uint32_t b, uint32_t c, uint32_t m, int method, const uint32_t* x, uint64_t n,
                              uint32_t* quot, uint32_t* rem, hipStream_t st) {
  if (n == 0) return hipSuccess;
  switch (b) {
    case 32: return launch_wide_w<1>(method, c, m, x, n, quot, rem, st);
    case 64: return launch_wide_w<2>(method, c, m, x, n, quot, rem, st);
    case 128: return launch_wide_w<4>(method, c, m, x, n, quot, rem, st);
    case 256: return launch_wide_w<8>(method, c, m, x, n, quot, rem, st);
    case 512: return launch_wide_w<16>(method, c, m, x, n, quot, rem, st);
    case 1024: return launch_wide_w<32>(method, c, m, x, n, quot, rem, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace mcs
