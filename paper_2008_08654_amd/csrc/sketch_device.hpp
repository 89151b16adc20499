// sketch_device.hpp -- Count Sketch kernels and their launchers as templates
// over (prime, bucket/sign mode, k, key type, weight type), for Algorithm 2 of
// Ahle, Knudsen, Thorup, "The Power of Hashing with Mersenne Primes".
//
// Per key and row: Horner evaluation of the row's polynomial over p
// (Algorithm 1, field.hpp), branch-free final reduction (Algorithm 4), the
// bucket/sign split (Algorithm 3, the low-bit layout of Section 1.2.1, two
// polynomials, or Algorithm 8 for any bucket count), and a signed int64 add
// into the row's counters.
//
// Coefficients live in device memory as one 16-byte record per coefficient
// (32-bit limbs w0, w1, w2, and the bucket count r in the spare fourth word),
// indexed [row][poly][i]; the row loop is the outer loop so each row's
// coefficients are wave-uniform scalar loads.
//
// Each (prime, mode) pair is instantiated in a translation unit of its own
// (sketch_p*_*.hip); the non-template kernels and the dispatch live in
// sketch_kernels.hip.
#pragma once
#include <algorithm>
#include <atomic>

#include "device_util.hpp"
#include "sketch_kernels.hpp"

namespace mcs {

// ---------------------------------------------------------------------------
// hashing of one key in one row
// ---------------------------------------------------------------------------
// A row's coefficients, read once per row and kept in scalar registers
// (readfirstlane): all lanes hash with the same polynomial.
template <int K, int NP>
struct RowCoeffs {
  uint32_t w[NP * K][3];
  uint32_t r;  // bucket count (used by the arbitrary-r split)
};

template <int K, int NP>
__device__ __forceinline__ RowCoeffs<K, NP> load_row_coeffs(const uint4* __restrict__ c) {
  RowCoeffs<K, NP> rc;
  // the coefficients do not change during a launch: read them through the
  // constant address space, so they come in scalar loads
  const auto* cc = (const __attribute__((address_space(4))) uint32_t*)c;
#pragma unroll
  for (int i = 0; i < NP * K; ++i) {
    rc.w[i][0] = __builtin_amdgcn_readfirstlane(cc[4 * i]);
    rc.w[i][1] = __builtin_amdgcn_readfirstlane(cc[4 * i + 1]);
    rc.w[i][2] = __builtin_amdgcn_readfirstlane(cc[4 * i + 2]);
    if (i == 0) rc.r = __builtin_amdgcn_readfirstlane(cc[3]);
  }
  return rc;
}

// Horner's rule (Algorithm 1) for polynomial q of the row, before the final
// reduction: a value < 2p congruent to h(x).
template <int K, int NP>
__device__ __forceinline__ F61 horner61_x32(const RowCoeffs<K, NP>& c, int q, uint32_t x) {
  // the steps before the last fold at bit 64 (p61_step_x32_lazy); on a carry
  // in any lane the wave takes the exact steps (see code61_x32)
  uint64_t carry = 0;
  F61 y{c.w[q * K + K - 1][0], c.w[q * K + K - 1][1]};
#pragma unroll
  for (int i = K - 2; i >= 1; --i) y = p61_step_x32_lazy(y, x, F61{c.w[q * K + i][0], c.w[q * K + i][1]}, carry);
  if (__builtin_expect(carry != 0, 0)) {
    asm volatile("");  // keeps this path a branch, not a select
    y = F61{c.w[q * K + K - 1][0], c.w[q * K + K - 1][1]};
#pragma unroll
    for (int i = K - 2; i >= 1; --i) y = p61_step_x32(y, x, F61{c.w[q * K + i][0], c.w[q * K + i][1]});
  }
  return p61_step_x32(y, x, F61{c.w[q * K][0], c.w[q * K][1]});
}

// The code (low word of the reduced hash value) of key x < 2^32 under
// polynomial q: Horner's rule (Algorithm 1) whose last step adds a_0 + 1, then
// p61_lo_from_inc in place of the final reduction.  Every step folds at bit
// 61 (p61_step_x32): exact, the path taken when a faster one saw a carry.
template <int K, int NP>
__device__ __forceinline__ uint32_t code61_x32_exact(const RowCoeffs<K, NP>& c, int q, uint32_t x) {
  F61 y{c.w[q * K + K - 1][0], c.w[q * K + K - 1][1]};
#pragma unroll
  for (int i = K - 2; i >= 1; --i) y = p61_step_x32(y, x, F61{c.w[q * K + i][0], c.w[q * K + i][1]});
  y = p61_step_x32(y, x, (uint64_t)c.w[q * K][0] + 1u, c.w[q * K][1]);
  return p61_lo_from_inc(y);
}

// The same value: the steps before the last at bit 64 (p61_step_x32_lazy, one
// instruction less each), the last one without a fold (p61_last_lo).  If any
// lane's lazy fold carried out of 64 bits, or any lane's last step is one
// p61_last_lo does not cover, the wave recomputes with the exact steps (both
// tests are wave-uniform).
template <int K, int NP>
__device__ __forceinline__ uint32_t code61_x32(const RowCoeffs<K, NP>& c, int q, uint32_t x) {
  uint64_t carry = 0;
  F61 y{c.w[q * K + K - 1][0], c.w[q * K + K - 1][1]};
#pragma unroll
  for (int i = K - 2; i >= 1; --i) y = p61_step_x32_lazy(y, x, F61{c.w[q * K + i][0], c.w[q * K + i][1]}, carry);
  uint32_t bits;
  const uint32_t code = p61_last_lo(y, x, F61{c.w[q * K][0], c.w[q * K][1]}, bits);
  if (__builtin_expect(carry != 0 || __any(bits >= kP61LastGuard), 0)) {
    // the volatile statement keeps the compiler from computing this path
    // always and selecting its result
    asm volatile("");
    return code61_x32_exact<K, NP>(c, q, x);
  }
  return code;
}

// The same for NK keys (NK even), two keys' steps interleaved (the chains are
// independent, so each fills the other's dependency stalls), with one test for
// all of them: the largest of the last steps' bits 32..60 is compared once.
template <int K, int NP, int NK, int NX>
__device__ __forceinline__ void code61_x32_tile(const RowCoeffs<K, NP>& c, int q, const uint32_t (&x)[NX],
                                                uint32_t (&code)[NK]) {
  static_assert(NK % 2 == 0 && NK <= NX, "keys are hashed in pairs, the first NK of x");
  uint64_t carry = 0;
  uint32_t top = 0;
  const F61 a0{c.w[q * K][0], c.w[q * K][1]};
  // the leading coefficient in vector registers: the first step's products
  // then take their coefficient addends from scalar registers, as the later
  // steps do, and need no copies of them
  F61 top_c;
  asm volatile("v_mov_b32 %0, %2\n\tv_mov_b32 %1, %3"
               : "=v"(top_c.w0), "=v"(top_c.w1)
               : "s"(c.w[q * K + K - 1][0]), "s"(c.w[q * K + K - 1][1]));
#pragma unroll
  for (int j = 0; j < NK; j += 2) {
    F61 ya = top_c;
    F61 yb = ya;
#pragma unroll
    for (int i = K - 2; i >= 1; --i) {
      const F61 a{c.w[q * K + i][0], c.w[q * K + i][1]};
      ya = p61_step_x32_lazy(ya, x[j], a, carry);
      yb = p61_step_x32_lazy(yb, x[j + 1], a, carry);
    }
    uint32_t ba, bb;
    code[j] = p61_last_lo(ya, x[j], a0, ba);
    code[j + 1] = p61_last_lo(yb, x[j + 1], a0, bb);
    top = max(top, max(ba, bb));
  }
  if (__builtin_expect(carry != 0 || __any(top >= kP61LastGuard), 0)) {
    asm volatile("");  // as in code61_x32
#pragma unroll
    for (int j = 0; j < NK; ++j) code[j] = code61_x32_exact<K, NP>(c, q, x[j]);
  }
}

template <int K, int NP>
__device__ __forceinline__ F61 horner61_x64(const RowCoeffs<K, NP>& c, int q, uint32_t x0, uint32_t x1) {
  F61 y{c.w[q * K + K - 1][0], c.w[q * K + K - 1][1]};
#pragma unroll
  for (int i = K - 2; i >= 0; --i) y = p61_step_x64(y, x0, x1, F61{c.w[q * K + i][0], c.w[q * K + i][1]});
  return y;
}

template <int K, int NP>
__device__ __forceinline__ uint64_t hash61_x32(const RowCoeffs<K, NP>& c, int q, uint32_t x) {
  return p61_final(horner61_x32<K, NP>(c, q, x));
}

template <int K, int NP>
__device__ __forceinline__ uint64_t hash61_x64(const RowCoeffs<K, NP>& c, int q, uint32_t x0, uint32_t x1) {
  return p61_final(horner61_x64<K, NP>(c, q, x0, x1));
}

template <int K, int NP>
__device__ __forceinline__ F89 hash89(const RowCoeffs<K, NP>& c, int q, uint32_t x0, uint32_t x1) {
  F89 y{c.w[q * K + K - 1][0], c.w[q * K + K - 1][1], c.w[q * K + K - 1][2]};
#pragma unroll
  for (int i = K - 2; i >= 0; --i)
    y = p89_step(y, x0, x1, F89{c.w[q * K + i][0], c.w[q * K + i][1], c.w[q * K + i][2]});
  return p89_final(y);
}

// The low word of the reduced hash value of key (x0, x1) over 2^89 - 1, as
// code61_x32: the last Horner step unfolded (p89_last_lo); if any lane's last
// step is one that does not cover, the wave takes that step with the fold
// (adding a_0 + 1, then p89_lo_from_inc).
template <int K, int NP>
__device__ __forceinline__ uint32_t code89(const RowCoeffs<K, NP>& c, int q, uint32_t x0, uint32_t x1) {
  F89 y{c.w[q * K + K - 1][0], c.w[q * K + K - 1][1], c.w[q * K + K - 1][2]};
#pragma unroll
  for (int i = K - 2; i >= 1; --i)
    y = p89_step(y, x0, x1, F89{c.w[q * K + i][0], c.w[q * K + i][1], c.w[q * K + i][2]});
  const F89 a0{c.w[q * K][0], c.w[q * K][1], c.w[q * K][2]};
  uint32_t bits;
  const uint32_t code = p89_last_lo(y, x0, x1, a0, bits);
  if (__builtin_expect(__any(bits >= kP89LastGuard), 0)) {
    asm volatile("");  // as in code61_x32
    return p89_lo_from_inc(p89_step(y, x0, x1, a0, (uint64_t)a0.w0 + 1u));
  }
  return code;
}

// code89 for NK keys with one guard test: the steps before the last are kept
// per key, so a wave with a lane at the guard only redoes the last step.
template <int K, int NP, int NK>
__device__ __forceinline__ void code89_tile(const RowCoeffs<K, NP>& c, int q, const uint32_t (&x0)[NK],
                                            const uint32_t (&x1)[NK], uint32_t (&code)[NK]) {
  const F89 a0{c.w[q * K][0], c.w[q * K][1], c.w[q * K][2]};
  F89 y[NK];
  uint32_t top = 0;
#pragma unroll
  for (int j = 0; j < NK; ++j) {
    y[j] = F89{c.w[q * K + K - 1][0], c.w[q * K + K - 1][1], c.w[q * K + K - 1][2]};
#pragma unroll
    for (int i = K - 2; i >= 1; --i)
      y[j] = p89_step(y[j], x0[j], x1[j], F89{c.w[q * K + i][0], c.w[q * K + i][1], c.w[q * K + i][2]});
    uint32_t bits;
    code[j] = p89_last_lo(y[j], x0[j], x1[j], a0, bits);
    top = max(top, bits);
  }
  if (__builtin_expect(__any(top >= kP89LastGuard), 0)) {
    asm volatile("");  // as in code61_x32
#pragma unroll
    for (int j = 0; j < NK; ++j) code[j] = p89_lo_from_inc(p89_step(y[j], x0[j], x1[j], a0, (uint64_t)a0.w0 + 1u));
  }
}

// Bucket and sign bit of key (x0, x1) under a row's coefficients.  WIDE
// selects the two-limb key path for p61.
template <int PRIME, int MODE, int K, bool WIDE, int NP>
__device__ __forceinline__ void bucket_sign(const RowCoeffs<K, NP>& c, uint32_t x0, uint32_t x1, uint32_t log2m,
                                            uint32_t& bucket, uint32_t& a) {
  const uint32_t mask = (1u << log2m) - 1u;
  if constexpr (PRIME == kPrime61 && !WIDE && (MODE == kTwoForOne || MODE == kTwoPoly)) {
    // these splits read only low bits of the hash values
    const uint32_t h = code61_x32<K, NP>(c, 0, x0);
    if constexpr (MODE == kTwoForOne) {
      a = h & 1u;
      bucket = (h >> 1) & mask;
    } else {
      a = code61_x32<K, NP>(c, 1, x0) & 1u;
      bucket = h & mask;
    }
  } else if constexpr (PRIME == kPrime61) {
    uint64_t h = WIDE ? hash61_x64<K, NP>(c, 0, x0, x1) : hash61_x32<K, NP>(c, 0, x0);
    if constexpr (MODE == kTwoForOne) {
      a = (uint32_t)h & 1u;
      bucket = ((uint32_t)h >> 1) & mask;
    } else if constexpr (MODE == kTwoForOneMsb) {
      a = (uint32_t)(h >> 60) & 1u;
      bucket = (uint32_t)h & mask;
    } else if constexpr (MODE == kArbR) {
      // Algorithm 8: h+1 (never 0), its low 60 bits j scaled into [r] by
      // floor(r j / 2^60), its bit 60 the sign bit.  r < 2^32 and j < 2^60: the
      // 92-bit product is built from two 32x32 products.
      const uint64_t hx = h + 1;
      a = (uint32_t)(hx >> 60);
      const uint64_t j = hx & ((1ull << 60) - 1);
      const uint64_t lo = (uint64_t)(uint32_t)j * c.r;
      const uint64_t hi = (j >> 32) * c.r + (lo >> 32);
      bucket = (uint32_t)(hi >> 28);
    } else {
      uint64_t h2 = WIDE ? hash61_x64<K, NP>(c, 1, x0, x1) : hash61_x32<K, NP>(c, 1, x0);
      a = (uint32_t)h2 & 1u;
      bucket = (uint32_t)h & mask;
    }
  } else if constexpr (MODE == kTwoForOne || MODE == kTwoPoly) {
    // over 2^89 - 1 too these splits read only the low words
    const uint32_t h = code89<K, NP>(c, 0, x0, x1);
    if constexpr (MODE == kTwoForOne) {
      a = h & 1u;
      bucket = (h >> 1) & mask;
    } else {
      a = code89<K, NP>(c, 1, x0, x1) & 1u;
      bucket = h & mask;
    }
  } else {
    F89 h = hash89<K, NP>(c, 0, x0, x1);
    if constexpr (MODE == kTwoForOneMsb) {
      a = (h.w2 >> 24) & 1u;
      bucket = h.w0 & mask;
    } else {  // kArbR
      // Algorithm 8 with b = 89: h+1 in 32-bit limbs, sign bit 88, and
      // floor(r j / 2^88) for the low 88 bits j (three 32x32 products).
      const uint64_t s0 = (uint64_t)h.w0 + 1u;
      const uint64_t s1 = (uint64_t)h.w1 + (s0 >> 32);
      const uint32_t x2 = h.w2 + (uint32_t)(s1 >> 32);
      a = (x2 >> 24) & 1u;
      const uint64_t t0 = (uint64_t)(uint32_t)s0 * c.r;
      const uint64_t t1 = (uint64_t)(uint32_t)s1 * c.r + (t0 >> 32);
      const uint64_t t2 = (uint64_t)(x2 & 0xFFFFFFu) * c.r + (t1 >> 32);
      bucket = (uint32_t)(t2 >> 24);
    }
  }
}

// Bucket and sign bit packed as code = bucket << 1 | a (bits above bit log2m
// unspecified).  With the low-bit split of Algorithm 3 the reduced hash value
// already has this layout, so its low word is the code.
template <int PRIME, int MODE, int K, bool WIDE, int NP>
__device__ __forceinline__ uint32_t bucket_code(const RowCoeffs<K, NP>& c, uint32_t x0, uint32_t x1, uint32_t log2m) {
  if constexpr (PRIME == kPrime61 && MODE == kTwoForOne) {
    if constexpr (WIDE)
      return p61_final_lo(horner61_x64<K, NP>(c, 0, x0, x1));
    else
      return code61_x32<K, NP>(c, 0, x0);
  } else if constexpr (PRIME == kPrime89 && MODE == kTwoForOne) {
    return code89<K, NP>(c, 0, x0, x1);
  } else if constexpr (PRIME == kPrime61 && MODE == kTwoPoly && !WIDE) {
    // bucket from h1's low bits, sign from bit 0 of h2; bits above the bucket
    // may hold anything
    return (code61_x32<K, NP>(c, 0, x0) << 1) | (code61_x32<K, NP>(c, 1, x0) & 1u);
  } else {
    uint32_t bk, a;
    bucket_sign<PRIME, MODE, K, WIDE, NP>(c, x0, x1, log2m, bk, a);
    return (bk << 1) | a;
  }
}

// Bucket and sign mask (0 or all ones) of a key: from the code for the
// low-bit split, where the code is the hash's low word, else directly.
template <int PRIME, int MODE, int K, bool WIDE, int NP>
__device__ __forceinline__ void bucket_mask(const RowCoeffs<K, NP>& c, uint32_t x0, uint32_t x1, uint32_t log2m,
                                            uint32_t& bucket, uint32_t& m) {
  if constexpr (MODE == kTwoForOne) {
    const uint32_t code = bucket_code<PRIME, MODE, K, WIDE, NP>(c, x0, x1, log2m);
    bucket = __builtin_amdgcn_ubfe(code, 1u, log2m);
    m = (uint32_t)__builtin_amdgcn_sbfe((int)code, 0, 1);
  } else {
    uint32_t a;
    bucket_sign<PRIME, MODE, K, WIDE, NP>(c, x0, x1, log2m, bucket, a);
    m = 0u - a;
  }
}

template <typename KeyT>
__device__ __forceinline__ void load_key(const KeyT* __restrict__ keys, uint64_t i, uint32_t& x0, uint32_t& x1) {
  if constexpr (sizeof(KeyT) == 4) {
    x0 = keys[i];
    x1 = 0;
  } else {
    uint64_t v = keys[i];
    x0 = (uint32_t)v;
    x1 = (uint32_t)(v >> 32);
  }
}

template <typename WT>
__device__ __forceinline__ int64_t load_weight(const WT* __restrict__ w, uint64_t i) {
  return (int64_t)w[i];
}

// Keys and weights at positions base + j * stride + tid, j < kKpt.  A position
// at or past `end` (end > base) loads position end - 1 instead and comes back
// with ok = false (its key and weight are that position's, so every use must
// test ok): the loads have no branches and no value is used before all of
// them are issued.
template <int kKpt, typename KeyT, typename WT>
__device__ __forceinline__ void load_tile(const KeyT* __restrict__ keys, const WT* __restrict__ weights, uint64_t base,
                                          uint32_t stride, uint32_t tid, uint64_t end, uint32_t (&x0)[kKpt],
                                          uint32_t (&x1)[kKpt], int64_t (&wv)[kKpt], bool (&ok)[kKpt]) {
  KeyT kr[kKpt];
  WT wr[kKpt];
#pragma unroll
  for (int j = 0; j < kKpt; ++j) {
    const uint64_t i = base + (uint64_t)j * stride + tid;
    ok[j] = i < end;
    const uint64_t at = ok[j] ? i : end - 1;
    kr[j] = keys[at];
    wr[j] = weights[at];
  }
  // Keep the scheduler from moving uses of the first loads between the others;
  // the empty statements stop the weights' widening from being fused into
  // their loads (it would then sit next to each load and wait for it).
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int j = 0; j < kKpt; ++j) asm volatile("" : "+v"(wr[j]));
#pragma unroll
  for (int j = 0; j < kKpt; ++j) {
    const uint64_t k = (uint64_t)kr[j];
    x0[j] = (uint32_t)k;
    x1[j] = (uint32_t)(k >> 32);
    wv[j] = (int64_t)wr[j];
  }
}

// Issues the loads of keys and weights at kp[j * 64], wp[j * 64], j < kKpt (all
// in range): one base address per array and immediate offsets.  The values
// are used later (tile_unpack), so the loads stay in flight meanwhile.
template <int kKpt, typename KeyT, typename WT>
__device__ __forceinline__ void tile_issue(const KeyT* __restrict__ kp, const WT* __restrict__ wp, KeyT (&kr)[kKpt],
                                           WT (&wr)[kKpt]) {
#pragma unroll
  for (int j = 0; j < kKpt; ++j) {
    kr[j] = kp[j * 64];
    wr[j] = wp[j * 64];
  }
}

// Splits loaded keys into 32-bit limbs and weights into 32 bits.  big: some
// weight does not fit 32 bits (never, for 32-bit weights); any_hi: the
// largest of the keys' high words (zero iff every key has one limb; its bits
// from 28 on tell a key >= 2^60).  A maximum, not an or: the compiler turns
// an or of high words into an or of whole keys and a compare, twice the
// instructions.
template <int kKpt, typename KeyT, typename WT>
__device__ __forceinline__ void tile_unpack(const KeyT (&kr)[kKpt], const WT (&wr)[kKpt], uint32_t (&x0)[kKpt],
                                            uint32_t (&x1)[kKpt], int32_t (&wf)[kKpt], bool& big, uint32_t& any_hi) {
#pragma unroll
  for (int j = 0; j < kKpt; ++j) {
    const uint64_t k = (uint64_t)kr[j];
    x0[j] = (uint32_t)k;
    x1[j] = (uint32_t)(k >> 32);
    any_hi = x1[j] > any_hi ? x1[j] : any_hi;
    if constexpr (sizeof(WT) == 8) big |= (int64_t)(int32_t)wr[j] != (int64_t)wr[j];
    wf[j] = (int32_t)wr[j];
  }
}

__device__ __forceinline__ unsigned long long signed_weight(int64_t w, uint32_t a) {
  return (unsigned long long)(a ? -w : w);
}

// s*w for a sign mask m (0 for s = 1, all ones for s = -1), given w and
// wd = w ^ -w: w ^ (wd & m).
__device__ __forceinline__ unsigned long long masked_signed(uint32_t m, int64_t w, uint64_t wd) {
  const uint64_t wp = (uint64_t)w;
  const uint32_t lo = (uint32_t)wp ^ ((uint32_t)wd & m);
  const uint32_t hi = (uint32_t)(wp >> 32) ^ ((uint32_t)(wd >> 32) & m);
  return ((unsigned long long)hi << 32) | lo;
}

// ---------------------------------------------------------------------------
// Single pass with the whole table in LDS.  Each block zeroes its private
// table, processes a contiguous key range, then adds the non-zero partial
// counters into the global table with coalesced int64 atomics.
// ---------------------------------------------------------------------------
// Zero the block's LDS table, add keys [begin, end) of `args` into it, then add
// its non-zero counters into args.table.  Used by the single-sketch and the
// batched kernels.
template <int PRIME, int MODE, int K, typename KeyT, typename WT>
__device__ __forceinline__ void lds_block_update(const UpdateArgs<KeyT, WT>& args, uint64_t begin, uint64_t end,
                                                 unsigned long long* lds) {
  const uint32_t cells = args.rows << args.log2m;
  for (uint32_t i = threadIdx.x; i < cells; i += kBlock) lds[i] = 0;
  __syncthreads();
  constexpr int kKpt = kKeysPerThread;
  constexpr int NP = MODE == kTwoPoly ? 2 : 1;
  uint32_t bad = 0;

  for (uint64_t base = begin; base < end; base += (uint64_t)kBlock * kKpt) {
    uint32_t x0[kKpt], x1[kKpt];
    int64_t wv[kKpt];
    bool ok[kKpt];
    load_tile<kKpt>(args.keys, args.weights, base, kBlock, threadIdx.x, end, x0, x1, wv, ok);
    uint32_t any_hi = 0;
#pragma unroll
    for (int j = 0; j < kKpt; ++j) any_hi |= x1[j];
    if constexpr (PRIME == kPrime61) bad |= any_hi >> 28;  // key >= 2^60 breaks p >= 2u - 1
    // wave-uniform choice of the one-limb key path (all keys < 2^32)
    const bool wide = PRIME == kPrime61 && sizeof(KeyT) == 8 && __any(any_hi != 0);
    // w ^ -w of each weight, so a row applies the sign with bit operations
    uint64_t wneg[kKpt];
#pragma unroll
    for (int j = 0; j < kKpt; ++j) wneg[j] = (uint64_t)wv[j] ^ (uint64_t)(-wv[j]);
    for (uint32_t r = 0; r < args.rows; ++r) {
      const auto c = load_row_coeffs<K, NP>(args.coeffs + (size_t)r * NP * K);
      unsigned long long* row = lds + ((size_t)r << args.log2m);
      if (wide) {
#pragma unroll
        for (int j = 0; j < kKpt; ++j) {
          uint32_t bk, m;
          bucket_mask<PRIME, MODE, K, true, NP>(c, x0[j], x1[j], args.log2m, bk, m);
          if (ok[j]) atomicAdd(&row[bk], masked_signed(m, wv[j], wneg[j]));
        }
      } else if constexpr (PRIME == kPrime61 && MODE == kTwoForOne && kKpt % 2 == 0) {
        // the low-bit split: the codes of the lane's keys with one guard test
        uint32_t code[kKpt];
        code61_x32_tile<K, NP, kKpt>(c, 0, x0, code);
#pragma unroll
        for (int j = 0; j < kKpt; ++j) {
          const uint32_t bk = __builtin_amdgcn_ubfe(code[j], 1u, args.log2m);
          const uint32_t m = (uint32_t)__builtin_amdgcn_sbfe((int)code[j], 0, 1);
          if (ok[j]) atomicAdd(&row[bk], masked_signed(m, wv[j], wneg[j]));
        }
      } else {
#pragma unroll
        for (int j = 0; j < kKpt; ++j) {
          uint32_t bk, m;
          bucket_mask<PRIME, MODE, K, false, NP>(c, x0[j], x1[j], args.log2m, bk, m);
          if (ok[j]) atomicAdd(&row[bk], masked_signed(m, wv[j], wneg[j]));
        }
      }
    }
  }
  if (bad) atomicOr(args.flags, kFlagDomain);
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < cells; i += kBlock) {
    unsigned long long v = lds[i];
    if (v) atomicAdd(&args.table[i], v);
  }
}

template <int PRIME, int MODE, int K, typename KeyT, typename WT>
__global__ __launch_bounds__(kBlock) void k_update_lds(UpdateArgs<KeyT, WT> args) {
  extern __shared__ unsigned long long lds[];
  const uint64_t begin = (uint64_t)blockIdx.x * args.keys_per_block;
  const uint64_t end = min(args.n, begin + args.keys_per_block);
  lds_block_update<PRIME, MODE, K, KeyT, WT>(args, begin, end, lds);
}

// ---------------------------------------------------------------------------
// Table in global memory, one device-scope int64 atomic per (key, row).
// ---------------------------------------------------------------------------
template <int PRIME, int MODE, int K, typename KeyT, typename WT>
__device__ __forceinline__ void global_block_update(const UpdateArgs<KeyT, WT>& args, uint64_t begin, uint64_t end) {
  constexpr int kKpt = kKeysPerThread;
  constexpr int NP = MODE == kTwoPoly ? 2 : 1;
  uint32_t bad = 0;
  for (uint64_t base = begin; base < end; base += (uint64_t)kBlock * kKpt) {
    uint32_t x0[kKpt], x1[kKpt];
    int64_t wv[kKpt];
    bool ok[kKpt];
    load_tile<kKpt>(args.keys, args.weights, base, kBlock, threadIdx.x, end, x0, x1, wv, ok);
    uint32_t any_hi = 0;
#pragma unroll
    for (int j = 0; j < kKpt; ++j) any_hi |= x1[j];
    if constexpr (PRIME == kPrime61) bad |= any_hi >> 28;
    const bool wide = PRIME == kPrime61 && sizeof(KeyT) == 8 && __any(any_hi != 0);
    for (uint32_t r = 0; r < args.rows; ++r) {
      const auto c = load_row_coeffs<K, NP>(args.coeffs + (size_t)r * NP * K);
      unsigned long long* row = args.table + ((size_t)r << args.log2m);
#pragma unroll
      for (int j = 0; j < kKpt; ++j) {
        uint32_t bk, a;
        if (wide)
          bucket_sign<PRIME, MODE, K, true, NP>(c, x0[j], x1[j], args.log2m, bk, a);
        else
          bucket_sign<PRIME, MODE, K, false, NP>(c, x0[j], x1[j], args.log2m, bk, a);
        if (ok[j]) atomicAdd(&row[bk], signed_weight(wv[j], a));
      }
    }
  }
  if (bad) atomicOr(args.flags, kFlagDomain);
}

template <int PRIME, int MODE, int K, typename KeyT, typename WT>
__global__ __launch_bounds__(kBlock) void k_update_global(UpdateArgs<KeyT, WT> args) {
  const uint64_t begin = (uint64_t)blockIdx.x * args.keys_per_block;
  const uint64_t end = min(args.n, begin + args.keys_per_block);
  global_block_update<PRIME, MODE, K, KeyT, WT>(args, begin, end);
}

// ---------------------------------------------------------------------------
// Row-resident update for tables of up to 2^16 buckets per row (a row of
// 16-bit fields is at most 128 KiB of LDS).
//
// A block holds the counters of one row group (rpg rows) as 16-bit fields,
// two per 32-bit LDS word: bucket 2i in the low half of word i, bucket 2i+1 in
// the high half, each holding its running sum plus 2^15.  The blocks of a
// group split the key tiles among themselves and hash every key for the
// group's rows only, so each (key, row) is hashed once (Algorithm 2, Process)
// and nothing is written per key.  A tile is read once per group: from HBM by
// the first group to reach it, from L2 or the last-level cache by the others.
//
// Every add is a 32-bit LDS atomic that returns the old word.  A field whose
// biased value leaves [0, 2^16) wraps, and the add that wrapped it sees so in
// the old word; it then adds what the fields lost to the global int64
// counters with device-scope atomics: +-2^16 on its own bucket and, for a low
// field, the carry c that went into the high half (-c on the high bucket,
// +-2^16 more if that carry wrapped the high half out of the word).  A field
// must drift 2^15 from its bias to wrap, so these adds are rare for small
// weights; a weight of 2^15 or more always wraps its field and takes that
// path, which is exact for every 32-bit weight (the LDS add is exact modulo
// 2^32 and the carried multiples of 2^16 are taken in 64 bits).  At the end
// each block adds field - 2^15 of every non-zero field into the global
// counters.  Every step is an integer add, so the counters are exact in any
// order.  64-bit weights that do not fit 32 bits skip the fields and go to
// the global counters directly.
// ---------------------------------------------------------------------------
// The rows of a row group for one wave's keys: hash, add each s*w into its
// field, carry wraps into the global counters.  ESC: some keys have weights
// that bypass the fields (esc[j]); without ESC every wf[j] is the key's weight.
// One row (local index r of the block's group, global index row, coefficients
// c) for one wave's keys.  ROW0: r is 0 (the block's group is one row), so the
// LDS address is the code's bucket bits alone.
template <int PRIME, int MODE, int K, int NP, bool WIDE, bool ESC, int NK, bool ROW0 = false, typename KeyT,
          typename WT>
__device__ __forceinline__ void row_update(const RowArgs<KeyT, WT>& args, const RowCoeffs<K, NP>& c, uint32_t row,
                                           uint32_t r, uint32_t* words, const uint32_t (&x0)[NK],
                                           const uint32_t (&x1)[NK], const int32_t (&wf)[NK],
                                           const int64_t* wv, const bool* esc, bool any_esc) {
  const uint32_t m = 1u << args.log2m;
  const uint32_t amask = 2u * m - 4u;  // byte offset of a bucket's word in its row: code & amask
  {
    // byte offset of the row in LDS, a multiple of 2m, or-ed onto code & amask;
    // kept in a vector register so that the and-or takes one instruction
    uint32_t rowoff = 0;
    if (!ROW0) asm volatile("v_mov_b32 %0, %1" : "=v"(rowoff) : "s"(r * 2u * m));
    uint32_t code[NK], old[NK], sh[NK];
    int32_t sw[NK];
    if constexpr (PRIME == kPrime61 && MODE == kTwoForOne && !WIDE && NK % 2 == 0) {
      // the low-bit split: the code is the low word of the reduced hash
      code61_x32_tile<K, NP, NK>(c, 0, x0, code);
    } else if constexpr (PRIME == kPrime61 && MODE == kTwoPoly && !WIDE && NK % 2 == 0) {
      // two polynomials: bucket from the first's low word, sign from the
      // second's bit 0 (bucket_code's layout), each with one guard test
      uint32_t sg[NK];
      code61_x32_tile<K, NP, NK>(c, 0, x0, code);
      code61_x32_tile<K, NP, NK>(c, 1, x0, sg);
#pragma unroll
      for (int j = 0; j < NK; ++j) code[j] = (code[j] << 1) | (sg[j] & 1u);
    } else {
#pragma unroll
      for (int j = 0; j < NK; ++j) code[j] = bucket_code<PRIME, MODE, K, WIDE, NP>(c, x0[j], x1[j], args.log2m);
    }
#pragma unroll
    for (int j = 0; j < NK; ++j) {
      // s * w with s = 1 - 2a, a = bit 0 of the code; the field's half is bit 0
      // of the bucket (bit 1 of the code)
      const int32_t sgn = __builtin_amdgcn_sbfe((int)code[j], 0, 1);
      sw[j] = (wf[j] ^ sgn) - sgn;
      sh[j] = (code[j] & 2u) << 3;
      old[j] = atomicAdd((uint32_t*)((unsigned char*)words + ((code[j] & amask) | rowoff)), (uint32_t)sw[j] << sh[j]);
    }
    // The field wrapped iff its old value plus s*w leaves [0, 2^16).  Taken in
    // 32 bits this test is exact for every 32-bit weight: the true sum lies in
    // [-2^31, 2^31 + 2^16), and no value there outside [0, 2^16) is congruent
    // modulo 2^32 to one inside.
    bool wr[NK];
    bool any_wr = false;
#pragma unroll
    for (int j = 0; j < NK; ++j) {
      const int32_t t = (int32_t)__builtin_amdgcn_ubfe(old[j], sh[j], 16u) + sw[j];
      wr[j] = (uint32_t)t > 0xFFFFu;
      any_wr |= wr[j];
    }
    unsigned long long* const grow = args.table + ((size_t)row << args.log2m);
    if (__any(any_wr)) {
#pragma unroll
      for (int j = 0; j < NK; ++j)
        if (wr[j]) {
          // In 64 bits: s*w is 2^31 for w = -2^31, and a weight of many times
          // 2^16 moves the field by many multiples of 2^16.  The 32-bit add in
          // LDS was exact modulo 2^32, so the field (and, for the low half,
          // the high half above it) now holds the sum modulo 2^16; cw
          // multiples of 2^16 went missing from the field (floor division),
          // and for the low half they went into the high half instead.
          const uint32_t bucket = (code[j] >> 1) & (m - 1u);
          // s*w from the 32-bit sw: only s = -1, w = -2^31 gives 2^31, which
          // 32 bits hold as -2^31
          const int64_t swl = (code[j] & 1u) && sw[j] == INT32_MIN ? (int64_t)1 << 31 : (int64_t)sw[j];
          const int64_t t = (int64_t)__builtin_amdgcn_ubfe(old[j], sh[j], 16u) + swl;
          const int64_t cw = t >> 16;
          atomicAdd(&grow[bucket], (unsigned long long)(cw * 65536));
          if (sh[j] == 0) {  // the high half received cw and lost e multiples of 2^16
            const int64_t e = ((int64_t)(old[j] >> 16) + cw) >> 16;
            atomicAdd(&grow[bucket + 1], (unsigned long long)(e * 65536 - cw));
          }
        }
    }
    if (ESC && any_esc) {
#pragma unroll
      for (int j = 0; j < NK; ++j)
        if (esc[j]) {
          const uint32_t bucket = (code[j] >> 1) & (m - 1u);
          atomicAdd(&grow[bucket], signed_weight(wv[j], code[j] & 1u));
        }
    }
  }
}

// The rows of the block's group for one wave's keys.
template <int PRIME, int MODE, int K, int NP, bool WIDE, bool ESC, int NK, typename KeyT, typename WT>
__device__ __forceinline__ void rows_tile(const RowArgs<KeyT, WT>& args, uint32_t r0, uint32_t* words,
                                          const uint32_t (&x0)[NK], const uint32_t (&x1)[NK],
                                          const int32_t (&wf)[NK], const int64_t* wv, const bool* esc,
                                          bool any_esc) {
  for (uint32_t r = 0; r < args.rpg; ++r) {
    const auto c = load_row_coeffs<K, NP>(args.coeffs + (size_t)(r0 + r) * NP * K);
    row_update<PRIME, MODE, K, NP, WIDE, ESC, NK>(args, c, r0 + r, r, words, x0, x1, wf, wv, esc, any_esc);
  }
}

// A wave tile (64 * KPT keys from `base`) of the rows of the block's group in
// the general way: positions past n, weights that bypass the fields, keys of
// two limbs; in two halves of KPT / 2 keys per lane, so that it needs few
// registers.  Returns domain-error bits.
template <int PRIME, int MODE, int K, int NP, int KPT, typename KeyT, typename WT>
__device__ __forceinline__ uint32_t rows_wave_tile_slow(const RowArgs<KeyT, WT>& args, uint32_t r0, uint32_t* words,
                                                        uint64_t base, uint32_t lane) {
  constexpr int NK = KPT / 2;
  uint32_t bad = 0;
  for (uint32_t h = 0; h < 2; ++h) {
    const uint64_t hb = base + h * 64 * NK;
    if (hb >= args.n) break;
    uint32_t x0[NK], x1[NK];
    int64_t wv[NK];
    bool ok[NK];
    int32_t wf[NK];
    bool esc[NK];
    load_tile<NK>(args.keys, args.weights, hb, 64, lane, args.n, x0, x1, wv, ok);
    uint32_t any_hi = 0;
    bool any_e = false;
#pragma unroll
    for (int j = 0; j < NK; ++j) {
      any_hi |= x1[j];
      const bool fits = wv[j] == (int64_t)(int32_t)wv[j];
      wf[j] = ok[j] && fits ? (int32_t)wv[j] : 0;  // positions past n add 0
      esc[j] = ok[j] && !fits;
      any_e |= esc[j];
    }
    if constexpr (PRIME == kPrime61) bad |= any_hi >> 28;  // key >= 2^60 breaks p >= 2u - 1
    const bool any_esc = __any(any_e);
    if (PRIME == kPrime61 && sizeof(KeyT) == 8 && __any(any_hi != 0))
      rows_tile<PRIME, MODE, K, NP, true, true, NK>(args, r0, words, x0, x1, wf, wv, esc, any_esc);
    else
      rows_tile<PRIME, MODE, K, NP, false, true, NK>(args, r0, words, x0, x1, wf, wv, esc, any_esc);
  }
  return bad;
}

// One wave tile `wt` (64 * KPT keys, loaded into kk, ww when the tile is full:
// `full`, the same for all lanes) of the rows of the block's group (first row
// r0; c1 holds row r0's coefficients, used when the group is that one row).
// Common case: a full tile whose keys have one limb (p61) and whose weights fit
// the fields; the rest goes to the general path.  Returns domain-error bits.
template <int PRIME, int MODE, int K, int NP, int KPT, typename KeyT, typename WT>
__device__ __forceinline__ uint32_t rows_wave_tile(const RowArgs<KeyT, WT>& args, const RowCoeffs<K, NP>& c1, bool one,
                                                   uint32_t r0, uint32_t* words, uint64_t wt, bool full,
                                                   const KeyT (&kk)[KPT], const WT (&ww)[KPT], uint32_t lane) {
  constexpr uint64_t kWt = 64 * KPT;
  uint32_t bad = 0;
  if (full) {
    uint32_t x0[KPT], x1[KPT];
    int32_t wf[KPT];
    bool big = false;
    uint32_t any_hi = 0;
    tile_unpack<KPT>(kk, ww, x0, x1, wf, big, any_hi);
    if constexpr (PRIME == kPrime61) bad |= any_hi >> 28;  // key >= 2^60 breaks p >= 2u - 1
    const bool two_limb = PRIME == kPrime61 && sizeof(KeyT) == 8 && __any(any_hi != 0);
    if (!two_limb && !__any(big)) {
      if constexpr (PRIME == kPrime61) {
#pragma unroll
        for (int j = 0; j < KPT; ++j) x1[j] = 0;  // the one-limb hash reads no high words
      }
      if (one)
        row_update<PRIME, MODE, K, NP, false, false, KPT, true>(args, c1, r0, 0, words, x0, x1, wf, nullptr, nullptr,
                                                          false);
      else
        rows_tile<PRIME, MODE, K, NP, false, false, KPT>(args, r0, words, x0, x1, wf, nullptr, nullptr, false);
      return bad;
    }
  }
  return bad | rows_wave_tile_slow<PRIME, MODE, K, NP, KPT, KeyT, WT>(args, r0, words, wt * kWt, lane);
}

// Adds field - 2^15 of every non-zero field of the block's group (rpg rows
// from row r0, nwords LDS words) into the global counters.  The group's rows
// are contiguous in the table, so field c of the group (the low or high half
// of word c / 2) is counter (r0 << log2m) + c: lane l of a wave adds counter
// base + l, and one atomic instruction covers 64 consecutive counters (eight
// 64-byte lines).  Blocks of one group flush at about the same time into the
// same counters; block `rank` of `ranks` starts its pass at its own fraction
// of the fields.
template <typename KeyT, typename WT>
__device__ __forceinline__ void rows_flush(const RowArgs<KeyT, WT>& args, uint32_t r0, const uint32_t* words,
                                           uint32_t nwords, uint32_t rank, uint32_t ranks) {
  const uint32_t nf = 2u * nwords;
  const uint32_t start = (uint32_t)(((uint64_t)nf * (rank % ranks) / ranks) & ~63ull);
  unsigned long long* const base = args.table + ((size_t)r0 << args.log2m);
  for (uint32_t k = threadIdx.x; k < nf; k += kRowBlock) {
    const uint32_t c = k + start < nf ? k + start : k + start - nf;
    const int32_t v = (int32_t)((words[c >> 1] >> ((c & 1u) << 4)) & 0xFFFFu) - 32768;
    if (v) atomicAdd(base + c, (unsigned long long)(long long)v);
  }
}

// atomicAdd(p, v) whose result is waited for only where it is used.  With a
// uniform address the compiler's atomic optimizer rewrites an atomic into one
// per wave whose old value is broadcast to the lanes at once, which waits for
// the round trip right there; an address the compiler cannot prove uniform
// (p plus a zero it cannot see) keeps the atomic as written, so the value can
// be taken ahead of its use.
__device__ __forceinline__ uint32_t atomic_add_ahead(uint32_t* p, uint32_t v) {
  uint32_t zero;
  asm volatile("v_mov_b32 %0, 0" : "=v"(zero));
  return atomicAdd(p + zero, v);
}

// The wave tiles are cut into contiguous ranges, one per XCD plus a pool, and
// every (range, row group) pair has a queue: a counter of taken chunks of
// kRowChunk wave tiles.  A wave takes chunks for its block's group from its
// home range first, then from the others in turn until all are empty; every
// wave tile of every group is taken exactly once (the counters are zero at
// launch) and no wave waits for another.
//
// The groups read each tile through the L2 of the XCD whose range holds it,
// and a tile stays there only while the groups pass it at about the same
// time, so every XCD gets the same number of blocks per group: with
// range_blocks > 0, block b counts as block b / xcds of XCD b mod xcds (the
// hardware's round-robin placement), the first range_blocks of each XCD
// take group j mod groups and the XCD's range (the XCD they actually run on,
// read from the hardware), and the rest take groups in turn and the pool,
// which holds the pool blocks' share of the tiles.  Without it (few blocks)
// block b takes group b mod groups and there is no pool.  Either way every
// group has a block, so every queue is drained.
template <int PRIME, int MODE, int K, typename KeyT, typename WT>
__global__ __launch_bounds__(kRowBlock) void k_update_rows(RowArgs<KeyT, WT> args) {
  // static, so that LDS addresses need no base: one block per CU holds it all
  __shared__ __align__(16) uint32_t words[kRowLdsBytes / 4];

  constexpr int NP = MODE == kTwoPoly ? 2 : 1;
  const uint32_t G = args.groups;
  const uint32_t X = args.xcds;
  uint32_t xcc;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(xcc));
  const uint32_t RB = args.range_blocks;
  const uint32_t per_xcd = gridDim.x / X, j = blockIdx.x / X;
  const bool pool_block = RB && j >= RB;
  const uint32_t g = !RB ? blockIdx.x % G
                     : j < RB ? j % G
                              : ((blockIdx.x % X) * (per_xcd - RB) + (j - RB)) % G;
  const uint32_t NR = RB && per_xcd > RB ? X + 1 : X;  // ranges: the XCDs' and the pool
  const uint32_t home = pool_block ? X : (xcc & 15u) % X;
  const uint32_t r0 = g * args.rpg;
  const uint32_t nwords = args.rpg << (args.log2m - 1);
  for (uint32_t i = threadIdx.x; i < nwords; i += kRowBlock) words[i] = 0x80008000u;
  __syncthreads();
  const uint32_t lane = threadIdx.x & 63;
  // wave tiles (at most 2^40 keys per launch: fewer than 2^31) and the full ones
  // among them; 32-bit tile indices keep the loop's tests in scalar compares
  const uint32_t W = (uint32_t)((args.n + 64 * kRowKpt - 1) / (64 * kRowKpt));
  const uint32_t Wfull = (uint32_t)(args.n / (64 * kRowKpt));
  // the XCD ranges end where the pool begins: the pool blocks' share of the tiles
  const uint32_t Wx = NR > X ? (uint32_t)((uint64_t)W * RB / per_xcd) : W;
  uint32_t bad = 0;
  // a group of one row keeps that row's coefficients for the whole launch
  const auto c1 = load_row_coeffs<K, NP>(args.coeffs + (size_t)r0 * NP * K);
  const bool one = args.rpg == 1;
  constexpr uint64_t kWt = 64 * kRowKpt;  // keys per wave tile
  for (uint32_t k = 0; k < NR; ++k) {
    const uint32_t x = home + k < NR ? home + k : home + k - NR;
    const uint32_t lo = x < X ? (uint32_t)((uint64_t)Wx * x / X) : Wx;
    const uint32_t hi = x < X ? (uint32_t)((uint64_t)Wx * (x + 1) / X) : W;
    uint32_t* const q = args.queues + x * G + g;
    if (k > 0) {
      // Another XCD's range: most are drained by the time a wave gets here.
      // A counter only grows during the launch, so a plain read that already
      // shows the range drained needs no atomic (the atomics of one counter
      // are served one after another; thousands of waves probing every range
      // with them cost more than the hashing of a small update).
      uint32_t seen = 0;
      if (lane == 0) seen = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (__builtin_amdgcn_readfirstlane(seen) * kRowChunk >= hi - lo) continue;
    }
    // the next chunk is taken before the current one is processed, so the
    // atomic's round trip overlaps the hashing
    uint32_t next = 0;
    if (lane == 0) next = atomic_add_ahead(q, 1u);
    for (;;) {
      const uint32_t c = __builtin_amdgcn_readfirstlane(next);
      // 32 bits hold c * kRowChunk: a counter passes the range's chunks by at
      // most one per wave (each takes one chunk too many)
      if (c * kRowChunk >= hi - lo) break;
      const uint32_t wt0 = lo + c * kRowChunk;
      if (lane == 0) next = atomic_add_ahead(q, 1u);
      const uint32_t wt1 = hi - wt0 > kRowChunk ? wt0 + kRowChunk : hi;
      for (uint32_t wt = wt0; wt < wt1; ++wt) {
        KeyT ka[kRowKpt];
        WT wa[kRowKpt];
        const bool full = wt < Wfull;
        if (full)
          tile_issue<kRowKpt>(args.keys + (uint64_t)wt * kWt + lane, args.weights + (uint64_t)wt * kWt + lane, ka,
                              wa);
        __builtin_amdgcn_sched_barrier(0);
        bad |= rows_wave_tile<PRIME, MODE, K, NP, kRowKpt>(args, c1, one, r0, words, wt, full, ka, wa, lane);
      }
    }
  }
  if (bad) atomicOr(args.flags, kFlagDomain);
  __syncthreads();
  rows_flush(args, r0, words, nwords, blockIdx.x / G, gridDim.x / G);
}

// One wave tile (64 * KPT keys from `base`) added to every row of the sketch
// with device-scope int64 atomics; returns domain-error bits.
template <int PRIME, int MODE, int K, int NP, int KPT, typename KeyT, typename WT>
__device__ __forceinline__ uint32_t direct_wave_tile(const RowArgs<KeyT, WT>& args, uint64_t base, uint32_t lane) {
  uint32_t x0[KPT], x1[KPT];
  int64_t wv[KPT];
  bool ok[KPT];
  load_tile<KPT>(args.keys, args.weights, base, 64, lane, args.n, x0, x1, wv, ok);
  uint32_t any_hi = 0;
#pragma unroll
  for (int j = 0; j < KPT; ++j) any_hi |= x1[j];
  const uint32_t bad = PRIME == kPrime61 ? any_hi >> 28 : 0u;  // key >= 2^60 breaks p >= 2u - 1
  const bool wide = PRIME == kPrime61 && sizeof(KeyT) == 8 && __any(any_hi != 0);
  uint64_t wneg[KPT];
#pragma unroll
  for (int j = 0; j < KPT; ++j) wneg[j] = (uint64_t)wv[j] ^ (uint64_t)(-wv[j]);
  for (uint32_t r = 0; r < args.rows; ++r) {
    const auto c = load_row_coeffs<K, NP>(args.coeffs + (size_t)r * NP * K);
    unsigned long long* const row = args.table + ((size_t)r << args.log2m);
    if (wide) {
#pragma unroll
      for (int j = 0; j < KPT; ++j) {
        uint32_t bk, m;
        bucket_mask<PRIME, MODE, K, true, NP>(c, x0[j], x1[j], args.log2m, bk, m);
        if (ok[j]) atomicAdd(&row[bk], masked_signed(m, wv[j], wneg[j]));
      }
    } else {
#pragma unroll
      for (int j = 0; j < KPT; ++j) {
        uint32_t bk, m;
        bucket_mask<PRIME, MODE, K, false, NP>(c, x0[j], x1[j], args.log2m, bk, m);
        if (ok[j]) atomicAdd(&row[bk], masked_signed(m, wv[j], wneg[j]));
      }
    }
  }
  return bad;
}

// Batched row-resident update: a persistent grid of one 1024-thread block per
// CU takes items from one queue (zero at launch), in the order the host
// listed them (largest first).  A rows item is one row group of one sketch
// over a range of its wave tiles: the block sets the group's 16-bit fields to
// their bias, its waves split the range's tiles, and the block then adds the
// fields into the sketch's counters, all as k_update_rows does.  A direct item
// (rpg 0) adds each key of its range to every row of its sketch with
// device-scope atomics (streams much shorter than the table).  The next
// item's index is taken while the current one runs.
template <int PRIME, int MODE, int K, typename KeyT, typename WT, int KPT>
__global__ __launch_bounds__(kRowBlock) void k_batch_rows(const BatchSketch* __restrict__ sks,
                                                          const BatchRowItem* __restrict__ items, uint32_t nitems,
                                                          uint32_t* __restrict__ queue) {
  // the fields; between items, words[0] passes the next item's index to the block
  __shared__ __align__(16) uint32_t words[kRowLdsBytes / 4];
  constexpr int NP = MODE == kTwoPoly ? 2 : 1;
  constexpr uint64_t kWt = 64 * KPT;
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (threadIdx.x == 0) words[0] = atomicAdd(queue, 1u);
  __syncthreads();
  uint32_t it = __builtin_amdgcn_readfirstlane(words[0]);
  __syncthreads();  // read by all before the fields are set
  while (it < nitems) {
    uint32_t pre = 0;
    if (threadIdx.x == 0) pre = atomic_add_ahead(queue, 1u);
    const BatchRowItem item = uniform_load(items + it);
    const BatchSketch sk = uniform_load(sks + item.sketch);
    const RowArgs<KeyT, WT> a{(const KeyT*)sk.keys, (const WT*)sk.weights, sk.n, sk.coeffs, sk.rows, sk.log2m,
                              item.rpg, 0, 0, sk.table, sk.flags, nullptr, 0, 0};
    uint32_t bad = 0;
    if (item.rpg) {
      const uint32_t nwords = item.rpg << (sk.log2m - 1);
      for (uint32_t i = threadIdx.x; i < nwords; i += kRowBlock) words[i] = 0x80008000u;
      __syncthreads();
      const auto c1 = load_row_coeffs<K, NP>(sk.coeffs + (size_t)item.r0 * NP * K);
      const bool one = item.rpg == 1;
      for (uint64_t wt = item.wt_begin + wave; wt < item.wt_end; wt += kRowBlock / 64) {
        KeyT ka[KPT];
        WT wa[KPT];
        const bool full = (wt + 1) * kWt <= a.n;
        if (full) tile_issue<KPT>(a.keys + wt * kWt + lane, a.weights + wt * kWt + lane, ka, wa);
        __builtin_amdgcn_sched_barrier(0);
        bad |= rows_wave_tile<PRIME, MODE, K, NP, KPT>(a, c1, one, item.r0, words, wt, full, ka, wa, lane);
      }
      __syncthreads();
      rows_flush(a, item.r0, words, nwords, item.spread & 0xFFFFu, item.spread >> 16);
    } else {
      for (uint64_t wt = item.wt_begin + wave; wt < item.wt_end; wt += kRowBlock / 64)
        bad |= direct_wave_tile<PRIME, MODE, K, NP, KPT>(a, wt * kWt, lane);
    }
    if (bad) atomicOr(sk.flags, kFlagDomain);
    // every wave is done with the item (the flush has read the fields) before
    // the next index is written over them; all read it before the next item
    // sets the fields
    __syncthreads();
    if (threadIdx.x == 0) words[0] = pre;
    __syncthreads();
    it = __builtin_amdgcn_readfirstlane(words[0]);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Two-pass update for tables larger than LDS.
//
// The m buckets of a row are cut into G = m / R ranges of R = 2^log2r
// buckets; (row, range) is a partition.
// Pass 1 (k_bin): each block takes tiles of kBinTile keys.  For every row it
// hashes the tile's keys and writes one 4-byte record per key into the
// tile's region for that row, grouped by range.  A record is
// (bucket mod R) << (wb + 1) | a << wb | (s w mod 2^wb), wb = 31 - log2r,
// with the sign s = 1 - 2a applied to the weight (pass 2 reads the low wb
// bits as a signed number; bit wb, the sign bit a, is only carried along).
// A weight w with |w| >= 2^(wb-1) is added to the global table directly with
// an atomic instead.  The descriptors hold the offsets of
// the groups in the region, range-major (desc_index).
// Pass 2 (k_accumulate): persistent blocks take (partition, slice of tiles)
// items, add the item's records into an int64 LDS table of R counters, then
// add the non-zero counters into the global table with coalesced atomics.
// ---------------------------------------------------------------------------

// Exclusive prefix of in[0..G) into out[0..G] by one wave (out[G] = total):
// per 64 entries, DPP within 16-lane rows (row_shr 1, 2, 4, 8), then each
// row adds the totals of the rows before it.
__device__ __forceinline__ void wave_exclusive_scan(const uint32_t* in, uint32_t* out, uint32_t G, uint32_t lane) {
  uint32_t carry = 0;
  for (uint32_t b = 0; b < G; b += 64) {
    const uint32_t v0 = b + lane < G ? in[b + lane] : 0u;
    uint32_t v = v0;
    v += __builtin_amdgcn_update_dpp(0u, v, 0x111, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0u, v, 0x112, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0u, v, 0x114, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0u, v, 0x118, 0xf, 0xf, false);
    const uint32_t t0 = __builtin_amdgcn_readlane(v, 15);
    const uint32_t t1 = t0 + __builtin_amdgcn_readlane(v, 31);
    const uint32_t t2 = t1 + __builtin_amdgcn_readlane(v, 47);
    v += lane < 16 ? 0u : lane < 32 ? t0 : lane < 48 ? t1 : t2;
    if (b + lane < G) out[b + lane] = carry + v - v0;
    carry += __builtin_amdgcn_readlane(v, 63);
  }
  if (lane == 0) out[G] = carry;
}

__device__ __forceinline__ uint32_t dedup_slot(uint32_t x0, uint32_t x1) {
  return (x0 * 0x9E3779B1u) ^ (x1 * 0x85EBCA77u) ^ (x0 >> 15);
}

// Bits of a where m is set, of b elsewhere (one v_bfi_b32).
__device__ __forceinline__ uint32_t bitsel(uint32_t m, uint32_t a, uint32_t b) { return (m & a) | (~m & b); }

// Lanes below this one whose bit is set in the wave mask m.
__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Key combining: inserts a thread's kKpt keys (key j has tile index
// idx0 + j * stride) into an open-addressing table `slots` (smask + 1 entries
// of tile index + 1, 0 = empty, linear probing) whose keys and weights are
// skey/swt by tile index.  The first copy of a key owns its entry; later
// copies add their weight into the owner's swt.  Each probe round issues the
// compare-and-swaps of all j together; a settled j re-reads its slot with a
// compare value no entry holds.  Returns bit j set where key j owns its entry.
// Ends within smask + 1 rounds when the table holds at most half as many keys.
template <int kKpt>
__device__ __forceinline__ uint32_t combine_keys(uint32_t* slots, uint32_t smask, const unsigned long long* skey,
                                                 long long* swt, const uint32_t (&x0)[kKpt],
                                                 const uint32_t (&x1)[kKpt], const int64_t (&wv)[kKpt],
                                                 const bool (&ok)[kKpt], uint32_t idx0, uint32_t stride) {
  uint32_t h[kKpt], pend = 0, own = 0;
#pragma unroll
  for (int j = 0; j < kKpt; ++j) {
    h[j] = dedup_slot(x0[j], x1[j]) & smask;
    pend |= (ok[j] ? 1u : 0u) << j;
  }
  while (pend) {
    uint32_t cur[kKpt];
#pragma unroll
    for (int j = 0; j < kKpt; ++j)
      cur[j] = atomicCAS(&slots[h[j]], ((pend >> j) & 1u) ? 0u : 0xffffffffu, idx0 + (uint32_t)j * stride + 1u);
    unsigned long long other[kKpt];
#pragma unroll
    for (int j = 0; j < kKpt; ++j) other[j] = skey[cur[j] ? cur[j] - 1u : 0u];
#pragma unroll
    for (int j = 0; j < kKpt; ++j) {
      if (!((pend >> j) & 1u)) continue;
      const unsigned long long key = ((unsigned long long)x1[j] << 32) | x0[j];
      if (cur[j] == 0) {
        own |= 1u << j;
        pend &= ~(1u << j);
      } else if (other[j] == key) {
        atomicAdd((unsigned long long*)&swt[cur[j] - 1u], (unsigned long long)wv[j]);
        pend &= ~(1u << j);
      } else {
        h[j] = (h[j] + 1u) & smask;
      }
    }
  }
  return own;
}

// Whether key combining pays on a launch's keys: fewer than permille / 1000
// of the keys in the probe's sample windows are distinct (k_combine_probe).
// Wave-uniform.
__device__ __forceinline__ bool combine_pays(const uint32_t* probe, uint32_t samples, uint32_t permille) {
  const uint32_t lane = threadIdx.x & 63;
  uint32_t d = lane < samples ? probe[lane] : 0u;
  uint32_t c = lane < samples ? probe[kProbeTiles + lane] : 0u;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    d += __shfl_xor(d, o, 64);
    c += __shfl_xor(c, o, 64);
  }
  return (uint64_t)__builtin_amdgcn_readfirstlane(d) * 1000 < (uint64_t)__builtin_amdgcn_readfirstlane(c) * permille;
}

// LDS layout of k_bin: [combining: keys u64[T] | weights i64[T] | slots
// u32[2T]] | stage u32[T] | hist u32[rows*G] | offs u32[G+1] | spare u32
// (bin_lds_fixed_bytes() covers the parts before hist).
template <int PRIME, int MODE, int K, typename KeyT, typename WT, bool DEDUP>
__global__ __launch_bounds__(kBlock) void k_bin(BinArgs<KeyT, WT> args) {
  // every wave takes the same choice, so a block leaves before any barrier
  if (args.probe && combine_pays(args.probe, args.probe_tiles, args.probe_permille) != DEDUP) return;
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr uint32_t T = kBinTile;
  unsigned long long* skey = (unsigned long long*)smem;          // DEDUP
  long long* swt = (long long*)(smem + T * 8);                    // DEDUP
  uint32_t* slots = (uint32_t*)(smem + T * 16);                   // DEDUP, 2T entries
  uint32_t* stage = (uint32_t*)(smem + (DEDUP ? T * 24 : 0));
  uint32_t* hist = stage + T;
  const uint32_t G = 1u << args.log2g;
  uint32_t* offs = hist + args.rows * G;
  uint32_t* count = offs + G + 1;
  const uint32_t log2r = args.log2r, wb = 31u - log2r;
  constexpr int kKpt = kBinKpt;
  constexpr int NP = MODE == kTwoPoly ? 2 : 1;
  const uint32_t wbmask = (1u << wb) - 1u;
  const int64_t half = 1ll << (wb - 1);
  const uint32_t lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  uint32_t bad = 0;
  for (uint32_t tile = blockIdx.x; tile < args.tiles; tile += gridDim.x) {
    for (uint32_t i = threadIdx.x; i < args.rows * G; i += kBlock) hist[i] = 0;
    if (DEDUP)
      for (uint32_t i = threadIdx.x; i < 2 * T; i += kBlock) slots[i] = 0;
    const uint64_t base = (uint64_t)tile * T;
    uint32_t x0[kKpt], x1[kKpt];
    int64_t wv[kKpt];
    bool ok[kKpt];
    load_tile<kKpt>(args.keys, args.weights, base, kBlock, threadIdx.x, args.n, x0, x1, wv, ok);
    uint32_t any_hi = 0;
#pragma unroll
    for (int j = 0; j < kKpt; ++j) any_hi |= x1[j];
    if constexpr (PRIME == kPrime61) bad |= any_hi >> 28;
    if constexpr (DEDUP) {
      // Combine repeated keys of the tile: C[i(x)] += s(x) * sum of their
      // weights is the same update (the sketch is linear).
#pragma unroll
      for (int j = 0; j < kKpt; ++j) {
        const uint32_t idx = j * kBlock + threadIdx.x;
        skey[idx] = ((unsigned long long)x1[j] << 32) | x0[j];
        swt[idx] = wv[j];
      }
      __syncthreads();
      // bit j: key j is the first copy in the tile
      const uint32_t own = combine_keys<kKpt>(slots, 2 * T - 1, skey, swt, x0, x1, wv, ok, threadIdx.x, kBlock);
      __syncthreads();
      // compact the first copies (with their summed weights) to the front:
      // wave-local positions from one ballot per j, then the waves' totals
      unsigned long long ck[kKpt];
      long long cw[kKpt];
      uint32_t pos[kKpt], wtotal = 0;
#pragma unroll
      for (int j = 0; j < kKpt; ++j) {
        const uint32_t idx = j * kBlock + threadIdx.x;
        ck[j] = skey[idx];
        cw[j] = swt[idx];
        const uint64_t m = __ballot((own >> j) & 1u);
        pos[j] = wtotal + lanes_below(m);
        wtotal += (uint32_t)__popcll(m);
      }
      if (lane == 0) stage[wave] = wtotal;  // stage is free until the row loop
      __syncthreads();
      uint32_t before = 0, total = 0;
      for (uint32_t w = 0; w < kBlock / 64; ++w) {
        const uint32_t c = stage[w];
        if (w < wave) before += c;
        total += c;
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < kKpt; ++j)
        if ((own >> j) & 1u) {
          skey[before + pos[j]] = ck[j];
          swt[before + pos[j]] = cw[j];
        }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < kKpt; ++j) {
        const uint32_t e = j * kBlock + threadIdx.x;
        ok[j] = e < total;
        const unsigned long long key = ok[j] ? skey[e] : 0ull;
        x0[j] = (uint32_t)key;
        x1[j] = (uint32_t)(key >> 32);
        wv[j] = ok[j] ? swt[e] : 0;
      }
    }
    const bool wide = PRIME == kPrime61 && sizeof(KeyT) == 8 && __any(any_hi != 0);
    __syncthreads();
    for (uint32_t r = 0; r < args.rows; ++r) {
      const auto c = load_row_coeffs<K, NP>(args.coeffs + (size_t)r * NP * K);
      uint32_t rec[kKpt], grp[kKpt], tick[kKpt];
      uint32_t codes[kKpt];
      if constexpr (PRIME == kPrime89 && MODE == kTwoForOne) {
        // a guard test per four keys (all of a lane's keys at once would hold
        // too many registers)
        constexpr int Q = kKpt % 2 == 0 ? 2 : kKpt;
#pragma unroll
        for (int j0 = 0; j0 < kKpt; j0 += Q) {
          uint32_t qa[Q], qb[Q], qc[Q];
#pragma unroll
          for (int u = 0; u < Q; ++u) {
            qa[u] = x0[j0 + u];
            qb[u] = x1[j0 + u];
          }
          code89_tile<K, NP, Q>(c, 0, qa, qb, qc);
#pragma unroll
          for (int u = 0; u < Q; ++u) codes[j0 + u] = qc[u];
        }
      } else {
#pragma unroll
        for (int j = 0; j < kKpt; ++j)
          codes[j] = wide ? bucket_code<PRIME, MODE, K, true, NP>(c, x0[j], x1[j], args.log2m)
                          : bucket_code<PRIME, MODE, K, false, NP>(c, x0[j], x1[j], args.log2m);
      }
#pragma unroll
      for (int j = 0; j < kKpt; ++j) {
        const uint32_t code = codes[j];
        grp[j] = __builtin_amdgcn_ubfe(code, 1u + log2r, args.log2g);
        const int64_t sw = (code & 1u) ? -wv[j] : wv[j];
        rec[j] = (code << wb) | ((uint32_t)sw & wbmask);
        const bool fits = wv[j] > -half && wv[j] < half;
        tick[j] = 0xffffffffu;
        if (ok[j] && wv[j] != 0) {
          if (fits) {
            tick[j] = atomicAdd(&hist[r * G + grp[j]], 1u);
          } else {
            const uint32_t bk = (code >> 1) & ((1u << args.log2m) - 1u);
            atomicAdd(&args.table[((size_t)r << args.log2m) + bk], (unsigned long long)sw);
          }
        }
      }
      __syncthreads();
      if (wave == 0) {
        wave_exclusive_scan(hist + r * G, offs, G, lane);
        for (uint32_t g = lane; g <= G; g += 64) args.desc[desc_index(r, g, G, args.tiles, tile)] = offs[g];
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < kKpt; ++j)
        if (tick[j] != 0xffffffffu) stage[offs[grp[j]] + tick[j]] = rec[j];
      __syncthreads();
      // coalesced copy of the row's records to the tile region
      const uint32_t nrec = offs[G];
      uint4* out = (uint4*)(args.recs + ((size_t)tile * args.rows + r) * T);
      const uint4* st4 = (const uint4*)stage;
      for (uint32_t q = threadIdx.x; q * 4 < nrec; q += kBlock) out[q] = st4[q];
      __syncthreads();
    }
  }
  (void)count;
  if (bad) atomicOr(args.flags, kFlagDomain);
}

// Wave-level LDS ordering point: every LDS access of the wave issued before
// it is complete and visible to the wave's other lanes after it.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Pass 1 with one tile of kWaveTile keys per wave (for G <= 16 ranges per
// row): tickets, prefix sums, key combining and staging are wave-local, so
// the kernel has no block barriers.  Same record and descriptor format as
// k_bin with tiles of kWaveTile keys.

// Rows of one wave tile: hash every slot straight-line (no branches, so the
// slots' Horner chains interleave), take tickets, prefix the group counts,
// stage the records in sorted order and copy them out with 16-byte stores.
// Tickets: a record of range g takes its ticket from counter 2g + c, c the
// top bit of its bucket mod R (two counters per range halve the lanes that
// hit one LDS address; the range's records stay contiguous).  A slot without
// a record (no key, weight 0, or a weight added directly) takes its ticket
// from spare counter 2G + (lane mod 2G) instead: the spare counters come after
// the real ones in the staging order and are never copied out, so no slot
// needs a branch or a select of its addresses.  rmask[j] is ~0 for a slot
// with a record, else 0; spare is the lane's spare counter.
template <int PRIME, int MODE, int K, int NP, bool WIDE, int kKpt, int kUse, typename BA>
__device__ __forceinline__ void bin_rows_wave(const BA& args, uint32_t tile, uint32_t G, uint32_t lane, uint32_t* hist,
                                              uint32_t* stage, const uint32_t (&x0)[kKpt], const uint32_t (&x1)[kKpt],
                                              const int64_t (&wv)[kKpt], const uint32_t (&wpos)[kKpt],
                                              const uint32_t (&wdiff)[kKpt], const uint32_t (&rmask)[kKpt],
                                              uint32_t spare, uint32_t esc, bool any_esc) {
  static_assert(kUse <= kKpt, "more slots than the tile holds");
  const uint32_t log2r = args.log2r, wb = 31u - log2r;
  const uint32_t NC = 4 * G;  // counters per row: 2G real, 2G spare; NC <= 64
  // this lane's descriptor (group `lane` of the tile) in row 0; rows follow at
  // a stride of (G + 1) * tiles words
  uint32_t* dsc = args.desc + desc_index(0, lane, G, args.tiles, tile);
  const size_t dstride = (size_t)(G + 1) * args.tiles;
  for (uint32_t r = 0; r < args.rows; ++r, dsc += dstride) {
    const auto c = load_row_coeffs<K, NP>(args.coeffs + (size_t)r * NP * K);
    uint32_t* const hrow = hist + r * NC;
    uint32_t code[kUse], gq[kUse], tick[kUse];
    if constexpr (PRIME == kPrime61 && MODE == kTwoForOne && !WIDE && kUse % 2 == 0) {
      code61_x32_tile<K, NP, kUse>(c, 0, x0, code);  // one guard test for the lane's keys
    } else {
#pragma unroll
      for (int j = 0; j < kUse; ++j) code[j] = bucket_code<PRIME, MODE, K, WIDE, NP>(c, x0[j], x1[j], args.log2m);
    }
#pragma unroll
    for (int j = 0; j < kUse; ++j) {
      gq[j] = bitsel(rmask[j], __builtin_amdgcn_ubfe(code[j], log2r, args.log2g + 1u), spare);
      tick[j] = atomicAdd(&hrow[gq[j]], 4u);  // counts in bytes of staging
    }
    if (any_esc) {  // weights too large for a record go straight to the table
#pragma unroll
      for (int j = 0; j < kUse; ++j)
        if ((esc >> j) & 1u) {
          const uint32_t bk = (code[j] >> 1) & ((1u << args.log2m) - 1u);
          const int64_t sw = (code[j] & 1u) ? -wv[j] : wv[j];
          atomicAdd(&args.table[((size_t)r << args.log2m) + bk], (unsigned long long)sw);
        }
    }
    wave_lds_sync();
    // exclusive prefix over the NC counters: DPP within 16-lane rows (row_shr
    // 1, 2, 4, 8), then each later row adds the totals of the rows before it
    const uint32_t cg = lane < NC ? hrow[lane] : 0u;
    uint32_t v = cg;
    v += __builtin_amdgcn_update_dpp(0u, v, 0x111, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0u, v, 0x112, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0u, v, 0x114, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0u, v, 0x118, 0xf, 0xf, false);
    if (NC > 32) {
      const uint32_t t0 = __builtin_amdgcn_readlane(v, 15);
      const uint32_t t1 = t0 + __builtin_amdgcn_readlane(v, 31);
      const uint32_t t2 = t1 + __builtin_amdgcn_readlane(v, 47);
      v += lane < 16 ? 0u : lane < 32 ? t0 : lane < 48 ? t1 : t2;
    } else if (NC > 16) {
      v += lane < 16 ? 0u : __builtin_amdgcn_readlane(v, 15);
    }
    // lane c: byte offset of counter c's records in the staging area; range g
    // starts at counter 2g, and counter 2G (the first spare) ends the records
    const uint32_t off = v - cg;
    const uint32_t nrec = __builtin_amdgcn_readlane(off, 2 * G) >> 2;
    const uint32_t goff = (uint32_t)__builtin_amdgcn_ds_bpermute((int)(lane << 3), (int)off);
    if (lane <= G) *dsc = goff >> 2;
    unsigned char* const stage_b = (unsigned char*)stage;
#pragma unroll
    for (int j = 0; j < kUse; ++j) {
      const uint32_t o = (uint32_t)__builtin_amdgcn_ds_bpermute((int)(gq[j] << 2), (int)off);
      // weight field with the sign applied: wneg = wpos ^ wdiff where bit 0 of
      // the code is set
      const uint32_t sgn = (uint32_t)__builtin_amdgcn_sbfe((int)code[j], 0, 1);
      *(uint32_t*)(stage_b + o + tick[j]) = (code[j] << wb) | (wpos[j] ^ (wdiff[j] & sgn));
    }
    wave_lds_sync();
    uint4* out = (uint4*)(args.recs + ((size_t)tile * args.rows + r) * kWaveTile);
    const uint4* st4 = (const uint4*)stage;
    for (uint32_t q = lane; q * 4 < nrec; q += 64) out[q] = st4[q];
    wave_lds_sync();
  }
}

// The rows of a tile with only the slots that hold keys: `live` (wave-uniform)
// keys sit in slots 0 .. ceil(live/64) - 1, so the straight-line code is
// instantiated for 2, 4, 6 and 8 slots and picked once per tile.
template <int PRIME, int MODE, int K, int NP, bool WIDE, int kKpt, typename BA>
__device__ __forceinline__ void bin_rows_wave_live(uint32_t live, const BA& args, uint32_t tile, uint32_t G,
                                                   uint32_t lane, uint32_t* hist, uint32_t* stage,
                                                   const uint32_t (&x0)[kKpt], const uint32_t (&x1)[kKpt],
                                                   const int64_t (&wv)[kKpt], const uint32_t (&wpos)[kKpt],
                                                   const uint32_t (&wdiff)[kKpt], const uint32_t (&rmask)[kKpt],
                                                   uint32_t spare, uint32_t esc, bool any_esc) {
  static_assert(kKpt == 8, "slot variants assume 8 slots per lane");
  if (live > 6 * 64)
    bin_rows_wave<PRIME, MODE, K, NP, WIDE, kKpt, 8>(args, tile, G, lane, hist, stage, x0, x1, wv, wpos, wdiff, rmask, spare, esc, any_esc);
  else if (live > 4 * 64)
    bin_rows_wave<PRIME, MODE, K, NP, WIDE, kKpt, 6>(args, tile, G, lane, hist, stage, x0, x1, wv, wpos, wdiff, rmask, spare, esc, any_esc);
  else if (live > 2 * 64)
    bin_rows_wave<PRIME, MODE, K, NP, WIDE, kKpt, 4>(args, tile, G, lane, hist, stage, x0, x1, wv, wpos, wdiff, rmask, spare, esc, any_esc);
  else
    bin_rows_wave<PRIME, MODE, K, NP, WIDE, kKpt, 2>(args, tile, G, lane, hist, stage, x0, x1, wv, wpos, wdiff, rmask, spare, esc, any_esc);
}

// One wave tile of pass 1 (kWaveTile keys of `args`, wave-local LDS `mine`).
// Returns domain-error bits.
template <int PRIME, int MODE, int K, typename KeyT, typename WT, bool DEDUP>
__device__ __forceinline__ uint32_t bin_wave_tile(const BinArgs<KeyT, WT>& args, uint32_t tile, uint32_t lane,
                                                  unsigned char* mine) {
  constexpr uint32_t T = kWaveTile;
  constexpr int kKpt = T / 64;
  constexpr int NP = MODE == kTwoPoly ? 2 : 1;
  const uint32_t G = 1u << args.log2g;
  unsigned long long* skey = (unsigned long long*)mine;
  long long* swt = (long long*)(mine + T * 8);
  uint32_t* slots = (uint32_t*)(mine + (DEDUP ? T * 16 : 0));
  uint32_t* stage = slots;  // reused once the combining table is no longer needed
  uint32_t* hist = slots + 2 * T;
  const uint32_t wb = 31u - args.log2r;
  const uint32_t wbmask = (1u << wb) - 1u;
  const int64_t half = 1ll << (wb - 1);
  uint32_t bad = 0;
  {
    for (uint32_t i = lane; i < args.rows * 4 * G; i += 64) hist[i] = 0;
    if (DEDUP)
      for (uint32_t i = lane; i < 2 * T; i += 64) slots[i] = 0;
    const uint64_t base = (uint64_t)tile * T;
    // keys that reach the rows (after combining: the distinct ones), wave-uniform
    uint32_t live = (uint32_t)min((uint64_t)T, args.n - base);
    uint32_t x0[kKpt], x1[kKpt];
    int64_t wv[kKpt];
    bool ok[kKpt];
    load_tile<kKpt>(args.keys, args.weights, base, 64, lane, args.n, x0, x1, wv, ok);
    uint32_t any_hi = 0;
#pragma unroll
    for (int j = 0; j < kKpt; ++j) any_hi |= x1[j];
    if constexpr (PRIME == kPrime61) bad |= any_hi >> 28;
    if constexpr (DEDUP) {
      // Combine repeated keys of the tile (exact: the sketch is linear).
#pragma unroll
      for (int j = 0; j < kKpt; ++j) {
        const uint32_t idx = j * 64 + lane;
        skey[idx] = ((unsigned long long)x1[j] << 32) | x0[j];
        swt[idx] = wv[j];
      }
      wave_lds_sync();
      const uint32_t own = combine_keys<kKpt>(slots, 2 * T - 1, skey, swt, x0, x1, wv, ok, lane, 64);
      wave_lds_sync();
      // compact the first copies to the front, positions from one ballot per j
      unsigned long long ck[kKpt];
      long long cw[kKpt];
      uint32_t pos[kKpt], total = 0;
#pragma unroll
      for (int j = 0; j < kKpt; ++j) {
        const uint32_t idx = j * 64 + lane;
        ck[j] = skey[idx];
        cw[j] = swt[idx];
        const uint64_t m = __ballot((own >> j) & 1u);
        pos[j] = total + lanes_below(m);
        total += (uint32_t)__popcll(m);
      }
      live = __builtin_amdgcn_readfirstlane(total);
      wave_lds_sync();
#pragma unroll
      for (int j = 0; j < kKpt; ++j)
        if ((own >> j) & 1u) {
          skey[pos[j]] = ck[j];
          swt[pos[j]] = cw[j];
        }
      wave_lds_sync();
#pragma unroll
      for (int j = 0; j < kKpt; ++j) {
        const uint32_t e = j * 64 + lane;
        ok[j] = e < total;
        const unsigned long long key = ok[j] ? skey[e] : 0ull;
        x0[j] = (uint32_t)key;
        x1[j] = (uint32_t)(key >> 32);
        wv[j] = ok[j] ? swt[e] : 0;
      }
      wave_lds_sync();
    }
    const bool wide = PRIME == kPrime61 && sizeof(KeyT) == 8 && __any(any_hi != 0);
    // per key, independent of the row: the record's weight field for both
    // signs, whether the key has a record, its spare group, and the weights
    // added directly
    uint32_t esc = 0;  // bit j: key j's weight is added directly
    uint32_t wpos[kKpt], wdiff[kKpt], rmask[kKpt];
    const uint32_t spare = 2 * G + (lane & (2 * G - 1));
#pragma unroll
    for (int j = 0; j < kKpt; ++j) {
      const bool fits = wv[j] > -half && wv[j] < half;
      rmask[j] = ok[j] && wv[j] != 0 && fits ? ~0u : 0u;
      esc |= (ok[j] && !fits ? 1u : 0u) << j;
      wpos[j] = (uint32_t)wv[j] & wbmask;
      wdiff[j] = wpos[j] ^ ((uint32_t)(-wv[j]) & wbmask);
    }
    const bool any_esc = __any(esc != 0);
    if (wide)
      bin_rows_wave_live<PRIME, MODE, K, NP, true, kKpt>(live, args, tile, G, lane, hist, stage, x0, x1, wv, wpos, wdiff,
                                                         rmask, spare, esc, any_esc);
    else
      bin_rows_wave_live<PRIME, MODE, K, NP, false, kKpt>(live, args, tile, G, lane, hist, stage, x0, x1, wv, wpos,
                                                          wdiff, rmask, spare, esc, any_esc);
    }
  return bad;
}

template <int PRIME, int MODE, int K, typename KeyT, typename WT, bool DEDUP>
__global__ __launch_bounds__(kBlock) void k_bin_wave(BinArgs<KeyT, WT> args) {
  if (args.probe && combine_pays(args.probe, args.probe_tiles, args.probe_permille) != DEDUP) return;
  extern __shared__ __align__(16) unsigned char smem[];
  // wave index made explicitly uniform so the tile loop, the row loop and the
  // coefficient loads stay scalar
  const uint32_t lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  unsigned char* mine = smem + (size_t)wave * binw_lds_per_wave<DEDUP>(args.rows, 1u << args.log2g);
  const uint32_t nw = gridDim.x * (kBlock / 64);
  uint32_t bad = 0;
  for (uint32_t tile = blockIdx.x * (kBlock / 64) + wave; tile < args.tiles; tile += nw)
    bad |= bin_wave_tile<PRIME, MODE, K, KeyT, WT, DEDUP>(args, tile, lane, mine);
  if (bad) atomicOr(args.flags, kFlagDomain);
}

// Combining probe: block b (one wave) combines the 512-key window
// floor(b * windows / samples) of the keys exactly as pass 1 would and writes
// its distinct and total key counts to probe[b] and probe[kProbeTiles + b]
// (samples <= min(kProbeTiles, windows)).
template <typename KeyT>
__global__ __launch_bounds__(64) void k_combine_probe(const KeyT* __restrict__ keys, uint64_t n, uint32_t samples,
                                                      uint32_t* __restrict__ probe) {
  constexpr uint32_t T = kWaveTile;
  constexpr int kKpt = T / 64;
  __shared__ unsigned long long skey[T];
  __shared__ long long swt[T];
  __shared__ uint32_t slots[2 * T];
  const uint32_t lane = threadIdx.x;
  const uint64_t windows = (n + T - 1) / T;
  const uint64_t base = (uint64_t)blockIdx.x * windows / samples * T;
  for (uint32_t i = lane; i < 2 * T; i += 64) slots[i] = 0;
  uint32_t x0[kKpt], x1[kKpt];
  int64_t wv[kKpt];
  bool ok[kKpt];
#pragma unroll
  for (int j = 0; j < kKpt; ++j) {
    const uint64_t i = base + (uint64_t)j * 64 + lane;
    ok[j] = i < n;
    const uint64_t k = ok[j] ? (uint64_t)keys[i] : 0ull;
    x0[j] = (uint32_t)k;
    x1[j] = (uint32_t)(k >> 32);
    wv[j] = 0;
    skey[j * 64 + lane] = k;
    swt[j * 64 + lane] = 0;
  }
  wave_lds_sync();
  const uint32_t own = combine_keys<kKpt>(slots, 2 * T - 1, skey, swt, x0, x1, wv, ok, lane, 64);
  uint32_t distinct = 0, total = 0;
#pragma unroll
  for (int j = 0; j < kKpt; ++j) {
    distinct += (uint32_t)__popcll(__ballot((own >> j) & 1u));
    total += (uint32_t)__popcll(__ballot(ok[j]));
  }
  if (lane == 0) {
    probe[blockIdx.x] = distinct;
    probe[kProbeTiles + blockIdx.x] = total;
  }
}

// ---------------------------------------------------------------------------
// Point query: median over rows of s_j(x) C[j][i_j(x)] (Section 1.3.1).
// ---------------------------------------------------------------------------
template <int PRIME, int MODE, int K, typename KeyT>
__global__ __launch_bounds__(kBlock) void k_query(QueryArgs<KeyT> args) {
  constexpr int NP = MODE == kTwoPoly ? 2 : 1;
  uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= args.n) return;
  uint32_t x0, x1;
  load_key(args.keys, i, x0, x1);
  if (PRIME == kPrime61 && (x1 >> 28)) atomicOr(args.flags, kFlagDomain);
  int64_t vals[kMaxQueryRows];
  uint32_t rows = args.rows;
  for (uint32_t r = 0; r < rows; ++r) {
    uint32_t bk, a;
    const auto c = load_row_coeffs<K, NP>(args.coeffs + (size_t)r * NP * K);
    if (PRIME == kPrime61 && x1 != 0)
      bucket_sign<PRIME, MODE, K, true, NP>(c, x0, x1, args.log2m, bk, a);
    else
      bucket_sign<PRIME, MODE, K, false, NP>(c, x0, x1, args.log2m, bk, a);
    int64_t v = args.table[((size_t)r << args.log2m) + bk];
    v = a ? (int64_t)(0ull - (uint64_t)v) : v;
    // insertion into the sorted prefix
    uint32_t p = r;
    while (p > 0 && vals[p - 1] > v) {
      vals[p] = vals[p - 1];
      --p;
    }
    vals[p] = v;
  }
  args.out[i] = vals[(rows - 1) / 2];
}

// ---------------------------------------------------------------------------
// F2 estimate: per (row, slice) 128-bit partial sums of C^2, then one block
// adds them, checks the int64 range and takes the median over rows.
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Batched update: many independent sketches (same prime, mode and k) in one
// launch per pass.  Every work item is (sketch, keys), so a wave always hashes
// with one sketch's coefficients.
//   k_batch_lds:  items (sketch, key range) of sketches whose table fits LDS
//   k_batch_bin:  pass 1 over the wave tiles of all segments of a round;
//                 a wave finds its segment by binary search on tile_begin
//   k_batch_acc:  pass 2 items (segment, partition, slice)
// ---------------------------------------------------------------------------
template <int PRIME, int MODE, int K, typename KeyT, typename WT>
__global__ __launch_bounds__(kBlock) void k_batch_lds(const BatchSketch* __restrict__ sks,
                                                      const BatchLdsItem* __restrict__ items, uint32_t nitems) {
  extern __shared__ unsigned long long lds[];
  for (uint32_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    const BatchLdsItem item = uniform_load(items + it);
    const BatchSketch sk = uniform_load(sks + item.sketch);
    UpdateArgs<KeyT, WT> a{(const KeyT*)sk.keys, (const WT*)sk.weights, sk.n, 0, sk.coeffs, sk.rows, sk.log2m,
                           sk.table, sk.flags};
    __syncthreads();  // the previous item's flush has read the LDS table
    lds_block_update<PRIME, MODE, K, KeyT, WT>(a, item.begin, item.end, lds);
  }
}

template <int PRIME, int MODE, int K, typename KeyT, typename WT>
__global__ __launch_bounds__(kBlock) void k_batch_global(const BatchSketch* __restrict__ sks,
                                                         const BatchLdsItem* __restrict__ items, uint32_t nitems) {
  for (uint32_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    const BatchLdsItem item = uniform_load(items + it);
    const BatchSketch sk = uniform_load(sks + item.sketch);
    UpdateArgs<KeyT, WT> a{(const KeyT*)sk.keys, (const WT*)sk.weights, sk.n, 0, sk.coeffs, sk.rows, sk.log2m,
                           sk.table, sk.flags};
    global_block_update<PRIME, MODE, K, KeyT, WT>(a, item.begin, item.end);
  }
}

template <int PRIME, int MODE, int K, typename KeyT, typename WT, bool DEDUP>
__global__ __launch_bounds__(kBlock) void k_batch_bin(const BatchSegment* __restrict__ segs, uint32_t nsegs,
                                                      uint32_t total_tiles, uint32_t lds_per_wave) {
  extern __shared__ __align__(16) unsigned char smem[];
  const uint32_t lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  unsigned char* mine = smem + (size_t)wave * lds_per_wave;
  const uint32_t nw = gridDim.x * (kBlock / 64);
  for (uint32_t gt = blockIdx.x * (kBlock / 64) + wave; gt < total_tiles; gt += nw) {
    uint32_t lo = 0, hi = nsegs;  // last segment with tile_begin <= gt
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (uniform_load(&segs[mid].tile_begin) <= gt) lo = mid; else hi = mid;
    }
    const BatchSegment sg = uniform_load(segs + lo);
    BinArgs<KeyT, WT> a{(const KeyT*)sg.keys, (const WT*)sg.weights, sg.n, sg.coeffs, sg.rows, sg.log2m, sg.log2g,
                        sg.log2r, sg.tiles, sg.recs, sg.desc, sg.table, sg.flags};
    const uint32_t bad = bin_wave_tile<PRIME, MODE, K, KeyT, WT, DEDUP>(a, gt - sg.tile_begin, lane, mine);
    if (bad) atomicOr(sg.flags, kFlagDomain);
  }
}

template <int PRIME, int MODE, int K, typename KeyT, typename WT>
hipError_t launch_batch_t(const BatchLaunch& b, hipStream_t st) {
  if (b.prepare_only) {  // kernel attributes, set once before any launch or graph capture
    hipError_t e = hipFuncSetAttribute((const void*)k_batch_lds<PRIME, MODE, K, KeyT, WT>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e == hipSuccess) e = set_batch_acc_attribute();
    return e;
  }
  if (b.lds_items) {
    hipLaunchKernelGGL((k_batch_lds<PRIME, MODE, K, KeyT, WT>), dim3(b.lds_blocks), dim3(kBlock), b.lds_bytes, st,
                       b.sketches, b.lds_item_list, b.lds_items);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (b.glb_items) {
    hipLaunchKernelGGL((k_batch_global<PRIME, MODE, K, KeyT, WT>), dim3(b.glb_blocks), dim3(kBlock), 0, st,
                       b.sketches, b.glb_item_list, b.glb_items);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (b.row_items) {
    // the queue starts at zero on every launch (a kernel, not a memset, so
    // that a captured graph replays it)
    hipError_t e = launch_fill_zero((unsigned long long*)b.row_queue, 1, st);
    if (e != hipSuccess) return e;
    if (b.row_kpt == 2)
      hipLaunchKernelGGL((k_batch_rows<PRIME, MODE, K, KeyT, WT, 2>), dim3(b.row_blocks), dim3(kRowBlock), 0, st,
                         b.sketches, b.row_item_list, b.row_items, b.row_queue);
    else if (b.row_kpt == 4)
      hipLaunchKernelGGL((k_batch_rows<PRIME, MODE, K, KeyT, WT, 4>), dim3(b.row_blocks), dim3(kRowBlock), 0, st,
                         b.sketches, b.row_item_list, b.row_items, b.row_queue);
    else
      hipLaunchKernelGGL((k_batch_rows<PRIME, MODE, K, KeyT, WT, 8>), dim3(b.row_blocks), dim3(kRowBlock), 0, st,
                         b.sketches, b.row_item_list, b.row_items, b.row_queue);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  for (uint32_t r = 0; r < b.rounds; ++r) {
    const BatchRound& rd = b.round_list[r];
    if (b.dedup)
      hipLaunchKernelGGL((k_batch_bin<PRIME, MODE, K, KeyT, WT, true>), dim3(rd.bin_blocks), dim3(kBlock),
                         b.bin_lds_bytes, st, rd.segs, rd.nsegs, rd.total_tiles, b.bin_lds_per_wave);
    else
      hipLaunchKernelGGL((k_batch_bin<PRIME, MODE, K, KeyT, WT, false>), dim3(rd.bin_blocks), dim3(kBlock),
                         b.bin_lds_bytes, st, rd.segs, rd.nsegs, rd.total_tiles, b.bin_lds_per_wave);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_batch_acc(rd, b.acc_lds_bytes, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int PRIME, int MODE, int K>
hipError_t launch_batch_k(const BatchLaunch& b, hipStream_t st) {
  if (b.key_bytes == 4 && b.weight_bytes == 4) return launch_batch_t<PRIME, MODE, K, uint32_t, int32_t>(b, st);
  if (b.key_bytes == 4 && b.weight_bytes == 8) return launch_batch_t<PRIME, MODE, K, uint32_t, int64_t>(b, st);
  if (b.key_bytes == 8 && b.weight_bytes == 4) return launch_batch_t<PRIME, MODE, K, uint64_t, int32_t>(b, st);
  return launch_batch_t<PRIME, MODE, K, uint64_t, int64_t>(b, st);
}

template <int PRIME, int MODE>
hipError_t launch_batch_pm(const BatchLaunch& b, hipStream_t st) {
  switch (b.k) {
    case 2: return launch_batch_k<PRIME, MODE, 2>(b, st);
    case 8: return launch_batch_k<PRIME, MODE, 8>(b, st);
    default: return launch_batch_k<PRIME, MODE, 4>(b, st);
  }
}

// ---------------------------------------------------------------------------
// launch helpers (host side)
// ---------------------------------------------------------------------------
template <int PRIME, int MODE, int K, typename KeyT, typename WT>
hipError_t launch_update_t(const UpdatePlan& plan, const UpdateArgs<KeyT, WT>& a, hipStream_t st) {
  if (plan.variant == kVariantBinned) {
    BinArgs<KeyT, WT> b{a.keys, a.weights, a.n, a.coeffs, a.rows, a.log2m, plan.log2g, plan.log2r, plan.tiles,
                        plan.recs, plan.desc, a.table, a.flags};
    // dynamic LDS above 64 KiB needs the kernel attribute, once per device
    static std::atomic<uint64_t> attr_done{0};
    hipError_t ea = once_per_device(attr_done, [] {
      hipError_t e = set_accumulate_attribute();
      if (e == hipSuccess)
        e = hipFuncSetAttribute((const void*)k_bin<PRIME, MODE, K, KeyT, WT, true>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
      return e;
    });
    if (ea != hipSuccess) return ea;
    auto launch_bin = [&](bool dedup, uint32_t lds) {
      if (plan.wave_tiles && dedup)
        hipLaunchKernelGGL((k_bin_wave<PRIME, MODE, K, KeyT, WT, true>), dim3(plan.blocks), dim3(kBlock), lds, st, b);
      else if (plan.wave_tiles)
        hipLaunchKernelGGL((k_bin_wave<PRIME, MODE, K, KeyT, WT, false>), dim3(plan.blocks), dim3(kBlock), lds, st, b);
      else if (dedup)
        hipLaunchKernelGGL((k_bin<PRIME, MODE, K, KeyT, WT, true>), dim3(plan.blocks), dim3(kBlock), lds, st, b);
      else
        hipLaunchKernelGGL((k_bin<PRIME, MODE, K, KeyT, WT, false>), dim3(plan.blocks), dim3(kBlock), lds, st, b);
      return hipGetLastError();
    };
    hipError_t e;
    if (plan.combine_auto) {
      // The probe decides on the device; of the two pass-1 launches the one
      // that does not match leaves at once.  Block tiles need more duplicates
      // than wave tiles to gain: their combining table costs occupancy.
      const uint64_t windows = (a.n + kWaveTile - 1) / kWaveTile;
      const uint32_t samples = (uint32_t)std::min<uint64_t>(kProbeTiles, windows);
      hipLaunchKernelGGL((k_combine_probe<KeyT>), dim3(samples), dim3(64), 0, st, a.keys, a.n, samples, plan.probe);
      b.probe = plan.probe;
      b.probe_tiles = samples;
      b.probe_permille = plan.wave_tiles ? 900 : 750;
      if ((e = hipGetLastError()) != hipSuccess || (e = launch_bin(true, plan.lds_bytes)) != hipSuccess ||
          (e = launch_bin(false, plan.lds_bytes_plain)) != hipSuccess)
        return e;
    } else if ((e = launch_bin(plan.dedup, plan.lds_bytes)) != hipSuccess) {
      return e;
    }
    AccArgs c{plan.recs, plan.desc, plan.tiles, a.rows, a.log2m, plan.log2g, plan.log2r, plan.acc_slices,
              plan.wave_tiles ? kWaveTile : kBinTile, a.table};
    return launch_accumulate(c, plan.acc_blocks, plan.acc_lds_bytes, st);
  }
  if (plan.variant == kVariantRows) {
    RowArgs<KeyT, WT> r{a.keys, a.weights, a.n, a.coeffs, a.rows, a.log2m, plan.rpg, a.rows / plan.rpg,
                        plan.tiles, a.table, a.flags, plan.queues, kRowXcds, plan.range_blocks};
    // the queues start at zero (a fill kernel: no memset node in a captured graph)
    hipError_t ez = launch_fill_zero((unsigned long long*)plan.queues, kRowRanges * kMaxRows / 2, st);
    if (ez != hipSuccess) return ez;
    hipLaunchKernelGGL((k_update_rows<PRIME, MODE, K, KeyT, WT>), dim3(plan.blocks), dim3(kRowBlock), 0, st, r);
    return hipGetLastError();
  }
  if (plan.variant == kVariantLds) {
    hipLaunchKernelGGL((k_update_lds<PRIME, MODE, K, KeyT, WT>), dim3(plan.blocks), dim3(kBlock), plan.lds_bytes, st, a);
  } else {
    hipLaunchKernelGGL((k_update_global<PRIME, MODE, K, KeyT, WT>), dim3(plan.blocks), dim3(kBlock), 0, st, a);
  }
  return hipGetLastError();
}

template <int PRIME, int MODE, int K>
hipError_t launch_update_k(const UpdatePlan& plan, const UpdateArgsAny& a, hipStream_t st) {
  if (a.key_bytes == 4 && a.weight_bytes == 4)
    return launch_update_t<PRIME, MODE, K, uint32_t, int32_t>(plan, a.as<uint32_t, int32_t>(), st);
  if (a.key_bytes == 4 && a.weight_bytes == 8)
    return launch_update_t<PRIME, MODE, K, uint32_t, int64_t>(plan, a.as<uint32_t, int64_t>(), st);
  if (a.key_bytes == 8 && a.weight_bytes == 4)
    return launch_update_t<PRIME, MODE, K, uint64_t, int32_t>(plan, a.as<uint64_t, int32_t>(), st);
  return launch_update_t<PRIME, MODE, K, uint64_t, int64_t>(plan, a.as<uint64_t, int64_t>(), st);
}

template <int PRIME, int MODE>
hipError_t launch_update_pm(const UpdatePlan& plan, const UpdateArgsAny& a, hipStream_t st) {
  switch (a.k) {
    case 2: return launch_update_k<PRIME, MODE, 2>(plan, a, st);
    case 8: return launch_update_k<PRIME, MODE, 8>(plan, a, st);
    default: return launch_update_k<PRIME, MODE, 4>(plan, a, st);
  }
}

template <int PRIME, int MODE, int K, typename KeyT>
hipError_t launch_query_t(const QueryArgs<KeyT>& a, hipStream_t st) {
  uint64_t blocks = (a.n + kBlock - 1) / kBlock;
  hipLaunchKernelGGL((k_query<PRIME, MODE, K, KeyT>), dim3((uint32_t)blocks), dim3(kBlock), 0, st, a);
  return hipGetLastError();
}

template <int PRIME, int MODE, int K>
hipError_t launch_query_k(const QueryArgsAny& a, hipStream_t st) {
  if (a.key_bytes == 4) return launch_query_t<PRIME, MODE, K, uint32_t>(a.as<uint32_t>(), st);
  return launch_query_t<PRIME, MODE, K, uint64_t>(a.as<uint64_t>(), st);
}

template <int PRIME, int MODE>
hipError_t launch_query_pm(const QueryArgsAny& a, hipStream_t st) {
  switch (a.k) {
    case 2: return launch_query_k<PRIME, MODE, 2>(a, st);
    case 8: return launch_query_k<PRIME, MODE, 8>(a, st);
    default: return launch_query_k<PRIME, MODE, 4>(a, st);
  }
}

}  // namespace mcs
