// field.hpp -- integer arithmetic over Mersenne and pseudo-Mersenne primes for
// gfx950, written on 32-bit limbs so that every wide product is a chain of
// v_mad_u64_u32 (32x32+64 -> 64, full rate on CDNA4) and every reduction is
// shifts, masks and adds.
//
// Paper: Ahle, Knudsen, Thorup, "The Power of Hashing with Mersenne Primes".
//   eq. (Mersenne): y = (y & p) + (y >> b)  (mod p) for p = 2^b - 1
//   Algorithm 1: Horner's rule with that fold after every multiply-add; with
//     p >= 2u - 1 the value stays below 2p, so one reduction at the end suffices.
//   Algorithm 4: branch-free floor(v/p) and v mod p for v < 2^(2b).
//   Algorithms 5 and 6: floor(v/p) and v mod p for p = 2^b - c.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mcs {

constexpr uint64_t kP61 = (1ull << 61) - 1;
constexpr uint32_t kMask29 = (1u << 29) - 1;  // bits 32..60 of a 61-bit value
constexpr uint32_t kMask25 = (1u << 25) - 1;  // bits 64..88 of an 89-bit value

__device__ __forceinline__ uint64_t mad64(uint32_t a, uint32_t b, uint64_t c) {
  return (uint64_t)a * b + c;  // v_mad_u64_u32
}
__device__ __forceinline__ uint32_t lo32(uint64_t v) { return (uint32_t)v; }
__device__ __forceinline__ uint32_t hi32(uint64_t v) { return (uint32_t)(v >> 32); }
// (hi:lo) >> s for 0 < s < 32, one v_alignbit_b32
__device__ __forceinline__ uint32_t funnel(uint32_t hi, uint32_t lo, uint32_t s) {
  return __builtin_amdgcn_alignbit(hi, lo, s);
}

// ---------------------------------------------------------------------------
// p = 2^61 - 1.  Values are two limbs (w0 low 32 bits, w1 high).
// ---------------------------------------------------------------------------
struct F61 {
  uint32_t w0, w1;
};

// One Horner step y <- fold(y*x + a) for a key x < 2^32 (Algorithm 1), with
// the coefficient given as a_lo (its low limb, or that plus one, as a 64-bit
// value <= 2^32) and a_hi (its high limb, < 2^29).
// Preconditions: y < 2^64 (then u = y1*x + t_hi + a_hi < 2^64).  The fold
// leaves (P mod 2^61) + (P >> 61) < 2^61 + 2^35 < 2p.
__device__ __forceinline__ F61 p61_step_x32(F61 y, uint32_t x, uint64_t a_lo, uint32_t a_hi) {
  uint64_t t = mad64(y.w0, x, a_lo);                      // < 2^64: bits 0..63 partial
  uint64_t u = mad64(y.w1, x, (uint64_t)hi32(t) + a_hi);  // bits 32..95
  // P = u * 2^32 + lo32(t);  P & p = (u & (2^29-1)) * 2^32 + lo32(t);  P >> 61 = u >> 29
  uint64_t low = ((uint64_t)(lo32(u) & kMask29) << 32) | lo32(t);
  // keep low as one register pair: the low word is already in t's pair, so
  // forming it costs only the mask; without this the adds get reassociated
  // around extra moves when two keys' steps are interleaved
  asm volatile("" : "+v"(low));
  uint64_t r = low + (u >> 29);
  return F61{lo32(r), hi32(r)};
}
__device__ __forceinline__ F61 p61_step_x32(F61 y, uint32_t x, F61 a) { return p61_step_x32(y, x, a.w0, a.w1); }

// A Horner step that folds at bit 64 instead of bit 61: for y < 2^64 and
// x < 2^32, P = y*x + a < 2^96 + 2^61 has P >> 64 < 2^32, and 2^64 = 8 (mod p),
// so P = (P mod 2^64) + 8 * (P >> 64) (mod p), one v_mad_u64_u32.  The two
// partial products A = y0*x + a0 and B = y1*x + a1 are independent; P mod 2^64
// is A with lo32(B) added to its high word (v_add_co_u32, in place, so the
// pair needs no move) and P >> 64 is hi32(B) plus that carry
// (v_addc_co_u32): five instructions and no register move, where adding
// hi32(A) into B first costs four and two moves to pair the words.  The sum is
// exact unless it carries out of 64 bits (then the result is 8 short modulo
// p); the instruction's carry-out lane mask is or-ed into `carry`, which the
// caller tests once per tile (a carry needs P mod 2^64 >= 2^64 - 2^35: about
// one lane-step in 2^30) and then recomputes with the exact steps.  The result
// is any 64-bit value.
__device__ __forceinline__ F61 p61_step_x32_lazy(F61 y, uint32_t x, F61 a, uint64_t& carry) {
  const uint64_t A = mad64(y.w0, x, a.w0);  // y0 x + a0 < 2^64
  const uint64_t B = mad64(y.w1, x, a.w1);  // y1 x + a1 < 2^64 - 2^32
  // P = A + 2^32 B: P mod 2^64 = A + 2^32 lo32(B) (mod 2^64), whose carry goes
  // into P >> 64 = hi32(B) + carry (< 2^32)
  uint32_t mid = hi32(A), top;
  asm("v_add_co_u32 %0, vcc, %0, %2\n\tv_addc_co_u32 %1, vcc, 0, %3, vcc"
      : "+v"(mid), "=v"(top)
      : "v"(lo32(B)), "v"(hi32(B))
      : "vcc");
  const uint64_t low = ((uint64_t)mid << 32) | lo32(A);  // P mod 2^64
  uint64_t r, c;
  asm("v_mad_u64_u32 %0, %1, %2, 8, %3" : "=&v"(r), "=s"(c) : "v"(top), "v"(low));
  carry |= c;
  return F61{lo32(r), hi32(r)};
}

// The low word of h = v mod p, given r = the last Horner step's fold of
// y*x + a_0 + 1 (that step run with a_lo = a_0's low limb + 1).  r is congruent
// to h + 1 with 1 <= r < 2^61 + 2^35 < 2p + 1, so r is h + 1 or h + 1 + p and
// z = r >> 61 tells which; h = r - z*p - 1, whose low word is
// lo32(r) + z - 1 (p = 2^32 - 1 modulo 2^32).  This replaces the final
// reduction (Algorithm 4 for v < 2p) where only the low word is needed.
__device__ __forceinline__ uint32_t p61_lo_from_inc(F61 r) { return r.w0 + (r.w1 >> 29) - 1u; }

// The last Horner step for y < 2^64 (what p61_step_x32_lazy returns) and
// x < 2^32, giving the low word of h = P mod p for P = y*x + a (a < p) with
// neither a fold nor a final reduction: P < 2^96, so P >> 61 < 2^35, and when
// the bits 32..60 of P are below kP61LastGuard, P mod 2^61 < 2^61 - 2^35 and
// the folded sum (P mod 2^61) + (P >> 61) is at most 2^61 - 2 < p, that is h
// itself; its low word is lo32(P) + lo32(P >> 61) modulo 2^32 (one
// v_alignbit_b32 and one add).  `bits` receives bits 32..60 of P: a lane
// where they reach kP61LastGuard (about one in 2^26) is one the caller must
// recompute with the exact steps.
constexpr uint32_t kP61LastGuard = kMask29 - 7u;  // 0x1ffffff8: P mod 2^61 >= 2^61 - 2^35
__device__ __forceinline__ uint32_t p61_last_lo(F61 y, uint32_t x, F61 a, uint32_t& bits) {
  const uint64_t t = mad64(y.w0, x, a.w0);                      // < 2^64
  const uint64_t u = mad64(y.w1, x, (uint64_t)hi32(t) + a.w1);  // P >> 32 < 2^64
  bits = lo32(u) & kMask29;
  return lo32(t) + funnel(hi32(u), lo32(u), 29);
}

// One Horner step for a key x < 2^60 (two-limb key).  Preconditions: y < 2p,
// x < 2^60, a < p, so P = y*x + a < p^2 (Algorithm 1's invariant) and the
// fold gives a value < 2p.
__device__ __forceinline__ F61 p61_step_x64(F61 y, uint32_t x0, uint32_t x1, F61 a) {
  uint64_t t = mad64(y.w0, x0, a.w0);
  uint32_t p0 = lo32(t);
  uint64_t t1 = mad64(y.w0, x1, (uint64_t)hi32(t) + a.w1);  // < 2^60 + 2^33
  uint64_t u1 = mad64(y.w1, x0, lo32(t1));
  uint32_t p1 = lo32(u1);
  uint64_t t2 = mad64(y.w1, x1, (uint64_t)hi32(t1) + hi32(u1));  // < 2^58 + 2^33
  uint32_t p2 = lo32(t2), p3 = hi32(t2);
  // P = p0 + p1 2^32 + p2 2^64 + p3 2^96 (< 2^122).  P >> 61 = (p3:p2:p1) >> 29.
  uint32_t h0 = funnel(p2, p1, 29), h1 = funnel(p3, p2, 29);
  uint64_t low = ((uint64_t)(p1 & kMask29) << 32) | p0;
  uint64_t r = low + (((uint64_t)h1 << 32) | h0);
  return F61{lo32(r), hi32(r)};
}

// Final reduction of y < 2p to y mod p without a branch (Algorithm 4
// specialised to v < 2p: z = floor(v/p) = (v+1) >> 61 in {0,1}; v mod p =
// (v + z) & p).  Returns the full 61-bit value.
__device__ __forceinline__ uint64_t p61_final(F61 y) {
  uint64_t v = ((uint64_t)y.w1 << 32) | y.w0;
  uint64_t z = (v + 1) >> 61;
  return (v + z) & kP61;
}

// The low 32 bits of p61_final(y): (v + z) & p agrees with v + z below bit 61.
__device__ __forceinline__ uint32_t p61_final_lo(F61 y) {
  const uint64_t v = ((uint64_t)y.w1 << 32) | y.w0;
  return y.w0 + (uint32_t)((v + 1) >> 61);
}

// Algorithm 4 for b = 61 and v < 2^122: z = floor(v/p), y = v mod p.
__device__ __forceinline__ void p61_divmod(uint64_t v_lo, uint64_t v_hi, uint64_t& q, uint64_t& r) {
  unsigned __int128 v = ((unsigned __int128)v_hi << 64) | v_lo;
  unsigned __int128 v1 = v + 1;
  unsigned __int128 z = ((v1 >> 61) + v1) >> 61;
  q = (uint64_t)z;
  r = (uint64_t)((v + z) & kP61);
}

// ---------------------------------------------------------------------------
// p = 2^89 - 1.  Values are three limbs (w2 < 2^26 while y < 2p).
// ---------------------------------------------------------------------------
struct F89 {
  uint32_t w0, w1, w2;
};

// One Horner step y <- fold(y*x + a) for a 64-bit key x = (x1:x0).
// Preconditions: y < 2p, a < p: P = y*x + a < p^2 (p >= 2u - 1 with u = 2^64),
// P < 2^154 in five limbs; the fold leaves (P mod 2^89) + (P >> 89) < 2p.
// a_lo is the coefficient's low limb (or that plus one, <= 2^32), as in
// p61_step_x32; y*x + a + 1 <= p^2 keeps the bound.
__device__ __forceinline__ F89 p89_step(F89 y, uint32_t x0, uint32_t x1, F89 a, uint64_t a_lo) {
  uint64_t t = mad64(y.w0, x0, a_lo);
  uint32_t p0 = lo32(t);
  t = mad64(y.w0, x1, (uint64_t)hi32(t) + a.w1);  // <= 2^64 - 2^33 + 1 + 2^33 - 2
  uint64_t u = mad64(y.w1, x0, lo32(t));
  uint32_t p1 = lo32(u);
  uint64_t c = (uint64_t)hi32(t) + hi32(u);        // < 2^33
  t = mad64(y.w1, x1, c);                          // <= 2^64 - 1
  u = mad64(y.w2, x0, (uint64_t)lo32(t) + a.w2);   // y.w2 < 2^26
  uint32_t p2 = lo32(u);
  c = (uint64_t)hi32(t) + hi32(u);
  t = mad64(y.w2, x1, c);
  uint32_t p3 = lo32(t), p4 = hi32(t);
  // P >> 89 = (p4:p3:p2) >> 25
  uint32_t h0 = funnel(p3, p2, 25), h1 = funnel(p4, p3, 25), h2 = p4 >> 25;
  uint64_t s = (uint64_t)p0 + h0;
  uint32_t r0 = lo32(s);
  s = (uint64_t)p1 + h1 + hi32(s);
  uint32_t r1 = lo32(s);
  uint32_t r2 = (p2 & kMask25) + h2 + hi32(s);
  return F89{r0, r1, r2};
}

__device__ __forceinline__ F89 p89_step(F89 y, uint32_t x0, uint32_t x1, F89 a) { return p89_step(y, x0, x1, a, a.w0); }

// The low word of h = v mod p from r = the last step's fold of y*x + a_0 + 1,
// as p61_lo_from_inc: 1 <= r < 2^89 + 2^65 < 2p + 1, z = r >> 89 in {0, 1}.
__device__ __forceinline__ uint32_t p89_lo_from_inc(F89 r) { return r.w0 + (r.w2 >> 25) - 1u; }

// The last Horner step without a fold, as p61_last_lo: for y < 2p and a < p,
// P = y*x + a < 2^154 has P >> 89 < 2^65, so when bits 64..88 of P are below
// kP89LastGuard, P mod 2^89 < 2^89 - 2^65 and (P mod 2^89) + (P >> 89) is at
// most 2^89 - 2 < p, that is h itself, whose low word is lo32(P) + lo32(P >> 89).
// `bits` receives bits 64..88 of P; a lane where they reach the bound (about
// one in 2^24) is one the caller must finish with the fold (p89_step).
constexpr uint32_t kP89LastGuard = kMask25 - 1u;  // 2^25 - 2: P mod 2^89 >= 2^89 - 2^65
__device__ __forceinline__ uint32_t p89_last_lo(F89 y, uint32_t x0, uint32_t x1, F89 a, uint32_t& bits) {
  uint64_t t = mad64(y.w0, x0, a.w0);
  const uint32_t p0 = lo32(t);
  t = mad64(y.w0, x1, (uint64_t)hi32(t) + a.w1);
  uint64_t u = mad64(y.w1, x0, lo32(t));
  uint64_t c = (uint64_t)hi32(t) + hi32(u);
  t = mad64(y.w1, x1, c);
  u = mad64(y.w2, x0, (uint64_t)lo32(t) + a.w2);
  const uint32_t p2 = lo32(u);
  c = (uint64_t)hi32(t) + hi32(u);
  const uint32_t p3 = lo32(mad64(y.w2, x1, c));
  bits = p2 & kMask25;
  return p0 + funnel(p3, p2, 25);  // lo32(P) + lo32(P >> 89)
}

// y < 2p -> y mod p, branch-free (z = (y+1) >> 89 in {0,1}; (y+z) & p).
__device__ __forceinline__ F89 p89_final(F89 y) {
  uint64_t s = (uint64_t)y.w0 + 1;
  s = (uint64_t)y.w1 + hi32(s);
  uint32_t z = (y.w2 + hi32(s)) >> 25;  // bit 89 of y + 1
  s = (uint64_t)y.w0 + z;
  uint32_t r0 = lo32(s);
  s = (uint64_t)y.w1 + hi32(s);
  uint32_t r1 = lo32(s);
  uint32_t r2 = (y.w2 + hi32(s)) & kMask25;
  return F89{r0, r1, r2};
}

// Algorithm 4 for b = 89 and v < 2^178 given as limbs (v0, v1, v2):
// q = floor(v/p) (< 2^90, two limbs), r = v mod p (two limbs).
__device__ __forceinline__ void p89_divmod(uint64_t v0, uint64_t v1, uint64_t v2, uint64_t& q0,
                                           uint64_t& q1, uint64_t& r0, uint64_t& r1) {
  typedef unsigned __int128 u128;
  const u128 p = (((u128)1) << 89) - 1;
  u128 lo = ((u128)v1 << 64) | v0;
  // v' = v + 1
  u128 lo1 = lo + 1;
  uint64_t hi1 = v2 + (lo1 == 0 ? 1 : 0);
  // s = v' >> 89  (hi1 < 2^50, so hi1 << 39 < 2^89)
  u128 s = ((u128)hi1 << 39) | (lo1 >> 89);
  // w = s + v'  (192 bits) ; z = w >> 89
  u128 wlo = lo1 + s;
  uint64_t whi = hi1 + (wlo < s ? 1 : 0);
  u128 z = ((u128)whi << 39) | (wlo >> 89);
  u128 r = (lo + z) & p;  // only the low 89 bits of v + z matter
  q0 = (uint64_t)z;
  q1 = (uint64_t)(z >> 64);
  r0 = (uint64_t)r;
  r1 = (uint64_t)(r >> 64);
}

// ---------------------------------------------------------------------------
// p = 2^64 - c, c = 59 (pseudo-Mersenne).  Algorithm 5 with three steps
// (m = 3 covers v < (2^64/59)^3 > 2^174), then Algorithm 6 for the remainder.
// For v < p * 2^64 every intermediate z*c + v' stays below 2^128.
// ---------------------------------------------------------------------------
constexpr uint64_t kC59 = 59;

__device__ __forceinline__ void p64c_divmod(uint64_t v_lo, uint64_t v_hi, uint64_t& q, uint64_t& r) {
  typedef unsigned __int128 u128;
  u128 v = ((u128)v_hi << 64) | v_lo;
  u128 v1 = v + kC59;
  u128 z = v1 >> 64;
  z = ((u128)(uint64_t)z * kC59 + v1) >> 64;
  z = ((u128)(uint64_t)z * kC59 + v1) >> 64;
  q = (uint64_t)z;
  r = v_lo + q * kC59;  // Algorithm 6: (v + z c) mod 2^64
}

}  // namespace mcs
