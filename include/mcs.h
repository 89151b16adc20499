/*
 * mcs.h -- C ABI of the MI355X (gfx950) library for k-universal polynomial
 * hashing over Mersenne prime fields and Count Sketch second-moment
 * estimation, after Ahle, Knudsen and Thorup, "The Power of Hashing with
 * Mersenne Primes" (arXiv 2008.08654).
 *
 * Every compute step runs in the library's HIP kernels.  Pointers marked
 * "device" are device memory owned by the caller (for example torch tensors);
 * they must stay valid until the work enqueued on `stream` has finished.
 * Pointers marked "host" are ordinary host memory.  Calls never throw; each
 * returns a cs_status and, on error, leaves a message for cs_last_error().
 * Argument errors are detected on the host before anything is enqueued.
 */
#ifndef MCS_H
#define MCS_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CS_OK = 0,
  CS_EINVAL = -1,     /* bad argument; nothing was enqueued */
  CS_ENOMEM = -2,     /* device or pinned-host allocation failed */
  CS_EDOMAIN = -3,    /* an input was outside the domain the method requires (sticky) */
  CS_EOVERFLOW = -4,  /* an estimate does not fit in int64 (sticky) */
  CS_EDEVICE = -5,    /* a HIP runtime call failed */
  CS_EBUSY = -6       /* resource budget exhausted (serving runtime) */
} cs_status;

/* Primes.  Sketches use the Mersenne primes; 2^64-59 is for quotient and
 * remainder only (the two-for-one analysis is specific to Mersenne primes,
 * Sections 1.2.1 and 1.4). */
typedef enum {
  CS_P61 = 1,    /* p = 2^61 - 1 */
  CS_P89 = 2,    /* p = 2^89 - 1 */
  CS_P64_59 = 3  /* p = 2^64 - 59 (pseudo-Mersenne, Section 1.5) */
} cs_prime;

/* How a row's bucket i(x) in [m] (m = 2^l) and sign s(x) are obtained.
 * Sign bit a gives s = 1 - 2a (Algorithm 3). */
typedef enum {
  CS_TWO_FOR_ONE = 0,     /* one hash h per row: a = bit 0 of h, i = bits 1..l of h */
  CS_TWO_FOR_ONE_MSB = 1, /* Algorithm 3 as printed: i = low l bits, a = top bit b-1 */
  CS_TWO_POLY = 2,        /* two independent hashes per row: i = low l bits of h1, a = bit 0 of h2 */
  CS_ARB_R = 3            /* any bucket count r, Algorithm 8 (Section 3.3): with h' = h + 1,
                             i = floor(r * (h' mod 2^(b-1)) / 2^(b-1)), a = bit b-1 of h' */
} cs_mode;

typedef enum { CS_U32 = 0, CS_U64 = 1, CS_I32 = 2, CS_I64 = 3 } cs_dtype;

typedef struct cs_sketch cs_sketch; /* opaque, library-owned */

/* ---------------------------------------------------------------------------
 * Sketch lifetime.  Count Sketch, Algorithm 2 ("Initialize"), with `rows`
 * independent rows of `buckets` int64 counters each (the median over rows is
 * the concentration step of Section 1.3.1), and per row a uniformly random
 * degree-(k-1) polynomial over Z_p (Section 1.2), k = 4 by default.
 *
 *   rows     >= 1
 *   buckets  = 2^l; l <= b-1 for the two-for-one modes (sign bit and bucket
 *            bits must be distinct: premise of Lemma remove-si), l <= b for
 *            CS_TWO_POLY; in every mode l <= 30.  CS_ARB_R takes any count r in
 *            [2, 2^30]; its table rows are then padded to the next power of
 *            two (the padding counters stay zero)
 *   prime    CS_P61 or CS_P89
 *   seed     expanded with SplitMix64 into coefficients uniform in [p]
 *            (p61: low 61 bits of a draw, draws equal to p rejected; p89: one
 *            draw for the low 64 bits and the low 25 bits of the next for the
 *            high part, values >= p rejected), in row / polynomial / a_0..a_{k-1}
 *            order (polynomial 0 gives the bucket, 1 the sign in CS_TWO_POLY)
 *   k        number of coefficients per polynomial: 2, 4 or 8
 * The counter table and coefficients live on the current HIP device and are
 * owned by the sketch.  The table starts at zero.
 * ------------------------------------------------------------------------- */
cs_status cs_create(uint32_t rows, uint64_t buckets, cs_prime prime, uint64_t seed,
                    cs_sketch** out);
cs_status cs_create_ex(uint32_t rows, uint64_t buckets, cs_prime prime, uint64_t seed,
                       cs_mode mode, uint32_t k, cs_sketch** out);
/* Same with explicit coefficients (host): rows*npoly*k values, each < p; for
 * CS_P89 each value is two little-endian uint64 limbs. */
cs_status cs_create_with_coeffs(uint32_t rows, uint64_t buckets, cs_prime prime, cs_mode mode,
                                uint32_t k, const uint64_t* coeffs, cs_sketch** out);
/* Waits for the sketch's work and frees it.  NULL is accepted. */
void cs_destroy(cs_sketch* s);

/* Workspace.  The two-pass update path (BINNED) runs in rounds of at most
 * 2^27 keys through a workspace the sketch owns: records and group offsets
 * of the round, 4 * rows * (1 + about 1/16) bytes per key.  cs_create and
 * cs_set_update_path reserve one for rounds of 2^20 keys when the sketch's
 * path needs it; cs_reserve grows it to rounds of `keys` keys (fewer, larger
 * rounds).  cs_update never allocates: it runs as many rounds as its n needs
 * over the workspace it finds.  cs_reserve waits for the device before it
 * replaces a workspace.  Paths without a workspace reserve nothing. */
cs_status cs_reserve(cs_sketch* s, uint64_t keys);

/* ---------------------------------------------------------------------------
 * cs_update -- Algorithm 2 "Process(x, D)" for a batch: for every i < n and
 * every row j, C[j][i_j(x_i)] += s_j(x_i) * D_i, with int64 two's-complement
 * wrap-around.  Each i_j, s_j comes from Algorithm 1 (Horner over p with lazy
 * Mersenne reduction) plus a branch-free final reduction (Algorithm 4), then
 * the bucket/sign split of the sketch's mode.
 *   keys     device, n values of key_type (CS_U32 or CS_U64)
 *   weights  device, n values of weight_type (CS_I32 or CS_I64)
 * Key domain: for CS_P61 keys must be < 2^60 (Algorithm 1 requires
 * p >= 2u - 1); a larger key sets the sketch's sticky CS_EDOMAIN flag, which
 * the next synchronising call (cs_estimate_f2, cs_read_counters, cs_sync)
 * returns; the counters are then meaningless.  n = 0 is a no-op.
 * The work is enqueued on `stream` (0 = default stream) and the call returns
 * without waiting.  Every call on a sketch (update, reset, merge, estimate,
 * reads) must be ordered with the others, for example by issuing them all on
 * one stream: calls on different streams that overlap in time race on the
 * counters and on the update's workspace, and give undefined counters.
 * ------------------------------------------------------------------------- */
cs_status cs_update(cs_sketch* s, const void* keys, cs_dtype key_type, const void* weights,
                    cs_dtype weight_type, uint64_t n, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * cs_estimate_f2 -- Algorithm 2 "Output" per row, X_j = sum_i C[j][i]^2
 * (exact, accumulated in 128 bits), and the median over rows (element
 * (rows-1)/2 of the sorted X_j).  Writes the median to *f2 (host) and, if
 * rows_out (host) is not NULL, the `rows` values X_j.  Synchronises `stream`.
 * Returns CS_EOVERFLOW if some X_j >= 2^63 (that X_j reads INT64_MAX; this
 * concerns the call only, the counters stay valid), or a pending sticky
 * error (CS_EDOMAIN), which takes precedence.
 * ------------------------------------------------------------------------- */
cs_status cs_estimate_f2(cs_sketch* s, int64_t* f2, int64_t* rows_out, hipStream_t stream);

/* Point query f_x ~ median_j s_j(x) C[j][i_j(x)] (Section 1.3.1), for n keys:
 * out (device) gets n int64 estimates.  Enqueued on `stream`. */
cs_status cs_query(cs_sketch* s, const void* keys, cs_dtype key_type, uint64_t n, int64_t* out,
                   hipStream_t stream);

/* Update paths.  AUTO picks LDS when the whole table (rows*buckets*8 bytes)
 * fits in 64 KiB; else GLOBAL when the call has fewer than buckets/8 keys
 * (fewer adds than a per-block copy of the table would clear and flush); else
 * ROWS when a row has at most 2^16 buckets (each block
 * holds the rows of one row group in LDS as 16-bit fields, whose rare wraps
 * are carried into the int64 table exactly); else BINNED (two passes through
 * a library-owned workspace); else GLOBAL (one device-scope atomic per key and
 * row).  BINNED first combines repeated keys within each tile of keys (the
 * sketch is linear, so C[i(x)] += s(x) * (sum of their weights) is the same
 * update); BINNED_NOCOMBINE skips that step.  All paths give identical
 * counters; forcing one is for testing and tuning. */
enum { CS_PATH_AUTO = 0, CS_PATH_LDS = 1, CS_PATH_GLOBAL = 2, CS_PATH_BINNED = 3, CS_PATH_BINNED_NOCOMBINE = 4,
       CS_PATH_ROWS = 5 };
cs_status cs_set_update_path(cs_sketch* s, int path);

/* Copies the rows*buckets counters (row-major, no padding) to host memory;
 * synchronises. */
cs_status cs_read_counters(cs_sketch* s, int64_t* host_dst, hipStream_t stream);
/* Device pointer to the counter table (rows rows of int64, row-major, row
 * pitch = buckets rounded up to a power of two), owned by the sketch; valid
 * until cs_destroy. */
cs_status cs_table_device(cs_sketch* s, int64_t** dev_table);
/* Copies the coefficients (layout as in cs_create_with_coeffs) to host. */
cs_status cs_read_coeffs(cs_sketch* s, uint64_t* host_dst);
/* Shape queries. */
cs_status cs_info(const cs_sketch* s, uint32_t* rows, uint64_t* buckets, cs_prime* prime,
                  cs_mode* mode, uint32_t* k);
/* Zeroes the counters and clears sticky flags (enqueued on `stream`). */
cs_status cs_reset(cs_sketch* s, hipStream_t stream);
/* dst += src for two sketches with identical shape and coefficients (the
 * sketch is linear, Section 1.3.1).  Enqueued on `stream`. */
cs_status cs_merge(cs_sketch* dst, const cs_sketch* src, hipStream_t stream);
/* Waits for `stream` and returns any sticky error of the sketch. */
cs_status cs_sync(cs_sketch* s, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Quotient and remainder by p for a batch (Section 1.5 and Section 4):
 *   CS_P61:    Algorithm 4 (b = 61); x has 2 uint64 limbs per value, x < 2^122;
 *              quot and rem have 1 limb per value.
 *   CS_P89:    Algorithm 4 (b = 89); x has 3 limbs, x < 2^178; quot and rem 2 limbs.
 *   CS_P64_59: Algorithm 5 with c = 59 and three steps (enough for every
 *              x < 2^128 by Theorem simple-div) and Algorithm 6; x has 2 limbs,
 *              x < p*2^64 (so the quotient fits one limb); quot and rem 1 limb.
 * Limbs are little-endian uint64.  x, quot and rem are device pointers; quot
 * or rem may be NULL to skip that output.  Two-limb arrays (x for CS_P61 and
 * CS_P64_59, quot and rem for CS_P89) must be 16-byte aligned (CS_EINVAL).  A value outside the domain sets a
 * device flag that the call returns as CS_EDOMAIN on the next
 * mersenne_status call (outputs for such values are unspecified).  Enqueued
 * on `stream`.
 * ------------------------------------------------------------------------- */
cs_status mersenne_divmod(cs_prime prime, const uint64_t* x, uint64_t n, uint64_t* quot,
                          uint64_t* rem, hipStream_t stream);
cs_status mersenne_div(cs_prime prime, const uint64_t* x, uint64_t n, uint64_t* quot,
                       hipStream_t stream);
cs_status mersenne_mod(cs_prime prime, const uint64_t* x, uint64_t n, uint64_t* rem,
                       hipStream_t stream);
/* Comparator with the same contract: the compiler's wide `/` and `%`
 * (CS_P89: shift-and-subtract long division). */
cs_status mersenne_divmod_naive(cs_prime prime, const uint64_t* x, uint64_t n, uint64_t* quot,
                                uint64_t* rem, hipStream_t stream);
/* Most uniform maps of hash values v in [p] to [r] buckets (Section 1.4, Lemma
 * most-uniform; for 2^64-59 the note on bucket counts in Section 1.5):
 *   CS_MAP_EXACT:    floor(v * r / p) by the branch-free division of
 *                    Algorithm 4 (Mersenne) or Algorithms 5 and 6 (2^64-59);
 *   CS_MAP_MERSENNE: floor((v + 1) * r / 2^b), eq. most-uniform (Mersenne
 *                    primes only).
 *   v    device; one uint64 per value (CS_P61, CS_P64_59) or two limbs
 *        (CS_P89, 16-byte aligned); each v < p, else the domain flag is set
 *        (mersenne_status)
 *   r    1 <= r < 2^32
 *   out  device, n uint32 buckets
 * Enqueued on `stream`. */
enum { CS_MAP_EXACT = 0, CS_MAP_MERSENNE = 1 };
cs_status mersenne_bucket_map(cs_prime prime, int method, const uint64_t* v, uint64_t n, uint64_t r, uint32_t* out,
                              hipStream_t stream);

/* Wide quotient and remainder (the division experiment of Section 5): every x of
 * 2b bits divided by p = 2^b - c, for b in {32, 64, 128, 256, 512, 1024} and
 * 1 <= c < min(2^31, 2^(b/2)).
 *   CS_WIDE_ALG5: Algorithm 5 with m = ceil(2b / (b - ceil(log2 c))) steps (2 for
 *                 c = 1; Theorem simple-div), then Algorithm 6
 *   CS_WIDE_CCH:  the Crandall-Chung-Hasan algorithm (Algorithm 10), the paper's
 *                 comparator
 * Values are limb planes of uint32: limb j (bits 32j..32j+31) of value i at
 * x[j*n + i].  x: device, 2b/32 planes; quot: device, b/32 + 1 planes; rem:
 * device, b/32 planes; quot or rem may be NULL.  Every x < 2^(2b) is in the
 * domain.  Enqueued on `stream`. */
enum { CS_WIDE_ALG5 = 0, CS_WIDE_CCH = 1 };
cs_status mersenne_divmod_wide(uint32_t b, uint32_t c, int method, const uint32_t* x, uint64_t n, uint32_t* quot,
                               uint32_t* rem, hipStream_t stream);

/* Synchronises `stream` and returns (and clears) the domain flag of the
 * quotient/remainder calls on the current device. */
cs_status mersenne_status(hipStream_t stream);

/* The status the library reports for a HIP runtime error code (a hipError_t
 * value): CS_OK for success, CS_ENOMEM for an out-of-memory error, CS_EDEVICE
 * for every other error (for example a fault left behind by an earlier kernel,
 * which later runtime calls keep returning).  Needs no device. */
cs_status cs_status_from_hip_error(int hip_error);

/* Message for the last error on the calling thread ("" if none). */
const char* cs_last_error(void);
/* Library version string. */
const char* cs_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MCS_H */
