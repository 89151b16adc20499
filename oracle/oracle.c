/*
 * Oracle for "The Power of Hashing with Mersenne Primes" (Ahle, Knudsen, Thorup,
 * arXiv 2008.08654) -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct CPU statement of what the GPU library
 * computes. Only the test-suite, the smoke check and the benchmark's CPU
 * baseline may load this file. It shares no code with the GPU library: it
 * uses no Mersenne folding and no branch-free division (those are what the
 * GPU library is tested for); every reduction below is the compiler's own
 * unsigned __int128 `%` and `/`, or textbook long division built on them.
 *
 * Conventions
 *   - Coefficients of one polynomial are stored a_0, a_1, ..., a_{k-1}
 *     (a_i multiplies x^i), Section 1.2.
 *   - Coefficient arrays are row-major: row j, then polynomial q (bucket
 *     polynomial before sign polynomial in the two-polynomial mode), then
 *     a_0..a_{k-1}.  An 89-bit value is two little-endian 64-bit limbs.
 *   - Counter tables are int64[rows][m], row-major; additions wrap mod 2^64
 *     (two's complement), done in uint64_t to avoid signed overflow.
 *
 * Status codes mirror the library's: 0 ok, -1 invalid argument,
 * -3 key outside the domain, -4 F2 does not fit in int64.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;
typedef __int128 i128;

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_EDOMAIN (-3)
#define ORC_EOVERFLOW (-4)

enum { ORC_TWO_FOR_ONE = 0, ORC_TWO_FOR_ONE_MSB = 1, ORC_TWO_POLY = 2, ORC_ARB_R = 3 };

/* ------------------------------------------------------------------------ */
/* Seed expansion: SplitMix64 (Steele, Lea and Flood, OOPSLA 2014), the     */
/* generator the paper does not fix; the library implements it separately. */
/* ------------------------------------------------------------------------ */
uint64_t orc_splitmix64(uint64_t* state) {
  uint64_t z;
  *state += 0x9e3779b97f4a7c15ULL;
  z = *state;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

/* count coefficients uniform in [2^61-1]: low 61 bits of a draw, draws equal
 * to p rejected (uniform vector of Section 1.2). */
void orc_coeffs_p61(uint64_t seed, uint64_t count, uint64_t* out) {
  const uint64_t p = (1ULL << 61) - 1;
  uint64_t st = seed;
  for (uint64_t i = 0; i < count; ++i) {
    uint64_t v;
    do { v = orc_splitmix64(&st) & p; } while (v == p);
    out[i] = v;
  }
}

/* count coefficients uniform in [2^89-1]: a draw gives the low 64 bits, the
 * next draw's low 25 bits give the high part; values >= p rejected. */
void orc_coeffs_p89(uint64_t seed, uint64_t count, uint64_t* out /* 2 limbs each */) {
  uint64_t st = seed;
  const u128 p = (((u128)1) << 89) - 1;
  for (uint64_t i = 0; i < count; ++i) {
    u128 v;
    do {
      uint64_t lo = orc_splitmix64(&st);
      uint64_t hi = orc_splitmix64(&st) & ((1ULL << 25) - 1);
      v = ((u128)hi << 64) | lo;
    } while (v >= p);
    out[2 * i] = (uint64_t)v;
    out[2 * i + 1] = (uint64_t)(v >> 64);
  }
}

/* ------------------------------------------------------------------------ */
/* Hash, Section 1.2: h_a(x) = sum_i a_i x^i mod p, by Horner's rule with a  */
/* full reduction (`%`) after every multiply-add.  Valid for any p < 2^63.  */
/* ------------------------------------------------------------------------ */
uint64_t orc_hash_small(uint64_t p, const uint64_t* a, uint32_t k, uint64_t x) {
  u128 y = a[k - 1] % p;
  u128 xr = x % p;
  for (int i = (int)k - 2; i >= 0; --i) y = (y * xr + a[i]) % p;
  return (uint64_t)y;
}

/* Long division of a multi-limb number by an odd modulus p < 2^96, in base
 * 2^32 (schoolbook, one digit at a time), each step a u128 `/` and `%`.
 * limbs are 64-bit little-endian; returns the remainder, *quot gets the
 * quotient (the caller guarantees it fits in 128 bits). */
static u128 longdiv(const uint64_t* limbs, int nlimbs, u128 p, u128* quot) {
  u128 r = 0, q = 0;
  for (int i = nlimbs - 1; i >= 0; --i) {
    for (int half = 1; half >= 0; --half) {
      uint64_t digit = (limbs[i] >> (32 * half)) & 0xffffffffULL;
      u128 cur = (r << 32) | digit; /* r < p < 2^96, so cur < 2^128 */
      q = (q << 32) | (cur / p);
      r = cur % p;
    }
  }
  if (quot) *quot = q;
  return r;
}

/* product of a < 2^128 and x < 2^64 as three 64-bit limbs (schoolbook) */
static void mul_128_64(u128 a, uint64_t x, uint64_t out[3]) {
  u128 lo = (u128)(uint64_t)a * x;
  u128 hi = (u128)(uint64_t)(a >> 64) * x;
  u128 mid = (lo >> 64) + (uint64_t)hi;
  out[0] = (uint64_t)lo;
  out[1] = (uint64_t)mid;
  out[2] = (uint64_t)(hi >> 64) + (uint64_t)(mid >> 64);
}

/* The same Horner evaluation over p = 2^89 - 1 (64-bit keys; the products
 * reach about 2^153, so each step is a 3-limb long division). */
void orc_hash_p89(const uint64_t* a /* k x 2 limbs */, uint32_t k, uint64_t x, uint64_t out[2]) {
  const u128 p = (((u128)1) << 89) - 1;
  u128 y = (((u128)a[2 * (k - 1) + 1] << 64) | a[2 * (k - 1)]) % p;
  for (int i = (int)k - 2; i >= 0; --i) {
    uint64_t prod[3];
    u128 ai = ((u128)a[2 * i + 1] << 64) | a[2 * i];
    mul_128_64(y, x, prod);
    /* add a_i < 2^89 into the 3-limb product */
    u128 s0 = (u128)prod[0] + (uint64_t)ai;
    u128 s1 = (u128)prod[1] + (uint64_t)(ai >> 64) + (uint64_t)(s0 >> 64);
    prod[0] = (uint64_t)s0;
    prod[1] = (uint64_t)s1;
    prod[2] += (uint64_t)(s1 >> 64);
    y = longdiv(prod, 3, p, NULL);
  }
  out[0] = (uint64_t)y;
  out[1] = (uint64_t)(y >> 64);
}

/* ------------------------------------------------------------------------ */
/* Bucket and sign from hash values.                                        */
/*  TWO_FOR_ONE:     sign bit = bit 0 of h, bucket = bits 1..l of h         */
/*                   (selecting distinct bits, Section 1.2.1);              */
/*  TWO_FOR_ONE_MSB: Algorithm 3 as printed: bucket = low l bits, sign bit  */
/*                   = bit b-1 (the top bit of the b-bit value);            */
/*  TWO_POLY:        bucket = low l bits of h1, sign bit = bit 0 of h2      */
/*                   (h^r with r = 2^l and r = 2, Section 1.2).             */
/* The sign is s = 1 - 2a for sign bit a (Algorithm 3).                     */
/* h_lo is the low 64 bits of h (enough for every bit used when b <= 64);   */
/* h_top is bit b-1 of h.                                                   */
/* ------------------------------------------------------------------------ */
static void split(int mode, uint64_t m, uint64_t h1_lo, uint32_t h1_top, uint64_t h2_lo,
                  uint64_t* bucket, int* sign) {
  uint32_t a;
  if (mode == ORC_TWO_FOR_ONE) {
    a = (uint32_t)(h1_lo & 1);
    *bucket = (h1_lo >> 1) & (m - 1);
  } else if (mode == ORC_TWO_FOR_ONE_MSB) {
    a = h1_top;
    *bucket = h1_lo & (m - 1);
  } else {
    a = (uint32_t)(h2_lo & 1);
    *bucket = h1_lo & (m - 1);
  }
  *sign = 1 - 2 * (int)a;
}

/* ARB_R, any number r of buckets (Algorithm 8, Section 3.3): with
 * h_x = h(x) + 1 (a b-bit value, never 0), the bucket is
 * floor(r * j / 2^(b-1)) for j = the low b-1 bits of h_x, and the sign bit
 * is bit b-1 of h_x; s = 1 - 2a as the algorithm writes it.  Plain 128-bit
 * arithmetic: h < 2^89 and r < 2^32, so r * j < 2^120. */
static void split_arb(uint32_t b, uint64_t r, u128 h, uint64_t* bucket, int* sign) {
  const u128 hx = h + 1;
  const u128 j = hx & ((((u128)1) << (b - 1)) - 1);
  const uint32_t a = (uint32_t)(hx >> (b - 1)) & 1;
  *bucket = (uint64_t)(((u128)r * j) >> (b - 1));
  *sign = 1 - 2 * (int)a;
}

static int npoly(int mode) { return mode == ORC_TWO_POLY ? 2 : 1; }

/* m must be a power of two 2^l, with l <= b-1 when one hash value supplies
 * both the bucket and the sign bit (the bits must be distinct), l <= b
 * otherwise.  ARB_R takes any 2 <= m <= 2^(b-1) below 2^32. */
static int check_m(uint64_t m, uint32_t b, int mode) {
  if (mode == ORC_ARB_R) return m >= 2 && m < (1ULL << 32) && (b > 33 || m <= (1ULL << (b - 1)));
  if (m == 0 || (m & (m - 1)) != 0) return 0;
  uint32_t l = 0;
  while ((1ULL << l) < m) ++l;
  if (mode == ORC_TWO_POLY) return l <= b;
  return l + 1 <= b;
}

/* Hash key x in row j and return bucket and sign (small-prime / p61 form). */
int orc_bucket_sign_small(uint64_t p, uint32_t b, uint32_t k, int mode, uint64_t m,
                          const uint64_t* coeffs, uint32_t row, uint64_t x,
                          uint64_t* bucket, int* sign) {
  const uint64_t* a = coeffs + (uint64_t)row * npoly(mode) * k;
  uint64_t h1 = orc_hash_small(p, a, k, x);
  if (mode == ORC_ARB_R) {
    split_arb(b, m, h1, bucket, sign);
    return ORC_OK;
  }
  uint64_t h2 = mode == ORC_TWO_POLY ? orc_hash_small(p, a + k, k, x) : 0;
  split(mode, m, h1, (uint32_t)((h1 >> (b - 1)) & 1), h2, bucket, sign);
  return ORC_OK;
}

int orc_bucket_sign_p89(uint32_t k, int mode, uint64_t m, const uint64_t* coeffs, uint32_t row,
                        uint64_t x, uint64_t* bucket, int* sign) {
  const uint64_t* a = coeffs + (uint64_t)row * npoly(mode) * k * 2;
  uint64_t h1[2], h2[2] = {0, 0};
  orc_hash_p89(a, k, x, h1);
  if (mode == ORC_ARB_R) {
    split_arb(89, m, ((u128)h1[1] << 64) | h1[0], bucket, sign);
    return ORC_OK;
  }
  if (mode == ORC_TWO_POLY) orc_hash_p89(a + 2 * k, k, x, h2);
  split(mode, m, h1[0], (uint32_t)((h1[1] >> (88 - 64)) & 1), h2[0], bucket, sign);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Count Sketch, Algorithm 2: Process(x, D): C[i(x)] += s(x) * D, for each  */
/* of `rows` independent rows.  keys/weights are u64/i64.                   */
/* For p = 2^61 - 1 the key domain is x < 2^60 (p >= 2u - 1, Algorithm 1);  */
/* a key outside it returns ORC_EDOMAIN and leaves the table untouched.     */
/* Rows are independent, so they are processed in parallel (OpenMP); each   */
/* counter is written by one thread only.                                   */
/* ------------------------------------------------------------------------ */
int orc_cs_update_small(uint64_t p, uint32_t b, uint32_t k, int mode, uint32_t rows, uint64_t m,
                        const uint64_t* coeffs, const uint64_t* keys, const int64_t* weights,
                        uint64_t n, int64_t* table) {
  if (rows == 0 || k == 0 || mode < 0 || mode > 3 || !check_m(m, b, mode)) return ORC_EINVAL;
  if (p == (1ULL << 61) - 1) {
    for (uint64_t i = 0; i < n; ++i)
      if (keys[i] >= (1ULL << 60)) return ORC_EDOMAIN;
  }
#pragma omp parallel for schedule(dynamic, 1) if (rows > 1)
  for (uint32_t j = 0; j < rows; ++j) {
    uint64_t* row = (uint64_t*)table + (uint64_t)j * m;
    for (uint64_t i = 0; i < n; ++i) {
      uint64_t bucket; int s;
      orc_bucket_sign_small(p, b, k, mode, m, coeffs, j, keys[i], &bucket, &s);
      row[bucket] += (uint64_t)((int64_t)s * weights[i]);
    }
  }
  return ORC_OK;
}

int orc_cs_update_p89(uint32_t k, int mode, uint32_t rows, uint64_t m, const uint64_t* coeffs,
                      const uint64_t* keys, const int64_t* weights, uint64_t n, int64_t* table) {
  if (rows == 0 || k == 0 || mode < 0 || mode > 3 || !check_m(m, 89, mode)) return ORC_EINVAL;
#pragma omp parallel for schedule(dynamic, 1) if (rows > 1)
  for (uint32_t j = 0; j < rows; ++j) {
    uint64_t* row = (uint64_t*)table + (uint64_t)j * m;
    for (uint64_t i = 0; i < n; ++i) {
      uint64_t bucket; int s;
      orc_bucket_sign_p89(k, mode, m, coeffs, j, keys[i], &bucket, &s);
      row[bucket] += (uint64_t)((int64_t)s * weights[i]);
    }
  }
  return ORC_OK;
}

/* Same update with the keys split over threads instead of rows: each thread
 * fills a private table which is then added in (exact: integer addition
 * mod 2^64 does not depend on order).  Used only to time the oracle on many
 * cores when rows < cores. */
int orc_cs_update_small_keypar(uint64_t p, uint32_t b, uint32_t k, int mode, uint32_t rows,
                               uint64_t m, const uint64_t* coeffs, const uint64_t* keys,
                               const int64_t* weights, uint64_t n, int64_t* table, int nthreads) {
  if (rows == 0 || k == 0 || nthreads < 1 || mode < 0 || mode > 3 || !check_m(m, b, mode))
    return ORC_EINVAL;
  if (p == (1ULL << 61) - 1) {
    for (uint64_t i = 0; i < n; ++i)
      if (keys[i] >= (1ULL << 60)) return ORC_EDOMAIN;
  }
  uint64_t cells = (uint64_t)rows * m;
  uint64_t* priv = (uint64_t*)calloc((size_t)nthreads * cells, sizeof(uint64_t));
  if (!priv) return ORC_EINVAL;
#pragma omp parallel for num_threads(nthreads) schedule(static, 1)
  for (int th = 0; th < nthreads; ++th) {
    uint64_t lo = n * (uint64_t)th / (uint64_t)nthreads, hi = n * (uint64_t)(th + 1) / (uint64_t)nthreads;
    uint64_t* mine = priv + (uint64_t)th * cells;
    for (uint64_t i = lo; i < hi; ++i)
      for (uint32_t j = 0; j < rows; ++j) {
        uint64_t bucket; int s;
        orc_bucket_sign_small(p, b, k, mode, m, coeffs, j, keys[i], &bucket, &s);
        mine[(uint64_t)j * m + bucket] += (uint64_t)((int64_t)s * weights[i]);
      }
  }
  for (int th = 0; th < nthreads; ++th)
    for (uint64_t c = 0; c < cells; ++c) ((uint64_t*)table)[c] += priv[(uint64_t)th * cells + c];
  free(priv);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Count Sketch Output (Algorithm 2): X_j = sum_i C[j][i]^2 per row, and    */
/* the median over rows (Section 1.3.1: concentration by a median).  X_j is */
/* exact; a value that does not fit in int64 returns ORC_EOVERFLOW.  Median */
/* of t values: element (t-1)/2 of the sorted values (the lower median).    */
/* ------------------------------------------------------------------------ */
static int cmp_i64(const void* x, const void* y) {
  int64_t a = *(const int64_t*)x, b = *(const int64_t*)y;
  return (a > b) - (a < b);
}

int orc_cs_estimate(const int64_t* table, uint32_t rows, uint64_t m, int64_t* rows_out,
                    int64_t* median) {
  if (rows == 0 || m == 0) return ORC_EINVAL;
  int64_t* vals = (int64_t*)malloc(sizeof(int64_t) * rows);
  int status = ORC_OK;
  for (uint32_t j = 0; j < rows; ++j) {
    u128 acc = 0;
    int over = 0;
    for (uint64_t i = 0; i < m; ++i) {
      int64_t c = table[(uint64_t)j * m + i];
      u128 mag = c < 0 ? (u128)(-(i128)c) : (u128)c;
      u128 sq = mag * mag; /* <= 2^126 */
      acc += sq;
      if (acc > (u128)INT64_MAX) { over = 1; break; }
    }
    if (over) status = ORC_EOVERFLOW;
    vals[j] = over ? INT64_MAX : (int64_t)acc;
    if (rows_out) rows_out[j] = vals[j];
  }
  qsort(vals, rows, sizeof(int64_t), cmp_i64);
  if (median) *median = vals[(rows - 1) / 2];
  free(vals);
  return status;
}

/* Exact second moment of a stream (Section 1.3.1): f_x = sum of D over the
 * occurrences of x, F2 = sum_x f_x^2.  Sort by key, then add up runs.
 * Returns F2 as two's-complement 128 bits (lo, hi). */
typedef struct { uint64_t key; int64_t w; } kw_t;
static int cmp_kw(const void* x, const void* y) {
  uint64_t a = ((const kw_t*)x)->key, b = ((const kw_t*)y)->key;
  return (a > b) - (a < b);
}
int orc_exact_f2(const uint64_t* keys, const int64_t* weights, uint64_t n, uint64_t out[2]) {
  kw_t* v = (kw_t*)malloc(sizeof(kw_t) * (n ? n : 1));
  if (!v) return ORC_EINVAL;
  for (uint64_t i = 0; i < n; ++i) { v[i].key = keys[i]; v[i].w = weights[i]; }
  qsort(v, n, sizeof(kw_t), cmp_kw);
  i128 f2 = 0;
  uint64_t i = 0;
  while (i < n) {
    i128 f = 0;
    uint64_t j = i;
    while (j < n && v[j].key == v[i].key) f += v[j++].w;
    f2 += f * f;
    i = j;
  }
  free(v);
  out[0] = (uint64_t)(u128)f2;
  out[1] = (uint64_t)((u128)f2 >> 64);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Quotient and remainder (Section 1.5 and Section 4): q = floor(x/p) and   */
/* r = x mod p computed with the compiler's division.                       */
/*   prime 1: p = 2^61 - 1,  x < 2^122 given as 2 limbs, q and r 1 limb     */
/*   prime 3: p = 2^64 - 59, x < p*2^64 given as 2 limbs, q and r 1 limb    */
/*   prime 2: p = 2^89 - 1,  x < 2^178 given as 3 limbs, q and r 2 limbs    */
/* An input outside the domain returns ORC_EDOMAIN (outputs not written).   */
/* ------------------------------------------------------------------------ */
int orc_divmod(int prime, const uint64_t* x, uint64_t n, uint64_t* quot, uint64_t* rem) {
  if (prime == 1 || prime == 3) {
    u128 p = prime == 1 ? (u128)((1ULL << 61) - 1) : (u128)(0xFFFFFFFFFFFFFFFFULL - 58);
    for (uint64_t i = 0; i < n; ++i) {
      u128 v = ((u128)x[2 * i + 1] << 64) | x[2 * i];
      if (prime == 1 && (x[2 * i + 1] >> 58) != 0) return ORC_EDOMAIN;
      if (prime == 3 && x[2 * i + 1] >= (uint64_t)p) return ORC_EDOMAIN;
      if (quot) quot[i] = (uint64_t)(v / p);
      if (rem) rem[i] = (uint64_t)(v % p);
    }
    return ORC_OK;
  }
  if (prime == 2) {
    const u128 p = (((u128)1) << 89) - 1;
    for (uint64_t i = 0; i < n; ++i) {
      if ((x[3 * i + 2] >> 50) != 0) return ORC_EDOMAIN;
      u128 q;
      u128 r = longdiv(x + 3 * i, 3, p, &q);
      if (quot) { quot[2 * i] = (uint64_t)q; quot[2 * i + 1] = (uint64_t)(q >> 64); }
      if (rem) { rem[2 * i] = (uint64_t)r; rem[2 * i + 1] = (uint64_t)(r >> 64); }
    }
    return ORC_OK;
  }
  return ORC_EINVAL;
}

/* ------------------------------------------------------------------------ */
/* Maps of a hash value v in [p] to [r] buckets (Section 1.4 and the note on */
/* arbitrary bucket counts in Section 1.5), as plain definitions:           */
/*   exact:    floor(v * r / p)           (most uniform for any p)          */
/*   mersenne: floor((v + 1) * r / 2^b)   (eq. most-uniform, p = 2^b - 1)   */
/* v is given as two little-endian limbs, v < p < 2^89, r < 2^32.  A value  */
/* v >= p returns ORC_EDOMAIN.                                               */
/* ------------------------------------------------------------------------ */
int orc_bucket_map_exact(uint64_t p_lo, uint64_t p_hi, const uint64_t* v, uint64_t n, uint64_t r, uint32_t* out) {
  const u128 p = ((u128)p_hi << 64) | p_lo;
  if (r == 0 || r >= (1ULL << 32) || p < 2 || p_hi >= (1ULL << 25)) return ORC_EINVAL;
  for (uint64_t i = 0; i < n; ++i) {
    const u128 x = ((u128)v[2 * i + 1] << 64) | v[2 * i];
    if (x >= p) return ORC_EDOMAIN;
    out[i] = (uint32_t)((x * r) / p);
  }
  return ORC_OK;
}

int orc_bucket_map_mersenne(uint32_t b, const uint64_t* v, uint64_t n, uint64_t r, uint32_t* out) {
  if (r == 0 || r >= (1ULL << 32) || b < 2 || b > 89) return ORC_EINVAL;
  const u128 p = (((u128)1) << b) - 1;
  for (uint64_t i = 0; i < n; ++i) {
    const u128 x = ((u128)v[2 * i + 1] << 64) | v[2 * i];
    if (x >= p) return ORC_EDOMAIN;
    out[i] = (uint32_t)(((x + 1) * r) >> b);
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Exhaustive enumeration over every coefficient vector a in Z_p^k, for     */
/* the tiny-prime checks of the oracle against the paper's exact            */
/* statements.  Tuple index t = a_0 + p a_1 + p^2 a_2 + ... (a_0 fastest).  */
/* ------------------------------------------------------------------------ */
static int next_tuple(uint64_t* a, uint32_t k, uint64_t p) {
  for (uint32_t i = 0; i < k; ++i) {
    if (++a[i] < p) return 1;
    a[i] = 0;
  }
  return 0;
}

/* out[t * nkeys + i] = h_a(keys[i]) for every tuple t (p^k * nkeys values). */
int orc_enum_hash(uint64_t p, uint32_t k, const uint64_t* keys, uint32_t nkeys, uint64_t* out) {
  uint64_t a[16] = {0};
  if (k == 0 || k > 16) return ORC_EINVAL;
  uint64_t t = 0;
  do {
    for (uint32_t i = 0; i < nkeys; ++i) out[t * nkeys + i] = orc_hash_small(p, a, k, keys[i]);
    ++t;
  } while (next_tuple(a, k, p));
  return ORC_OK;
}

/* Bucket and sign of every key under every coefficient tuple of one row
 * (one polynomial; TWO_FOR_ONE or TWO_FOR_ONE_MSB). */
int orc_enum_bucket_sign(uint64_t p, uint32_t b, uint32_t k, int mode, uint64_t m,
                         const uint64_t* keys, uint32_t nkeys, uint64_t* buckets, int32_t* signs) {
  uint64_t a[16] = {0};
  if (k == 0 || k > 16 || mode == ORC_TWO_POLY || !check_m(m, b, mode)) return ORC_EINVAL;
  uint64_t t = 0;
  do {
    for (uint32_t i = 0; i < nkeys; ++i) {
      uint64_t bk; int s;
      orc_bucket_sign_small(p, b, k, mode, m, a, 0, keys[i], &bk, &s);
      buckets[t * nkeys + i] = bk;
      signs[t * nkeys + i] = s;
    }
    ++t;
  } while (next_tuple(a, k, p));
  return ORC_OK;
}

/* For every coefficient tuple (k values, or 2k in the two-polynomial mode)
 * build a one-row Count Sketch of the stream with orc_cs_update_small and
 * take its estimate X with orc_cs_estimate;
 * return sum_a X and sum_a X^2 exactly (two's complement 128 bits each,
 * lo/hi).  Needs p^k * X^2 < 2^127. */
int orc_enum_estimate_moments(uint64_t p, uint32_t b, uint32_t k, int mode, uint64_t m,
                              const uint64_t* keys, const int64_t* weights, uint64_t n,
                              uint64_t sum_x[2], uint64_t sum_x2[2]) {
  uint64_t a[32] = {0};
  uint32_t ncoef = (uint32_t)npoly(mode) * k;
  if (k == 0 || ncoef > 32 || mode < 0 || mode > 3 || !check_m(m, b, mode)) return ORC_EINVAL;
  int64_t* table = (int64_t*)malloc(sizeof(int64_t) * m);
  u128 s1 = 0, s2 = 0;
  do {
    memset(table, 0, sizeof(int64_t) * m);
    orc_cs_update_small(p, b, k, mode, 1, m, a, keys, weights, n, table);
    int64_t x;
    orc_cs_estimate(table, 1, m, NULL, &x);
    s1 += (u128)x;
    s2 += (u128)x * (u128)x;
  } while (next_tuple(a, ncoef, p));
  free(table);
  sum_x[0] = (uint64_t)s1; sum_x[1] = (uint64_t)(s1 >> 64);
  sum_x2[0] = (uint64_t)s2; sum_x2[1] = (uint64_t)(s2 >> 64);
  return ORC_OK;
}
