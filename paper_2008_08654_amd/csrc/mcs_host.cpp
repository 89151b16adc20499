// mcs_host.cpp -- host side of the C ABI declared in include/mcs.h: argument
// checking, coefficient expansion, device memory ownership, launch planning
// and sticky-error handling.  All compute is in the HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "mcs.h"
#include "sketch_kernels.hpp"
#include "mcs_internal.hpp"

using namespace mcs;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;

cs_status mcs::fail(cs_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

cs_status mcs::status_of(hipError_t e) {
  if (e == hipSuccess) return CS_OK;
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return CS_ENOMEM;
  return CS_EDEVICE;
}

cs_status mcs::hip_fail(hipError_t e, const char* what) {
  return fail(status_of(e) == CS_ENOMEM ? CS_ENOMEM : CS_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

extern "C" cs_status cs_status_from_hip_error(int hip_error) { return status_of((hipError_t)hip_error); }

#define HIP_TRY(call)                                       \
  do {                                                      \
    hipError_t e_ = (call);                                 \
    if (e_ != hipSuccess) return hip_fail(e_, #call);       \
  } while (0)

extern "C" const char* cs_last_error(void) { return g_last_error.c_str(); }
extern "C" const char* cs_version(void) { return "mcs 0.1 (gfx950)"; }

// ---------------------------------------------------------------------------
// device properties
// ---------------------------------------------------------------------------
const DeviceInfo& mcs::device_info(int dev) {
  static std::mutex mu;
  static std::vector<DeviceInfo> cache;
  std::lock_guard<std::mutex> lk(mu);
  if ((int)cache.size() <= dev) cache.resize(dev + 1);
  DeviceInfo& d = cache[dev];
  if (!d.valid) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
      d.cus = prop.multiProcessorCount;
      d.lds_per_block = (uint32_t)prop.sharedMemPerBlock;
      d.valid = true;
    } else {
      d.cus = 256;
      d.lds_per_block = 65536;
    }
  }
  return d;
}

// ---------------------------------------------------------------------------
// SplitMix64 seed expansion (Steele, Lea, Flood 2014)
// ---------------------------------------------------------------------------
namespace {
struct SplitMix64 {
  uint64_t state;
  uint64_t next() {
    state += 0x9E3779B97F4A7C15ull;
    uint64_t z = state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
};
}  // namespace

// fills `count` coefficients uniform in [p]: one uint64 each for p61, two for p89
static void expand_seed(cs_prime prime, uint64_t seed, size_t count, std::vector<uint64_t>& out) {
  SplitMix64 g{seed};
  if (prime == CS_P61) {
    out.resize(count);
    for (size_t i = 0; i < count; ++i) {
      uint64_t v;
      do v = g.next() & kP61;
      while (v == kP61);
      out[i] = v;
    }
  } else {
    out.resize(2 * count);
    for (size_t i = 0; i < count; ++i) {
      uint64_t lo, hi;
      do {
        lo = g.next();
        hi = g.next() & ((1ull << 25) - 1);
      } while (hi == (1ull << 25) - 1 && lo == ~0ull);  // value == 2^89 - 1
      out[2 * i] = lo;
      out[2 * i + 1] = hi;
    }
  }
}

static int npoly(cs_mode mode) { return mode == CS_TWO_POLY ? 2 : 1; }

static int log2_exact(uint64_t m) {
  if (m == 0 || (m & (m - 1))) return -1;
  int l = 0;
  while ((1ull << l) < m) ++l;
  return l;
}

// ---------------------------------------------------------------------------
// sketch lifetime
// ---------------------------------------------------------------------------
static cs_status check_shape(uint32_t rows, uint64_t buckets, cs_prime prime, cs_mode mode, uint32_t k,
                             int* log2m) {
  if (rows == 0 || rows > kMaxRows) return fail(CS_EINVAL, "rows must be in [1, %u]", kMaxRows);
  if (prime != CS_P61 && prime != CS_P89) return fail(CS_EINVAL, "sketch prime must be CS_P61 or CS_P89");
  if (mode != CS_TWO_FOR_ONE && mode != CS_TWO_FOR_ONE_MSB && mode != CS_TWO_POLY && mode != CS_ARB_R)
    return fail(CS_EINVAL, "unknown mode %d", (int)mode);
  if (k != 2 && k != 4 && k != 8) return fail(CS_EINVAL, "k must be 2, 4 or 8");
  if (mode == CS_ARB_R) {  // any count; rows are padded to the next power of two
    if (buckets < 2 || buckets > (1ull << kMaxLog2m))
      return fail(CS_EINVAL, "buckets must be in [2, 2^%u]", kMaxLog2m);
    int l = 0;
    while ((1ull << l) < buckets) ++l;
    *log2m = l;
    return CS_OK;
  }
  int l = log2_exact(buckets);
  if (l < 0) return fail(CS_EINVAL, "buckets must be a power of two");
  if ((uint32_t)l > kMaxLog2m) return fail(CS_EINVAL, "buckets must be at most 2^%u", kMaxLog2m);
  if (l == 0) return fail(CS_EINVAL, "buckets must be at least 2");
  *log2m = l;
  return CS_OK;
}

static cs_status reserve_for(cs_sketch* s, uint64_t keys);

static uint32_t est_slices_for(uint32_t log2m) {
  return (uint32_t)std::min<uint64_t>(256, std::max<uint64_t>(1, (1ull << log2m) / 16384));
}

size_t mcs::sketch_device_bytes(uint32_t rows, uint32_t log2m, cs_mode mode, uint32_t k) {
  const size_t ncoef = (size_t)rows * npoly(mode) * k;
  return ((size_t)rows << log2m) * 8 + ncoef * sizeof(uint4) + 64 + sizeof(uint32_t) * kRowRanges * kMaxRows +
         sizeof(EstPartial) * rows * est_slices_for(log2m) + sizeof(int64_t) * (rows + 2);
}

static cs_status create_common(uint32_t rows, uint64_t buckets, cs_prime prime, cs_mode mode, uint32_t k,
                               const std::vector<uint64_t>& coeffs, bool reserve, cs_sketch** out) {
  if (!out) return fail(CS_EINVAL, "out is NULL");
  *out = nullptr;
  int l;
  cs_status st = check_shape(rows, buckets, prime, mode, k, &l);
  if (st != CS_OK) return st;
  auto* s = new (std::nothrow) cs_sketch();
  if (!s) return fail(CS_ENOMEM, "host allocation");
  s->rows = rows;
  s->log2m = (uint32_t)l;
  s->buckets = buckets;
  s->prime = prime;
  s->mode = mode;
  s->k = k;
  s->h_coeffs = coeffs;
  HIP_TRY(hipGetDevice(&s->device));
  const size_t ncoef = (size_t)rows * npoly(mode) * k;
  std::vector<uint4> rec(ncoef);
  for (size_t i = 0; i < ncoef; ++i) {
    if (prime == CS_P61) {
      uint64_t v = coeffs[i];
      rec[i] = make_uint4((uint32_t)v, (uint32_t)(v >> 32), 0, (uint32_t)buckets);
    } else {
      uint64_t lo = coeffs[2 * i], hi = coeffs[2 * i + 1];
      rec[i] = make_uint4((uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi, (uint32_t)buckets);
    }
  }
  const size_t cells = (size_t)rows << l;
  hipError_t e;
  if ((e = hipMalloc(&s->d_table, cells * 8)) != hipSuccess ||
      (e = hipMalloc(&s->d_coeffs, ncoef * sizeof(uint4))) != hipSuccess ||
      (e = hipMalloc(&s->d_flags, 64)) != hipSuccess ||
      (e = hipMalloc(&s->d_queues, sizeof(uint32_t) * kRowRanges * kMaxRows)) != hipSuccess) {
    cs_destroy(s);
    return fail(CS_ENOMEM, "device allocation of %zu counters: %s", cells, hipGetErrorString(e));
  }
  s->est_slices = est_slices_for((uint32_t)l);
  if ((e = hipMalloc(&s->d_est_part, sizeof(EstPartial) * rows * s->est_slices)) != hipSuccess ||
      (e = hipMalloc(&s->d_est_out, sizeof(int64_t) * (rows + 2))) != hipSuccess ||
      (e = hipHostMalloc(&s->h_est_out, sizeof(int64_t) * (rows + 2), hipHostMallocDefault)) != hipSuccess) {
    cs_destroy(s);
    return fail(CS_ENOMEM, "estimate buffers: %s", hipGetErrorString(e));
  }
  if ((e = hipMemcpy(s->d_coeffs, rec.data(), ncoef * sizeof(uint4), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = launch_fill_zero((unsigned long long*)s->d_table, cells, 0)) != hipSuccess ||
      (e = launch_fill_zero((unsigned long long*)s->d_flags, 8, 0)) != hipSuccess ||
      (e = hipDeviceSynchronize()) != hipSuccess) {
    cs_destroy(s);
    return hip_fail(e, "sketch initialisation");
  }
  // the automatic path's workspace, if it needs one, for rounds of the default size
  if (reserve) {
    cs_status rs = reserve_for(s, kDefaultRoundKeys);
    if (rs != CS_OK) {
      cs_destroy(s);
      return rs;
    }
  }
  *out = s;
  return CS_OK;
}

extern "C" cs_status cs_create_ex(uint32_t rows, uint64_t buckets, cs_prime prime, uint64_t seed, cs_mode mode,
                                  uint32_t k, cs_sketch** out) {
  int l;
  cs_status st = check_shape(rows, buckets, prime, mode, k, &l);
  if (st != CS_OK) return st;
  std::vector<uint64_t> c;
  expand_seed(prime, seed, (size_t)rows * npoly(mode) * k, c);
  return create_common(rows, buckets, prime, mode, k, c, true, out);
}

cs_status mcs::create_unreserved(uint32_t rows, uint64_t buckets, cs_prime prime, uint64_t seed, cs_mode mode,
                                 uint32_t k, cs_sketch** out) {
  int l;
  cs_status st = check_shape(rows, buckets, prime, mode, k, &l);
  if (st != CS_OK) return st;
  std::vector<uint64_t> c;
  expand_seed(prime, seed, (size_t)rows * npoly(mode) * k, c);
  return create_common(rows, buckets, prime, mode, k, c, false, out);
}

extern "C" cs_status cs_create(uint32_t rows, uint64_t buckets, cs_prime prime, uint64_t seed, cs_sketch** out) {
  return cs_create_ex(rows, buckets, prime, seed, CS_TWO_FOR_ONE, 4, out);
}

extern "C" cs_status cs_create_with_coeffs(uint32_t rows, uint64_t buckets, cs_prime prime, cs_mode mode, uint32_t k,
                                           const uint64_t* coeffs, cs_sketch** out) {
  int l;
  cs_status st = check_shape(rows, buckets, prime, mode, k, &l);
  if (st != CS_OK) return st;
  if (!coeffs) return fail(CS_EINVAL, "coeffs is NULL");
  const size_t count = (size_t)rows * npoly(mode) * k;
  std::vector<uint64_t> c;
  if (prime == CS_P61) {
    c.assign(coeffs, coeffs + count);
    for (size_t i = 0; i < count; ++i)
      if (c[i] >= kP61) return fail(CS_EINVAL, "coefficient %zu is not below p", i);
  } else {
    c.assign(coeffs, coeffs + 2 * count);
    for (size_t i = 0; i < count; ++i) {
      uint64_t hi = c[2 * i + 1], lo = c[2 * i];
      if (hi >> 25 || (hi == (1ull << 25) - 1 && lo == ~0ull))
        return fail(CS_EINVAL, "coefficient %zu is not below p", i);
    }
  }
  return create_common(rows, buckets, prime, mode, k, c, true, out);
}

extern "C" void cs_destroy(cs_sketch* s) {
  if (!s) return;
  int cur = -1;
  (void)hipGetDevice(&cur);
  if (cur != s->device) (void)hipSetDevice(s->device);
  (void)hipDeviceSynchronize();
  if (s->d_table) (void)hipFree(s->d_table);
  if (s->d_coeffs) (void)hipFree(s->d_coeffs);
  if (s->d_flags) (void)hipFree(s->d_flags);
  if (s->d_queues) (void)hipFree(s->d_queues);
  if (s->d_est_part) (void)hipFree(s->d_est_part);
  if (s->d_est_out) (void)hipFree(s->d_est_out);
  if (s->h_est_out) (void)hipHostFree(s->h_est_out);
  release_workspace(s);
  if (cur >= 0 && cur != s->device) (void)hipSetDevice(cur);
  delete s;
}

// ---------------------------------------------------------------------------
// update
// ---------------------------------------------------------------------------
static cs_status check_dtypes(cs_dtype kt, cs_dtype wt, int* kb, int* wb) {
  if (kt != CS_U32 && kt != CS_U64) return fail(CS_EINVAL, "key type must be CS_U32 or CS_U64");
  if (wt != CS_I32 && wt != CS_I64) return fail(CS_EINVAL, "weight type must be CS_I32 or CS_I64");
  *kb = kt == CS_U32 ? 4 : 8;
  *wb = wt == CS_I32 ? 4 : 8;
  return CS_OK;
}

// Range width R = 2^log2r for the two-pass update: at most 32 ranges per row
// while R <= 2^14 (pass-2 LDS table of R int64), never below 2^11.
static bool binned_fits(const cs_sketch* s, uint32_t* log2g, uint32_t* log2r) {
  // up to 2^18 buckets: 8-16 ranges per row (wave tiles); beyond: 32 or more (block tiles)
  uint32_t lr = s->log2m <= 18 ? (s->log2m > 3 ? s->log2m - 3 : 0) : (s->log2m > 5 ? s->log2m - 5 : 0);
  lr = std::max(lr, kMinRangeLog2);
  lr = std::min(lr, kMaxRangeLog2);
  lr = std::min(lr, s->log2m);
  uint32_t lg = s->log2m - lr;
  if (lg > kMaxLog2g) return false;
  if (((uint64_t)s->rows << lg) + (1u << lg) + 2 > 8192) return false;  // pass-1 LDS counters
  *log2g = lg;
  *log2r = lr;
  return true;
}

// Rows per row group of the row-resident update: the largest divisor of rows
// whose 16-bit fields fit the block's LDS (0 if not even one row fits).
uint32_t mcs::rows_per_group(uint32_t rows, uint32_t log2m) {
  if (log2m > kRowMaxLog2m) return 0;
  const uint32_t fit = (uint32_t)(kRowLdsBytes / (2ull << log2m));
  for (uint32_t r = std::min(rows, fit); r >= 1; --r)
    if (rows % r == 0) return r;
  return 0;
}

UpdatePlan mcs::plan_update(const cs_sketch* s, uint64_t n) {
  const DeviceInfo& dev = device_info(s->device);
  const uint64_t cells = (uint64_t)s->rows << s->log2m;
  const uint64_t tile = (uint64_t)kBlock * kKeysPerThread;
  const uint64_t tiles = (n + tile - 1) / tile;
  UpdatePlan p{};
  uint32_t log2g = 0, log2r = 0;
  const uint32_t rpg = rows_per_group(s->rows, s->log2m);
  int path = s->path;
  if (path == 0)
    path = cells * 8 <= kLdsTableMax         ? CS_PATH_LDS
           : n * 8 < (1ull << s->log2m)      ? CS_PATH_GLOBAL
           : rpg                             ? CS_PATH_ROWS
           : binned_fits(s, &log2g, &log2r) ? CS_PATH_BINNED
                                            : CS_PATH_GLOBAL;
  if (path == CS_PATH_LDS && cells * 8 > kLdsTableMax) path = CS_PATH_GLOBAL;
  if (path == CS_PATH_ROWS && !rpg) path = CS_PATH_GLOBAL;
  if (path == CS_PATH_BINNED && !binned_fits(s, &log2g, &log2r)) path = CS_PATH_GLOBAL;
  if (path == CS_PATH_ROWS) {
    p.variant = kVariantRows;
    p.rpg = rpg;
    p.lds_bytes = (uint32_t)(rpg * (2ull << s->log2m));
    const uint64_t groups = s->rows / rpg;
    const uint64_t rtiles = (n + kRowTile - 1) / kRowTile;
    p.tiles = (uint32_t)std::min<uint64_t>(rtiles, 0xffffffffull);
    // Every block clears and flushes its group's fields, and the blocks of a
    // group flush into the same counters at about the same time; a block
    // therefore gets at least 2m keys (its flush then costs at most about half
    // its adds), up to one block per CU.
    const uint64_t per_group = std::max<uint64_t>(1, std::min<uint64_t>(rtiles, n / (2ull << s->log2m)));
    p.blocks = (uint32_t)std::max<uint64_t>(groups, std::min<uint64_t>((uint64_t)dev.cus, groups * per_group));
    // With at least one block per group on every XCD, the same number of
    // blocks per group on each XCD's range and the rest on the pool range
    // (k_update_rows); the grid is then a multiple of the XCD count.
    p.range_blocks = 0;
    if (p.blocks >= groups * kRowXcds && groups <= kMaxRows) {
      p.blocks -= p.blocks % kRowXcds;
      p.range_blocks = (uint32_t)(p.blocks / kRowXcds / groups * groups);
    }
    p.queues = s->d_queues;
  } else if (path == CS_PATH_LDS) {
    p.variant = kVariantLds;
    p.lds_bytes = (uint32_t)(cells * 8);
    uint64_t per_cu = std::max<uint64_t>(1, std::min<uint64_t>(8, kLdsPerCu / p.lds_bytes));
    uint64_t target = (uint64_t)dev.cus * per_cu * 2;
    p.blocks = (uint32_t)std::max<uint64_t>(1, std::min(tiles, target));
  } else if (path == CS_PATH_BINNED) {
    p.variant = kVariantBinned;
    p.log2g = log2g;
    p.log2r = log2r;
    p.dedup = s->combine;
    const uint32_t G = 1u << log2g;
    p.wave_tiles = G <= 16 && s->rows <= 16;
    // On the automatic path a probe of the keys chooses combining for block
    // tiles, whose combining table halves the occupancy; wave tiles combine
    // at little cost and always do.
    p.combine_auto = s->path == CS_PATH_AUTO && s->combine && !p.wave_tiles;
    uint32_t with = 0, without = 0;
    if (p.wave_tiles) {
      with = (kBlock / 64) * binw_lds_per_wave<true>(s->rows, G);
      without = (kBlock / 64) * binw_lds_per_wave<false>(s->rows, G);
    } else {
      const uint32_t counters = (uint32_t)(((uint64_t)s->rows * G + G + 2) * 4);
      with = bin_lds_fixed_bytes<true>() + counters;
      without = bin_lds_fixed_bytes<false>() + counters;
    }
    p.lds_bytes = p.dedup ? with : without;
    p.lds_bytes_plain = without;
    const uint32_t span = 1u << std::min(log2r, s->log2m);
    p.acc_lds_bytes = span * 8;
    const uint64_t per_cu = std::max<uint64_t>(1, std::min<uint64_t>(2, kLdsPerCu / p.acc_lds_bytes));
    p.acc_blocks = (uint32_t)(dev.cus * per_cu);
  } else {
    p.variant = kVariantGlobal;
    p.lds_bytes = 0;
    p.blocks = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(tiles, (uint64_t)dev.cus * 8));
  }
  return p;
}

extern "C" cs_status cs_update(cs_sketch* s, const void* keys, cs_dtype key_type, const void* weights,
                               cs_dtype weight_type, uint64_t n, hipStream_t stream) {
  if (!s) return fail(CS_EINVAL, "sketch is NULL");
  int kb, wb;
  cs_status st = check_dtypes(key_type, weight_type, &kb, &wb);
  if (st != CS_OK) return st;
  if (n == 0) return CS_OK;
  if (!keys || !weights) return fail(CS_EINVAL, "keys or weights is NULL");
  if (n > kMaxUpdateKeys) return fail(CS_EINVAL, "at most 2^40 keys per call");
  UpdatePlan plan = plan_update(s, n);
  return enqueue_update(s, plan, keys, kb, weights, wb, n, s->d_work, s->work_bytes, stream);
}

// Workspace of the two-pass update for rounds of `keys` keys (records,
// descriptors and the combining probe's counts).
static size_t twopass_work_bytes(const cs_sketch* s, const UpdatePlan& plan, uint64_t keys) {
  const uint32_t G = 1u << plan.log2g;
  const uint64_t tk = plan.wave_tiles ? kWaveTile : kBinTile;
  const uint64_t tiles = (std::min<uint64_t>(keys, kBinChunkKeys) + tk - 1) / tk;
  return (size_t)tiles * s->rows * (tk + G + 1) * 4 + 2 * kProbeTiles * sizeof(uint32_t);
}

// Grows the sketch's workspace to `bytes` (synchronising: the old one is freed).
static cs_status grow_workspace(cs_sketch* s, size_t bytes) {
  if (s->work_bytes >= bytes) return CS_OK;
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "workspace growth");
  release_workspace(s);
  e = hipMalloc(&s->d_work, bytes);
  if (e != hipSuccess) {
    s->d_work = nullptr;
    // out of memory is CS_ENOMEM; any other error (a fault an earlier kernel left
    // behind, which every later runtime call returns) is CS_EDEVICE
    return fail(status_of(e), "update workspace of %zu bytes: %s", bytes, hipGetErrorString(e));
  }
  s->work_bytes = bytes;
  return CS_OK;
}

// Reserves the workspace that updates of `keys` keys take on the sketch's
// current path (the two-pass path only; the others need none).
static cs_status reserve_for(cs_sketch* s, uint64_t keys) {
  const UpdatePlan plan = plan_update(s, std::max<uint64_t>(keys, 1));
  if (plan.variant != kVariantBinned) return CS_OK;
  return grow_workspace(s, twopass_work_bytes(s, plan, keys));
}

extern "C" cs_status cs_reserve(cs_sketch* s, uint64_t keys) {
  if (!s) return fail(CS_EINVAL, "sketch is NULL");
  int cur = -1;
  (void)hipGetDevice(&cur);
  if (cur != s->device) (void)hipSetDevice(s->device);
  cs_status st = reserve_for(s, keys);
  if (cur >= 0 && cur != s->device) (void)hipSetDevice(cur);
  return st;
}

cs_status mcs::enqueue_update(cs_sketch* s, const UpdatePlan& plan, const void* keys, int kb, const void* weights,
                              int wb, uint64_t n, void* work, size_t work_bytes, hipStream_t stream) {
  UpdateArgsAny a{};
  a.prime = s->prime == CS_P61 ? kPrime61 : kPrime89;
  a.mode = (int)s->mode;
  a.k = (int)s->k;
  a.key_bytes = kb;
  a.weight_bytes = wb;
  a.coeffs = (const uint4*)s->d_coeffs;
  a.rows = s->rows;
  a.log2m = s->log2m;
  a.table = (unsigned long long*)s->d_table;
  a.flags = s->d_flags;
  if (plan.variant == kVariantBinned) {
    const DeviceInfo& dev = device_info(s->device);
    const uint32_t G = 1u << plan.log2g;
    const uint64_t tk = plan.wave_tiles ? kWaveTile : kBinTile;
    // rounds as large as the workspace holds (at most kBinChunkKeys keys)
    const size_t probe_bytes = 2 * kProbeTiles * sizeof(uint32_t);
    const size_t per_tile = (size_t)s->rows * (tk + G + 1) * 4;
    const uint64_t fit_tiles = work_bytes > probe_bytes ? (work_bytes - probe_bytes) / per_tile : 0;
    if (fit_tiles == 0 || !work)
      return fail(CS_EINVAL, "the two-pass update needs a workspace of at least %zu bytes (cs_reserve)",
                  per_tile + probe_bytes);
    const uint64_t chunk = std::min<uint64_t>(std::min<uint64_t>(n, kBinChunkKeys), fit_tiles * tk);
    const uint64_t tiles_c = (chunk + tk - 1) / tk;
    const size_t rec_bytes = (size_t)tiles_c * s->rows * tk * 4;
    const size_t desc_bytes = (size_t)tiles_c * s->rows * (G + 1) * 4;
    for (uint64_t off = 0; off < n; off += chunk) {
      const uint64_t len = std::min<uint64_t>(chunk, n - off);
      UpdatePlan p = plan;
      p.tiles = (uint32_t)((len + tk - 1) / tk);
      const uint64_t tiles_per_block = plan.wave_tiles ? kBlock / 64 : 1;
      p.blocks = (uint32_t)std::min<uint64_t>((p.tiles + tiles_per_block - 1) / tiles_per_block, (uint64_t)dev.cus * 8);
      // pass-2 items: enough (partition, slice) pairs to keep every block busy
      const uint64_t parts = (uint64_t)s->rows << plan.log2g;
      uint64_t slices = (4ull * plan.acc_blocks + parts - 1) / parts;
      slices = std::max<uint64_t>(1, std::min<uint64_t>(slices, std::max<uint64_t>(1, p.tiles / 64)));
      p.acc_slices = (uint32_t)slices;
      p.recs = (uint32_t*)work;
      p.desc = (uint32_t*)((char*)work + rec_bytes);
      p.probe = plan.combine_auto ? (uint32_t*)((char*)work + rec_bytes + desc_bytes) : nullptr;
      a.keys = (const char*)keys + off * kb;
      a.weights = (const char*)weights + off * wb;
      a.n = len;
      hipError_t e = launch_update(p, a, stream);
      if (e != hipSuccess) return hip_fail(e, "cs_update launch");
    }
    return CS_OK;
  }
  a.keys = keys;
  a.weights = weights;
  a.n = n;
  if (plan.variant == kVariantRows) {
    hipError_t e = launch_update(plan, a, stream);
    if (e != hipSuccess) return hip_fail(e, "cs_update launch");
    return CS_OK;
  }
  const uint64_t tile = (uint64_t)kBlock * kKeysPerThread;
  uint64_t per = (n + plan.blocks - 1) / plan.blocks;
  a.keys_per_block = (per + tile - 1) / tile * tile;
  UpdatePlan p = plan;
  p.blocks = (uint32_t)((n + a.keys_per_block - 1) / a.keys_per_block);
  hipError_t e = launch_update(p, a, stream);
  if (e != hipSuccess) return hip_fail(e, "cs_update launch");
  return CS_OK;
}

extern "C" cs_status cs_set_update_path(cs_sketch* s, int path) {
  if (!s) return fail(CS_EINVAL, "sketch is NULL");
  if (path < CS_PATH_AUTO || path > CS_PATH_ROWS) return fail(CS_EINVAL, "unknown update path %d", path);
  s->path = path == CS_PATH_BINNED_NOCOMBINE ? CS_PATH_BINNED : path;
  s->combine = path != CS_PATH_BINNED_NOCOMBINE;
  // a path with a workspace gets the default one now, so that cs_update never allocates
  return s->work_bytes ? CS_OK : reserve_for(s, kDefaultRoundKeys);
}

// ---------------------------------------------------------------------------
// estimate, query, reads
// ---------------------------------------------------------------------------
cs_status mcs::flags_status(uint32_t flags) {
  if (flags & kFlagDomain)
    return fail(CS_EDOMAIN, "a key was outside the domain (p = 2^61-1 needs keys < 2^60)");
  if (flags & kFlagOverflow) return fail(CS_EOVERFLOW, "an F2 row estimate does not fit in int64");
  return CS_OK;
}

static cs_status sticky(const cs_sketch*, uint32_t flags) { return flags_status(flags); }

extern "C" cs_status cs_estimate_f2(cs_sketch* s, int64_t* f2, int64_t* rows_out, hipStream_t stream) {
  if (!s || !f2) return fail(CS_EINVAL, "sketch or f2 is NULL");
  hipError_t e = launch_estimate(s->d_table, s->rows, s->log2m, s->est_slices, (EstPartial*)s->d_est_part,
                                 s->d_est_out, s->d_flags, stream);
  if (e != hipSuccess) return hip_fail(e, "estimate launch");
  HIP_TRY(hipMemcpyAsync(s->h_est_out, s->d_est_out, sizeof(int64_t) * (s->rows + 2), hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  *f2 = s->h_est_out[0];
  if (rows_out) memcpy(rows_out, s->h_est_out + 1, sizeof(int64_t) * s->rows);
  return sticky(s, (uint32_t)s->h_est_out[1 + s->rows]);
}

extern "C" cs_status cs_query(cs_sketch* s, const void* keys, cs_dtype key_type, uint64_t n, int64_t* out,
                              hipStream_t stream) {
  if (!s) return fail(CS_EINVAL, "sketch is NULL");
  if (key_type != CS_U32 && key_type != CS_U64) return fail(CS_EINVAL, "key type must be CS_U32 or CS_U64");
  if (s->rows > kMaxQueryRows) return fail(CS_EINVAL, "point queries support at most %u rows", kMaxQueryRows);
  if (n == 0) return CS_OK;
  if (!keys || !out) return fail(CS_EINVAL, "keys or out is NULL");
  if (n > (uint64_t)kBlock * 0x7fffffffull) return fail(CS_EINVAL, "too many keys in one call");
  QueryArgsAny a{};
  a.prime = s->prime == CS_P61 ? kPrime61 : kPrime89;
  a.mode = (int)s->mode;
  a.k = (int)s->k;
  a.key_bytes = key_type == CS_U32 ? 4 : 8;
  a.keys = keys;
  a.n = n;
  a.coeffs = (const uint4*)s->d_coeffs;
  a.rows = s->rows;
  a.log2m = s->log2m;
  a.table = s->d_table;
  a.out = out;
  a.flags = s->d_flags;
  hipError_t e = launch_query(a, stream);
  if (e != hipSuccess) return hip_fail(e, "query launch");
  return CS_OK;
}

extern "C" cs_status cs_sync(cs_sketch* s, hipStream_t stream) {
  if (!s) return fail(CS_EINVAL, "sketch is NULL");
  HIP_TRY(hipStreamSynchronize(stream));
  uint32_t flags = 0;
  HIP_TRY(hipMemcpy(&flags, s->d_flags, 4, hipMemcpyDeviceToHost));
  return sticky(s, flags);
}

extern "C" cs_status cs_read_counters(cs_sketch* s, int64_t* host_dst, hipStream_t stream) {
  if (!s || !host_dst) return fail(CS_EINVAL, "sketch or destination is NULL");
  HIP_TRY(hipStreamSynchronize(stream));
  if (s->buckets == (1ull << s->log2m)) {
    HIP_TRY(hipMemcpy(host_dst, s->d_table, ((size_t)s->rows << s->log2m) * 8, hipMemcpyDeviceToHost));
  } else {  // drop the padding of each row
    HIP_TRY(hipMemcpy2D(host_dst, s->buckets * 8, s->d_table, (size_t)8 << s->log2m, s->buckets * 8, s->rows,
                        hipMemcpyDeviceToHost));
  }
  uint32_t flags = 0;
  HIP_TRY(hipMemcpy(&flags, s->d_flags, 4, hipMemcpyDeviceToHost));
  return sticky(s, flags);
}

extern "C" cs_status cs_table_device(cs_sketch* s, int64_t** dev_table) {
  if (!s || !dev_table) return fail(CS_EINVAL, "sketch or out pointer is NULL");
  *dev_table = s->d_table;
  return CS_OK;
}

extern "C" cs_status cs_read_coeffs(cs_sketch* s, uint64_t* host_dst) {
  if (!s || !host_dst) return fail(CS_EINVAL, "sketch or destination is NULL");
  memcpy(host_dst, s->h_coeffs.data(), s->h_coeffs.size() * 8);
  return CS_OK;
}

extern "C" cs_status cs_info(const cs_sketch* s, uint32_t* rows, uint64_t* buckets, cs_prime* prime, cs_mode* mode,
                             uint32_t* k) {
  if (!s) return fail(CS_EINVAL, "sketch is NULL");
  if (rows) *rows = s->rows;
  if (buckets) *buckets = s->buckets;
  if (prime) *prime = s->prime;
  if (mode) *mode = s->mode;
  if (k) *k = s->k;
  return CS_OK;
}

extern "C" cs_status cs_reset(cs_sketch* s, hipStream_t stream) {
  if (!s) return fail(CS_EINVAL, "sketch is NULL");
  hipError_t e = launch_fill_zero((unsigned long long*)s->d_table, (uint64_t)s->rows << s->log2m, stream);
  if (e == hipSuccess) e = launch_fill_zero((unsigned long long*)s->d_flags, 8, stream);
  if (e != hipSuccess) return hip_fail(e, "reset");
  return CS_OK;
}

extern "C" cs_status cs_merge(cs_sketch* dst, const cs_sketch* src, hipStream_t stream) {
  if (!dst || !src) return fail(CS_EINVAL, "sketch is NULL");
  if (dst->rows != src->rows || dst->buckets != src->buckets || dst->prime != src->prime || dst->mode != src->mode ||
      dst->k != src->k || dst->h_coeffs != src->h_coeffs)
    return fail(CS_EINVAL, "sketches differ in shape or coefficients");
  hipError_t e = launch_add_tables((unsigned long long*)dst->d_table, (const unsigned long long*)src->d_table,
                                   (uint64_t)dst->rows << dst->log2m, stream);
  if (e != hipSuccess) return hip_fail(e, "merge");
  return CS_OK;
}

// ---------------------------------------------------------------------------
// quotient / remainder
// ---------------------------------------------------------------------------
static uint32_t* divmod_flags() {
  static std::mutex mu;
  static std::vector<uint32_t*> per_dev;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lk(mu);
  if ((int)per_dev.size() <= dev) per_dev.resize(dev + 1, nullptr);
  if (!per_dev[dev]) {
    uint32_t* p = nullptr;
    if (hipMalloc(&p, 64) != hipSuccess) return nullptr;
    if (launch_fill_zero((unsigned long long*)p, 8, 0) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
      (void)hipFree(p);
      return nullptr;
    }
    per_dev[dev] = p;
  }
  return per_dev[dev];
}

static cs_status divmod_common(cs_prime prime, const uint64_t* x, uint64_t n, uint64_t* quot, uint64_t* rem,
                               hipStream_t stream, bool naive) {
  if (prime != CS_P61 && prime != CS_P89 && prime != CS_P64_59) return fail(CS_EINVAL, "unknown prime");
  if (n == 0) return CS_OK;
  if (!x) return fail(CS_EINVAL, "x is NULL");
  if (!quot && !rem) return fail(CS_EINVAL, "quot and rem are both NULL");
  // the kernels move two-limb values as 16-byte vectors
  if (prime != CS_P89 && ((uintptr_t)x & 15)) return fail(CS_EINVAL, "x must be 16-byte aligned");
  if (prime == CS_P89 && (((uintptr_t)quot & 15) || ((uintptr_t)rem & 15)))
    return fail(CS_EINVAL, "quot and rem must be 16-byte aligned for CS_P89");
  uint32_t* flags = divmod_flags();
  if (!flags) return fail(CS_ENOMEM, "flag allocation");
  int p = prime == CS_P61 ? kPrime61 : prime == CS_P89 ? kPrime89 : kPrime64c;
  hipError_t e = launch_divmod(p, naive, x, n, quot, rem, flags, stream);
  if (e != hipSuccess) return hip_fail(e, "divmod launch");
  return CS_OK;
}

extern "C" cs_status mersenne_divmod(cs_prime prime, const uint64_t* x, uint64_t n, uint64_t* quot, uint64_t* rem,
                                     hipStream_t stream) {
  return divmod_common(prime, x, n, quot, rem, stream, false);
}
extern "C" cs_status mersenne_div(cs_prime prime, const uint64_t* x, uint64_t n, uint64_t* quot, hipStream_t stream) {
  if (!quot && n) return fail(CS_EINVAL, "quot is NULL");
  return divmod_common(prime, x, n, quot, nullptr, stream, false);
}
extern "C" cs_status mersenne_mod(cs_prime prime, const uint64_t* x, uint64_t n, uint64_t* rem, hipStream_t stream) {
  if (!rem && n) return fail(CS_EINVAL, "rem is NULL");
  return divmod_common(prime, x, n, nullptr, rem, stream, false);
}
extern "C" cs_status mersenne_divmod_naive(cs_prime prime, const uint64_t* x, uint64_t n, uint64_t* quot,
                                           uint64_t* rem, hipStream_t stream) {
  return divmod_common(prime, x, n, quot, rem, stream, true);
}
extern "C" cs_status mersenne_bucket_map(cs_prime prime, int method, const uint64_t* v, uint64_t n, uint64_t r,
                                         uint32_t* out, hipStream_t stream) {
  if (prime != CS_P61 && prime != CS_P89 && prime != CS_P64_59) return fail(CS_EINVAL, "unknown prime %d", (int)prime);
  if (method != CS_MAP_EXACT && method != CS_MAP_MERSENNE) return fail(CS_EINVAL, "unknown map %d", method);
  if (method == CS_MAP_MERSENNE && prime == CS_P64_59)
    return fail(CS_EINVAL, "the (v+1)r >> b map is most uniform only for Mersenne primes");
  if (r == 0 || r >= (1ull << 32)) return fail(CS_EINVAL, "r must be in [1, 2^32)");
  if (n == 0) return CS_OK;
  if (!v || !out) return fail(CS_EINVAL, "v or out is NULL");
  if (prime == CS_P89 && ((uintptr_t)v & 15)) return fail(CS_EINVAL, "v must be 16-byte aligned for CS_P89");
  uint32_t* flags = divmod_flags();
  if (!flags) return fail(CS_ENOMEM, "flag allocation");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  const int pk = prime == CS_P61 ? kPrime61 : prime == CS_P89 ? kPrime89 : kPrime64c;
  hipError_t e = launch_bucket_map(pk, method == CS_MAP_MERSENNE, v, n, (uint32_t)r, out, flags,
                                   (uint32_t)device_info(dev).cus, stream);
  if (e != hipSuccess) return hip_fail(e, "bucket map launch");
  return CS_OK;
}

extern "C" cs_status mersenne_divmod_wide(uint32_t b, uint32_t c, int method, const uint32_t* x, uint64_t n,
                                          uint32_t* quot, uint32_t* rem, hipStream_t stream) {
  if (b != 32 && b != 64 && b != 128 && b != 256 && b != 512 && b != 1024)
    return fail(CS_EINVAL, "b must be 32, 64, 128, 256, 512 or 1024");
  if (c == 0 || c >= (1u << 31)) return fail(CS_EINVAL, "c must be in [1, 2^31)");
  if (method != CS_WIDE_ALG5 && method != CS_WIDE_CCH) return fail(CS_EINVAL, "unknown method %d", method);
  if (n == 0) return CS_OK;
  if (!x) return fail(CS_EINVAL, "x is NULL");
  if (!quot && !rem) return fail(CS_EINVAL, "quot and rem are both NULL");
  // Algorithm 5's step count: (2^b / c)^m >= 2^(2b) > x holds once m (b - ceil(log2 c)) >= 2b
  uint32_t lc = 0;
  while ((1ull << lc) < c) ++lc;
  if (2 * lc >= b) return fail(CS_EINVAL, "c must be below 2^(b/2)");
  const uint32_t m = (2 * b + (b - lc) - 1) / (b - lc);
  hipError_t e = launch_wide_divmod(b, c, m, method, x, n, quot, rem, stream);
  if (e != hipSuccess) return hip_fail(e, "wide divmod launch");
  return CS_OK;
}

extern "C" cs_status mersenne_status(hipStream_t stream) {
  uint32_t* flags = divmod_flags();
  if (!flags) return fail(CS_ENOMEM, "flag allocation");
  HIP_TRY(hipStreamSynchronize(stream));
  uint32_t v = 0;
  HIP_TRY(hipMemcpy(&v, flags, 4, hipMemcpyDeviceToHost));
  if (v) {
    hipError_t e = launch_fill_zero((unsigned long long*)flags, 8, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "flag reset");
    return fail(CS_EDOMAIN, "a value was outside the quotient/remainder domain");
  }
  return CS_OK;
}
