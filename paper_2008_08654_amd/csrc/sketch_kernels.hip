// sketch_kernels.hip -- Count Sketch kernels for gfx950 (Algorithm 2 of Ahle,
// Knudsen, Thorup, "The Power of Hashing with Mersenne Primes").
//
// Per key and row: Horner evaluation of the row's polynomial over p
// (Algorithm 1, field.hpp), branch-free final reduction (Algorithm 4), the
// bucket/sign split (Algorithm 3 or the low-bit layout of Section 1.2.1), and
// a signed int64 add into the row's counters.
//
// Coefficients live in device memory as one 16-byte record per coefficient
// (32-bit limbs w0, w1, w2, 0), indexed [row][poly][i]; the row loop is the
// outer loop so each row's coefficients are wave-uniform scalar loads.
#include <algorithm>

#include "sketch_kernels.hpp"

namespace mcs {

// ---------------------------------------------------------------------------
// hashing of one key in one row
// ---------------------------------------------------------------------------
template <int K>
__device__ __forceinline__ uint64_t hash61_x32(const uint4* __restrict__ c, uint32_t x) {
  F61 y{c[K - 1].x, c[K - 1].y};
#pragma unroll
  for (int i = K - 2; i >= 0; --i) y = p61_step_x32(y, x, F61{c[i].x, c[i].y});
  return p61_final(y);
}

template <int K>
__device__ __forceinline__ uint64_t hash61_x64(const uint4* __restrict__ c, uint32_t x0, uint32_t x1) {
  F61 y{c[K - 1].x, c[K - 1].y};
#pragma unroll
  for (int i = K - 2; i >= 0; --i) y = p61_step_x64(y, x0, x1, F61{c[i].x, c[i].y});
  return p61_final(y);
}

template <int K>
__device__ __forceinline__ F89 hash89(const uint4* __restrict__ c, uint32_t x0, uint32_t x1) {
  F89 y{c[K - 1].x, c[K - 1].y, c[K - 1].z};
#pragma unroll
  for (int i = K - 2; i >= 0; --i) y = p89_step(y, x0, x1, F89{c[i].x, c[i].y, c[i].z});
  return p89_final(y);
}

// Bucket and sign bit of key (x0, x1) in the row whose first coefficient
// record is `c`.  WIDE selects the two-limb key path for p61.
template <int PRIME, int MODE, int K, bool WIDE>
__device__ __forceinline__ void bucket_sign(const uint4* __restrict__ c, uint32_t x0, uint32_t x1,
                                            uint32_t log2m, uint32_t& bucket, uint32_t& a) {
  const uint32_t mask = (1u << log2m) - 1u;
  if constexpr (PRIME == kPrime61) {
    uint64_t h = WIDE ? hash61_x64<K>(c, x0, x1) : hash61_x32<K>(c, x0);
    if constexpr (MODE == kTwoForOne) {
      a = (uint32_t)h & 1u;
      bucket = ((uint32_t)h >> 1) & mask;
    } else if constexpr (MODE == kTwoForOneMsb) {
      a = (uint32_t)(h >> 60) & 1u;
      bucket = (uint32_t)h & mask;
    } else {
      uint64_t h2 = WIDE ? hash61_x64<K>(c + K, x0, x1) : hash61_x32<K>(c + K, x0);
      a = (uint32_t)h2 & 1u;
      bucket = (uint32_t)h & mask;
    }
  } else {
    F89 h = hash89<K>(c, x0, x1);
    if constexpr (MODE == kTwoForOne) {
      a = h.w0 & 1u;
      bucket = (h.w0 >> 1) & mask;
    } else if constexpr (MODE == kTwoForOneMsb) {
      a = (h.w2 >> 24) & 1u;
      bucket = h.w0 & mask;
    } else {
      F89 h2 = hash89<K>(c + K, x0, x1);
      a = h2.w0 & 1u;
      bucket = h.w0 & mask;
    }
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

__device__ __forceinline__ unsigned long long signed_weight(int64_t w, uint32_t a) {
  return (unsigned long long)(a ? -w : w);
}

// ---------------------------------------------------------------------------
// Single pass with the whole table in LDS.  Each block zeroes its private
// table, processes a contiguous key range, then adds the non-zero partial
// counters into the global table with coalesced int64 atomics.
// ---------------------------------------------------------------------------
template <int PRIME, int MODE, int K, typename KeyT, typename WT>
__global__ __launch_bounds__(kBlock) void k_update_lds(UpdateArgs<KeyT, WT> args) {
  extern __shared__ unsigned long long lds[];
  const uint32_t cells = args.rows << args.log2m;
  for (uint32_t i = threadIdx.x; i < cells; i += kBlock) lds[i] = 0;
  __syncthreads();

  const uint64_t begin = (uint64_t)blockIdx.x * args.keys_per_block;
  const uint64_t end = min(args.n, begin + args.keys_per_block);
  constexpr int kKpt = kKeysPerThread;
  constexpr int NP = MODE == kTwoPoly ? 2 : 1;
  uint32_t bad = 0;

  for (uint64_t base = begin; base < end; base += (uint64_t)kBlock * kKpt) {
    uint32_t x0[kKpt], x1[kKpt];
    int64_t wv[kKpt];
    bool ok[kKpt];
#pragma unroll
    for (int j = 0; j < kKpt; ++j) {
      uint64_t i = base + (uint64_t)j * kBlock + threadIdx.x;
      ok[j] = i < end;
      x0[j] = x1[j] = 0;
      wv[j] = 0;
      if (ok[j]) {
        load_key(args.keys, i, x0[j], x1[j]);
        wv[j] = load_weight(args.weights, i);
      }
    }
    uint32_t any_hi = 0;
#pragma unroll
    for (int j = 0; j < kKpt; ++j) any_hi |= x1[j];
    if constexpr (PRIME == kPrime61) bad |= any_hi >> 28;  // key >= 2^60 breaks p >= 2u - 1
    // wave-uniform choice of the one-limb key path (all keys < 2^32)
    const bool wide = PRIME == kPrime61 && sizeof(KeyT) == 8 && __any(any_hi != 0);
    for (uint32_t r = 0; r < args.rows; ++r) {
      const uint4* c = args.coeffs + (size_t)r * NP * K;
      unsigned long long* row = lds + ((size_t)r << args.log2m);
      if (wide) {
#pragma unroll
        for (int j = 0; j < kKpt; ++j) {
          uint32_t bk, a;
          bucket_sign<PRIME, MODE, K, true>(c, x0[j], x1[j], args.log2m, bk, a);
          if (ok[j]) atomicAdd(&row[bk], signed_weight(wv[j], a));
        }
      } else {
#pragma unroll
        for (int j = 0; j < kKpt; ++j) {
          uint32_t bk, a;
          bucket_sign<PRIME, MODE, K, false>(c, x0[j], x1[j], args.log2m, bk, a);
          if (ok[j]) atomicAdd(&row[bk], signed_weight(wv[j], a));
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

// ---------------------------------------------------------------------------
// Table in global memory, one device-scope int64 atomic per (key, row).
// ---------------------------------------------------------------------------
template <int PRIME, int MODE, int K, typename KeyT, typename WT>
__global__ __launch_bounds__(kBlock) void k_update_global(UpdateArgs<KeyT, WT> args) {
  const uint64_t begin = (uint64_t)blockIdx.x * args.keys_per_block;
  const uint64_t end = min(args.n, begin + args.keys_per_block);
  constexpr int kKpt = kKeysPerThread;
  constexpr int NP = MODE == kTwoPoly ? 2 : 1;
  uint32_t bad = 0;
  for (uint64_t base = begin; base < end; base += (uint64_t)kBlock * kKpt) {
    uint32_t x0[kKpt], x1[kKpt];
    int64_t wv[kKpt];
    bool ok[kKpt];
#pragma unroll
    for (int j = 0; j < kKpt; ++j) {
      uint64_t i = base + (uint64_t)j * kBlock + threadIdx.x;
      ok[j] = i < end;
      x0[j] = x1[j] = 0;
      wv[j] = 0;
      if (ok[j]) {
        load_key(args.keys, i, x0[j], x1[j]);
        wv[j] = load_weight(args.weights, i);
      }
    }
    uint32_t any_hi = 0;
#pragma unroll
    for (int j = 0; j < kKpt; ++j) any_hi |= x1[j];
    if constexpr (PRIME == kPrime61) bad |= any_hi >> 28;
    const bool wide = PRIME == kPrime61 && sizeof(KeyT) == 8 && __any(any_hi != 0);
    for (uint32_t r = 0; r < args.rows; ++r) {
      const uint4* c = args.coeffs + (size_t)r * NP * K;
      unsigned long long* row = args.table + ((size_t)r << args.log2m);
#pragma unroll
      for (int j = 0; j < kKpt; ++j) {
        uint32_t bk, a;
        if (wide)
          bucket_sign<PRIME, MODE, K, true>(c, x0[j], x1[j], args.log2m, bk, a);
        else
          bucket_sign<PRIME, MODE, K, false>(c, x0[j], x1[j], args.log2m, bk, a);
        if (ok[j]) atomicAdd(&row[bk], signed_weight(wv[j], a));
      }
    }
  }
  if (bad) atomicOr(args.flags, kFlagDomain);
}

// ---------------------------------------------------------------------------
// Two-pass update for tables larger than LDS.
//
// Pass 1 (k_bin): each block takes tiles of kBinTile keys.  For every row it
// hashes the tile's keys, and writes one 4-byte record per key into the
// tile's region for that row, grouped by bucket range g = bucket >> 14
// (partition (row, g)).  A record is (bucket & (2^14-1)) << 18 | (signed
// weight & (2^18-1)); a signed weight outside [-2^17, 2^17) goes straight to
// the global table with an atomic instead.  desc[tile][row][0..G] holds the
// offsets of the groups inside the region (G = number of ranges per row).
//
// Pass 2 (k_accumulate): block (slice, partition) adds the records of its
// partition from a slice of tiles into an int64 LDS table of 2^14 counters
// and then adds the non-zero counters into the global table.
// ---------------------------------------------------------------------------
template <int PRIME, int MODE, int K, typename KeyT, typename WT>
__global__ __launch_bounds__(kBlock) void k_bin(BinArgs<KeyT, WT> args) {
  extern __shared__ uint32_t sh[];
  const uint32_t G = 1u << args.log2g;
  uint32_t* hist = sh;                 // rows x G
  uint32_t* offs = sh + args.rows * G; // G + 1
  constexpr int kKpt = kBinKpt;
  constexpr int NP = MODE == kTwoPoly ? 2 : 1;
  const uint32_t rmask = (1u << kRangeLog2) - 1u;
  uint32_t bad = 0;
  for (uint32_t tile = blockIdx.x; tile < args.tiles; tile += gridDim.x) {
    for (uint32_t i = threadIdx.x; i < args.rows * G; i += kBlock) hist[i] = 0;
    const uint64_t base = (uint64_t)tile * kBinTile;
    uint32_t x0[kKpt], x1[kKpt];
    int64_t wv[kKpt];
    bool ok[kKpt];
#pragma unroll
    for (int j = 0; j < kKpt; ++j) {
      uint64_t i = base + (uint64_t)j * kBlock + threadIdx.x;
      ok[j] = i < args.n;
      x0[j] = x1[j] = 0;
      wv[j] = 0;
      if (ok[j]) {
        load_key(args.keys, i, x0[j], x1[j]);
        wv[j] = load_weight(args.weights, i);
      }
    }
    uint32_t any_hi = 0;
#pragma unroll
    for (int j = 0; j < kKpt; ++j) any_hi |= x1[j];
    if constexpr (PRIME == kPrime61) bad |= any_hi >> 28;
    const bool wide = PRIME == kPrime61 && sizeof(KeyT) == 8 && __any(any_hi != 0);
    __syncthreads();
    for (uint32_t r = 0; r < args.rows; ++r) {
      const uint4* c = args.coeffs + (size_t)r * NP * K;
      uint32_t rec[kKpt], grp[kKpt], tick[kKpt];
#pragma unroll
      for (int j = 0; j < kKpt; ++j) {
        uint32_t bk, a;
        if (wide)
          bucket_sign<PRIME, MODE, K, true>(c, x0[j], x1[j], args.log2m, bk, a);
        else
          bucket_sign<PRIME, MODE, K, false>(c, x0[j], x1[j], args.log2m, bk, a);
        int64_t sw = a ? -wv[j] : wv[j];
        grp[j] = bk >> kRangeLog2;
        rec[j] = ((bk & rmask) << kRecWeightBits) | ((uint32_t)sw & ((1u << kRecWeightBits) - 1u));
        const bool fits = (uint64_t)(sw + (1ll << (kRecWeightBits - 1))) < (1ull << kRecWeightBits);
        tick[j] = 0xffffffffu;
        if (ok[j]) {
          if (fits)
            tick[j] = atomicAdd(&hist[r * G + grp[j]], 1u);
          else
            atomicAdd(&args.table[((size_t)r << args.log2m) + bk], (unsigned long long)sw);
        }
      }
      __syncthreads();
      // exclusive prefix over the row's G group counts
      uint32_t* d = args.desc + ((size_t)tile * args.rows + r) * (G + 1);
      for (uint32_t g = threadIdx.x; g <= G; g += kBlock) {
        uint32_t acc = 0;
        for (uint32_t q = 0; q < g; ++q) acc += hist[r * G + q];
        offs[g] = acc;
        d[g] = acc;
      }
      __syncthreads();
      uint32_t* out = args.recs + ((size_t)tile * args.rows + r) * kBinTile;
#pragma unroll
      for (int j = 0; j < kKpt; ++j)
        if (tick[j] != 0xffffffffu) out[offs[grp[j]] + tick[j]] = rec[j];
      __syncthreads();
    }
  }
  if (bad) atomicOr(args.flags, kFlagDomain);
}

__global__ __launch_bounds__(kAccBlock) void k_accumulate(AccArgs args) {
  __shared__ unsigned long long acc[1u << kRangeLog2];
  const uint32_t G = 1u << args.log2g;
  const uint32_t part = blockIdx.y;  // row * G + g
  const uint32_t r = part >> args.log2g, g = part & (G - 1);
  const uint32_t R = 1u << kRangeLog2;
  for (uint32_t i = threadIdx.x; i < R; i += kAccBlock) acc[i] = 0;
  __syncthreads();
  const uint32_t per = (args.tiles + gridDim.x - 1) / gridDim.x;
  const uint32_t t0 = blockIdx.x * per, t1 = min(args.tiles, t0 + per);
  const uint32_t wave = threadIdx.x / 64, lane = threadIdx.x % 64, nw = kAccBlock / 64;
  for (uint32_t tile = t0 + wave; tile < t1; tile += nw) {
    const uint32_t* d = args.desc + ((size_t)tile * args.rows + r) * (G + 1) + g;
    const uint32_t b = d[0], e = d[1];
    const uint32_t* rec = args.recs + ((size_t)tile * args.rows + r) * kBinTile;
    for (uint32_t i = b + lane; i < e; i += 64) {
      uint32_t v = rec[i];
      int64_t sw = (int64_t)((int32_t)(v << (32 - kRecWeightBits)) >> (32 - kRecWeightBits));
      atomicAdd(&acc[v >> kRecWeightBits], (unsigned long long)sw);
    }
  }
  __syncthreads();
  unsigned long long* dst = args.table + ((size_t)r << args.log2m) + ((size_t)g << kRangeLog2);
  const uint32_t span = args.log2m < kRangeLog2 ? (1u << args.log2m) : R;  // counters of this range
  for (uint32_t i = threadIdx.x; i < span; i += kAccBlock) {
    unsigned long long v = acc[i];
    if (v) atomicAdd(&dst[i], v);
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
    const uint4* c = args.coeffs + (size_t)r * NP * K;
    if (PRIME == kPrime61 && x1 != 0)
      bucket_sign<PRIME, MODE, K, true>(c, x0, x1, args.log2m, bk, a);
    else
      bucket_sign<PRIME, MODE, K, false>(c, x0, x1, args.log2m, bk, a);
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
__global__ __launch_bounds__(kBlock) void k_estimate_partial(const int64_t* __restrict__ table, uint32_t log2m,
                                                             uint32_t slices, EstPartial* __restrict__ part) {
  const uint32_t row = blockIdx.y, slice = blockIdx.x;
  const uint64_t m = 1ull << log2m;
  const uint64_t per = (m + slices - 1) / slices;
  const uint64_t b = (uint64_t)slice * per, e = min(m, b + per);
  const int64_t* t = table + ((size_t)row << log2m);
  unsigned __int128 acc = 0;
  uint32_t big = 0;
  for (uint64_t i = b + threadIdx.x; i < e; i += kBlock) {
    int64_t c = t[i];
    uint64_t mag = c < 0 ? 0ull - (uint64_t)c : (uint64_t)c;
    unsigned __int128 sq = (unsigned __int128)mag * mag;
    acc += sq;
    big |= (uint32_t)(acc >> 126);  // keeps the running sum far from wrapping
  }
  __shared__ unsigned long long s_lo[kBlock], s_hi[kBlock];
  __shared__ uint32_t s_big;
  if (threadIdx.x == 0) s_big = 0;
  s_lo[threadIdx.x] = (unsigned long long)acc;
  s_hi[threadIdx.x] = (unsigned long long)(acc >> 64);
  __syncthreads();
  if (big) atomicOr(&s_big, 1u);
  for (uint32_t w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      unsigned __int128 x = ((unsigned __int128)s_hi[threadIdx.x] << 64) | s_lo[threadIdx.x];
      unsigned __int128 y = ((unsigned __int128)s_hi[threadIdx.x + w] << 64) | s_lo[threadIdx.x + w];
      unsigned __int128 z = x + y;
      if (z >> 126) atomicOr(&s_big, 1u);
      s_lo[threadIdx.x] = (unsigned long long)z;
      s_hi[threadIdx.x] = (unsigned long long)(z >> 64);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    EstPartial& o = part[(size_t)row * slices + slice];
    o.lo = s_lo[0];
    o.hi = s_hi[0];
    o.big = s_big;
  }
}

__global__ void k_estimate_final(const EstPartial* __restrict__ part, uint32_t rows, uint32_t slices,
                                 int64_t* __restrict__ out, uint32_t* flags) {
  // out[0] = median, out[1..rows] = X_j ; one thread per row, then thread 0 sorts
  __shared__ int64_t vals[kMaxRows];
  __shared__ uint32_t over;
  if (threadIdx.x == 0) over = 0;
  __syncthreads();
  for (uint32_t r = threadIdx.x; r < rows; r += blockDim.x) {
    unsigned __int128 acc = 0;
    uint32_t big = 0;
    for (uint32_t s = 0; s < slices; ++s) {
      const EstPartial& p = part[(size_t)r * slices + s];
      acc += ((unsigned __int128)p.hi << 64) | p.lo;
      big |= p.big | (uint32_t)(acc >> 126);
    }
    int64_t v;
    if (big || acc > (unsigned __int128)INT64_MAX) {
      v = INT64_MAX;
      atomicOr(&over, 1u);
    } else {
      v = (int64_t)acc;
    }
    vals[r] = v;
    out[1 + r] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (uint32_t i = 1; i < rows; ++i) {
      int64_t v = vals[i];
      uint32_t j = i;
      while (j > 0 && vals[j - 1] > v) {
        vals[j] = vals[j - 1];
        --j;
      }
      vals[j] = v;
    }
    out[0] = vals[(rows - 1) / 2];
    // overflow concerns this estimate only; the sticky flags are reported alongside
    out[1 + rows] = (int64_t)((*(volatile uint32_t*)flags) | (over ? kFlagOverflow : 0u));
  }
}

__global__ void k_add_tables(unsigned long long* __restrict__ dst, const unsigned long long* __restrict__ src, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    dst[i] += src[i];
}

__global__ void k_fill_zero(unsigned long long* __restrict__ dst, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    dst[i] = 0;
}

// ---------------------------------------------------------------------------
// launch helpers (host side)
// ---------------------------------------------------------------------------
template <int PRIME, int MODE, int K, typename KeyT, typename WT>
static hipError_t launch_update_t(const UpdatePlan& plan, const UpdateArgs<KeyT, WT>& a, hipStream_t st) {
  if (plan.variant == kVariantBinned) {
    BinArgs<KeyT, WT> b{a.keys, a.weights, a.n, a.coeffs, a.rows, a.log2m, plan.log2g, plan.tiles,
                        plan.recs, plan.desc, a.table, a.flags};
    hipLaunchKernelGGL((k_bin<PRIME, MODE, K, KeyT, WT>), dim3(plan.blocks), dim3(kBlock), plan.lds_bytes, st, b);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    AccArgs c{plan.recs, plan.desc, plan.tiles, a.rows, a.log2m, plan.log2g, a.table};
    const uint32_t parts = a.rows << plan.log2g;
    hipLaunchKernelGGL(k_accumulate, dim3(plan.acc_slices, parts), dim3(kAccBlock), 0, st, c);
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
static hipError_t launch_update_k(const UpdatePlan& plan, const UpdateArgsAny& a, hipStream_t st) {
  if (a.key_bytes == 4 && a.weight_bytes == 4)
    return launch_update_t<PRIME, MODE, K, uint32_t, int32_t>(plan, a.as<uint32_t, int32_t>(), st);
  if (a.key_bytes == 4 && a.weight_bytes == 8)
    return launch_update_t<PRIME, MODE, K, uint32_t, int64_t>(plan, a.as<uint32_t, int64_t>(), st);
  if (a.key_bytes == 8 && a.weight_bytes == 4)
    return launch_update_t<PRIME, MODE, K, uint64_t, int32_t>(plan, a.as<uint64_t, int32_t>(), st);
  return launch_update_t<PRIME, MODE, K, uint64_t, int64_t>(plan, a.as<uint64_t, int64_t>(), st);
}

template <int PRIME, int MODE>
static hipError_t launch_update_m(const UpdatePlan& plan, const UpdateArgsAny& a, hipStream_t st) {
  switch (a.k) {
    case 2: return launch_update_k<PRIME, MODE, 2>(plan, a, st);
    case 8: return launch_update_k<PRIME, MODE, 8>(plan, a, st);
    default: return launch_update_k<PRIME, MODE, 4>(plan, a, st);
  }
}

hipError_t launch_update(const UpdatePlan& plan, const UpdateArgsAny& a, hipStream_t st) {
  if (a.prime == kPrime61) {
    if (a.mode == kTwoForOne) return launch_update_m<kPrime61, kTwoForOne>(plan, a, st);
    if (a.mode == kTwoForOneMsb) return launch_update_m<kPrime61, kTwoForOneMsb>(plan, a, st);
    return launch_update_m<kPrime61, kTwoPoly>(plan, a, st);
  }
  if (a.mode == kTwoForOne) return launch_update_m<kPrime89, kTwoForOne>(plan, a, st);
  if (a.mode == kTwoForOneMsb) return launch_update_m<kPrime89, kTwoForOneMsb>(plan, a, st);
  return launch_update_m<kPrime89, kTwoPoly>(plan, a, st);
}

template <int PRIME, int MODE, int K, typename KeyT>
static hipError_t launch_query_t(const QueryArgs<KeyT>& a, hipStream_t st) {
  uint64_t blocks = (a.n + kBlock - 1) / kBlock;
  hipLaunchKernelGGL((k_query<PRIME, MODE, K, KeyT>), dim3((uint32_t)blocks), dim3(kBlock), 0, st, a);
  return hipGetLastError();
}

template <int PRIME, int MODE, int K>
static hipError_t launch_query_k(const QueryArgsAny& a, hipStream_t st) {
  if (a.key_bytes == 4) return launch_query_t<PRIME, MODE, K, uint32_t>(a.as<uint32_t>(), st);
  return launch_query_t<PRIME, MODE, K, uint64_t>(a.as<uint64_t>(), st);
}

template <int PRIME, int MODE>
static hipError_t launch_query_m(const QueryArgsAny& a, hipStream_t st) {
  switch (a.k) {
    case 2: return launch_query_k<PRIME, MODE, 2>(a, st);
    case 8: return launch_query_k<PRIME, MODE, 8>(a, st);
    default: return launch_query_k<PRIME, MODE, 4>(a, st);
  }
}

hipError_t launch_query(const QueryArgsAny& a, hipStream_t st) {
  if (a.prime == kPrime61) {
    if (a.mode == kTwoForOne) return launch_query_m<kPrime61, kTwoForOne>(a, st);
    if (a.mode == kTwoForOneMsb) return launch_query_m<kPrime61, kTwoForOneMsb>(a, st);
    return launch_query_m<kPrime61, kTwoPoly>(a, st);
  }
  if (a.mode == kTwoForOne) return launch_query_m<kPrime89, kTwoForOne>(a, st);
  if (a.mode == kTwoForOneMsb) return launch_query_m<kPrime89, kTwoForOneMsb>(a, st);
  return launch_query_m<kPrime89, kTwoPoly>(a, st);
}

hipError_t launch_estimate(const int64_t* table, uint32_t rows, uint32_t log2m, uint32_t slices, EstPartial* part,
                           int64_t* out, uint32_t* flags, hipStream_t st) {
  hipLaunchKernelGGL(k_estimate_partial, dim3(slices, rows), dim3(kBlock), 0, st, table, log2m, slices, part);
  hipLaunchKernelGGL(k_estimate_final, dim3(1), dim3(kBlock), 0, st, part, rows, slices, out, flags);
  return hipGetLastError();
}

hipError_t launch_add_tables(unsigned long long* dst, const unsigned long long* src, uint64_t n, hipStream_t st) {
  uint64_t blocks = std::min<uint64_t>((n + kBlock - 1) / kBlock, 4096);
  hipLaunchKernelGGL(k_add_tables, dim3((uint32_t)blocks), dim3(kBlock), 0, st, dst, src, n);
  return hipGetLastError();
}

hipError_t launch_fill_zero(unsigned long long* dst, uint64_t n, hipStream_t st) {
  uint64_t blocks = std::min<uint64_t>((n + kBlock - 1) / kBlock, 4096);
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_zero, dim3((uint32_t)blocks), dim3(kBlock), 0, st, dst, n);
  return hipGetLastError();
}

}  // namespace mcs
