// sketch_kernels.hip -- the non-template Count Sketch kernels (pass 2 of the
// two-pass update, F2 estimates, table fill and add) and the dispatch from
// runtime (prime, mode) to the per-pair launchers instantiated in
// sketch_p*_*.hip.
#include <algorithm>

#include "device_util.hpp"
#include "sketch_kernels.hpp"

namespace mcs {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// One pass-2 item: records of partition `part` from the tiles of slice
// `slice`, accumulated in LDS `acc` and added into args.table.  A wave takes
// kU tiles at a time.  Each lane loads 16-byte chunks (4 records), 16 lanes
// per tile, so one load reads up to 64 records of each of 4 tiles; the
// kU / 4 loads of a round are issued before any record is used (a lane with
// no chunk of its tile loads a harmless chunk instead of branching), and
// each record of a chunk is kept only if it lies in the tile's group.
__device__ __forceinline__ void accumulate_item(const AccArgs& args, uint32_t part, uint32_t slice,
                                                unsigned long long* acc) {
  const uint32_t G = 1u << args.log2g;
  const uint32_t log2r = args.log2r, wb = 31u - log2r;  // weight field bits (record layout in k_bin)
  const uint32_t span = args.log2m < log2r ? (1u << args.log2m) : (1u << log2r);  // counters per range
  const uint32_t per = (args.tiles + args.slices - 1) / args.slices;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64), lane = threadIdx.x % 64;
  const uint32_t nw = kAccBlock / 64;
  constexpr uint32_t kU = 16;              // tiles per wave round
  constexpr uint32_t kLpt = 16;            // lanes per tile in one load
  constexpr uint32_t kTpl = 64 / kLpt;     // tiles per load
  constexpr uint32_t kLoads = kU / kTpl;   // loads per round
  const uint32_t r = part >> args.log2g, g = part & (G - 1);
  for (uint32_t i = threadIdx.x; i < span; i += kAccBlock) acc[i] = 0;
  __syncthreads();
  const uint32_t t0 = slice * per, t1 = min(args.tiles, t0 + per);
  const uint32_t sub = lane / kLpt, li = lane % kLpt;
  const uint4* const spare = (const uint4*)args.recs;
  for (uint32_t tb = t0 + wave * kU; tb < t1; tb += nw * kU) {
    // lanes 0..kU-1 fetch the group bounds of tiles tb + lane
    uint32_t lb = 0, le = 0;
    if (lane < kU && tb + lane < t1) {
      lb = args.desc[desc_index(r, g, G, args.tiles, tb + lane)];
      le = args.desc[desc_index(r, g + 1, G, args.tiles, tb + lane)];
    }
    uint32_t lo[kLoads], hi[kLoads];
    const uint4* src[kLoads];
#pragma unroll
    for (uint32_t q = 0; q < kLoads; ++q) {
      const uint32_t u = q * kTpl + sub;  // this lane's tile in load q
      lo[q] = __shfl(lb, u, 64);
      hi[q] = __shfl(le, u, 64);
      src[q] = (const uint4*)(args.recs + ((size_t)(tb + u) * args.rows + r) * args.tile_keys);
    }
    for (uint32_t c = li;; c += kLpt) {  // chunk index from the group's first chunk
      u32x4 v[kLoads];
      uint32_t pos[kLoads];
      bool more = false;
#pragma unroll
      for (uint32_t q = 0; q < kLoads; ++q) {
        const uint32_t ch = (lo[q] >> 2) + c;
        pos[q] = ch * 4;
        const u32x4* at = (const u32x4*)(pos[q] < hi[q] ? src[q] + ch : spare);
        v[q] = *at;
        more |= pos[q] + 4 * kLpt < hi[q];
      }
      // whole 16-byte loads, all issued before the first record is used (the
      // compiler would otherwise move a word's load into the branch using it)
#pragma unroll
      for (uint32_t q = 0; q < kLoads; ++q) asm volatile("" : "+v"(v[q]));
#pragma unroll
      for (uint32_t q = 0; q < kLoads; ++q) {
        const uint32_t w4[4] = {v[q].x, v[q].y, v[q].z, v[q].w};
#pragma unroll
        for (uint32_t e = 0; e < 4; ++e)
          if (pos[q] + e >= lo[q] && pos[q] + e < hi[q]) {
            const int64_t sw = (int64_t)((int32_t)(w4[e] << (log2r + 1)) >> (log2r + 1));
            atomicAdd(&acc[w4[e] >> (wb + 1)], (unsigned long long)sw);
          }
      }
      if (!__any(more)) break;
    }
  }
  __syncthreads();
  unsigned long long* dst = args.table + ((size_t)r << args.log2m) + ((size_t)g << log2r);
  for (uint32_t i = threadIdx.x; i < span; i += kAccBlock) {
    unsigned long long v = acc[i];
    if (v) atomicAdd(&dst[i], v);
  }
  __syncthreads();
}

// two 16-wave blocks per CU (8 waves per SIMD): at most 64 VGPRs
__global__ __launch_bounds__(kAccBlock, 8) void k_accumulate(AccArgs args) {
  extern __shared__ unsigned long long acc[];
  const uint32_t items = (args.rows << args.log2g) * args.slices;
  for (uint32_t item = blockIdx.x; item < items; item += gridDim.x)
    accumulate_item(args, item / args.slices, item % args.slices, acc);
}

// Sum of squares of one slice of one row (128-bit, with a flag once the
// running sum nears 2^126, far before it could wrap); block-wide.
__device__ __forceinline__ void est_partial_block(const int64_t* __restrict__ table, uint32_t log2m, uint32_t slices,
                                                  uint32_t row, uint32_t slice, EstPartial* __restrict__ part) {
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
    big |= (uint32_t)(acc >> 126);
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
  __syncthreads();  // the shared arrays are reused by the block's next item
}

// Row totals X_j, their median (element (rows-1)/2 of the sorted values) and
// the flags word: out[0] = median, out[1..rows] = X_j, out[1+rows] = flags.
// Block-wide.
__device__ __forceinline__ void est_final_block(const EstPartial* __restrict__ part, uint32_t rows, uint32_t slices,
                                                int64_t* __restrict__ out, const uint32_t* flags) {
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
    out[1 + rows] = (int64_t)((*(volatile const uint32_t*)flags) | (over ? kFlagOverflow : 0u));
  }
  __syncthreads();
}

__global__ __launch_bounds__(kBlock) void k_estimate_partial(const int64_t* __restrict__ table, uint32_t log2m,
                                                             uint32_t slices, EstPartial* __restrict__ part) {
  est_partial_block(table, log2m, slices, blockIdx.y, blockIdx.x, part);
}

__global__ __launch_bounds__(kBlock) void k_estimate_final(const EstPartial* __restrict__ part, uint32_t rows,
                                                           uint32_t slices, int64_t* __restrict__ out,
                                                           uint32_t* flags) {
  est_final_block(part, rows, slices, out, flags);
}

// Estimates of many sketches in two launches: blocks [first, first + rows *
// slices) of the partial kernel belong to item i; one final block per item.
__global__ __launch_bounds__(kBlock) void k_batch_est_partial(const BatchEstItem* __restrict__ items, uint32_t nitems,
                                                              uint32_t total_blocks) {
  for (uint32_t b = blockIdx.x; b < total_blocks; b += gridDim.x) {
    uint32_t lo = 0, hi = nitems;  // last item with first <= b
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (uniform_load(&items[mid].first_block) <= b) lo = mid; else hi = mid;
    }
    const BatchEstItem it = uniform_load(items + lo);
    const uint32_t local = b - it.first_block;
    est_partial_block(it.table, it.log2m, it.slices, local / it.slices, local % it.slices, it.part);
  }
}

__global__ __launch_bounds__(kBlock) void k_batch_est_final(const BatchEstItem* __restrict__ items, uint32_t nitems,
                                                            int64_t* __restrict__ out) {
  for (uint32_t i = blockIdx.x; i < nitems; i += gridDim.x) {
    const BatchEstItem it = uniform_load(items + i);
    est_final_block(it.part, it.rows, it.slices, out + it.out_offset, it.flags);
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

__global__ __launch_bounds__(kAccBlock, 8) void k_batch_acc(const BatchSegment* __restrict__ segs,
                                                        const BatchAccItem* __restrict__ items, uint32_t nitems) {
  extern __shared__ unsigned long long acc[];
  for (uint32_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    const BatchAccItem item = uniform_load(items + it);
    const BatchSegment sg = uniform_load(segs + item.segment);
    AccArgs a{sg.recs, sg.desc, sg.tiles, sg.rows, sg.log2m, sg.log2g, sg.log2r, item.slices, kWaveTile, sg.table};
    accumulate_item(a, item.part, item.slice, acc);
  }
}

hipError_t launch_accumulate(const AccArgs& c, uint32_t blocks, uint32_t lds_bytes, hipStream_t st) {
  hipLaunchKernelGGL(k_accumulate, dim3(blocks), dim3(kAccBlock), lds_bytes, st, c);
  return hipGetLastError();
}

hipError_t launch_batch_acc(const BatchRound& rd, uint32_t lds_bytes, hipStream_t st) {
  hipLaunchKernelGGL(k_batch_acc, dim3(rd.acc_blocks), dim3(kAccBlock), lds_bytes, st, rd.segs, rd.acc_items, rd.nacc);
  return hipGetLastError();
}

// pass 2 holds up to 2^kMaxRangeLog2 int64 counters in dynamic LDS (above the
// 64 KiB default)
hipError_t set_accumulate_attribute() {
  return hipFuncSetAttribute((const void*)k_accumulate, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)(sizeof(unsigned long long) << kMaxRangeLog2));
}

hipError_t set_batch_acc_attribute() {
  return hipFuncSetAttribute((const void*)k_batch_acc, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)(sizeof(unsigned long long) << kMaxRangeLog2));
}

hipError_t launch_batch(const BatchLaunch& b, hipStream_t st) {
  if (b.prime == kPrime61) {
    if (b.mode == kTwoForOne) return launch_batch_pm<kPrime61, kTwoForOne>(b, st);
    if (b.mode == kTwoForOneMsb) return launch_batch_pm<kPrime61, kTwoForOneMsb>(b, st);
    if (b.mode == kArbR) return launch_batch_pm<kPrime61, kArbR>(b, st);
    return launch_batch_pm<kPrime61, kTwoPoly>(b, st);
  }
  if (b.mode == kTwoForOne) return launch_batch_pm<kPrime89, kTwoForOne>(b, st);
  if (b.mode == kTwoForOneMsb) return launch_batch_pm<kPrime89, kTwoForOneMsb>(b, st);
  if (b.mode == kArbR) return launch_batch_pm<kPrime89, kArbR>(b, st);
  return launch_batch_pm<kPrime89, kTwoPoly>(b, st);
}

hipError_t launch_update(const UpdatePlan& plan, const UpdateArgsAny& a, hipStream_t st) {
  if (a.prime == kPrime61) {
    if (a.mode == kTwoForOne) return launch_update_pm<kPrime61, kTwoForOne>(plan, a, st);
    if (a.mode == kTwoForOneMsb) return launch_update_pm<kPrime61, kTwoForOneMsb>(plan, a, st);
    if (a.mode == kArbR) return launch_update_pm<kPrime61, kArbR>(plan, a, st);
    return launch_update_pm<kPrime61, kTwoPoly>(plan, a, st);
  }
  if (a.mode == kTwoForOne) return launch_update_pm<kPrime89, kTwoForOne>(plan, a, st);
  if (a.mode == kTwoForOneMsb) return launch_update_pm<kPrime89, kTwoForOneMsb>(plan, a, st);
  if (a.mode == kArbR) return launch_update_pm<kPrime89, kArbR>(plan, a, st);
  return launch_update_pm<kPrime89, kTwoPoly>(plan, a, st);
}

hipError_t launch_query(const QueryArgsAny& a, hipStream_t st) {
  if (a.prime == kPrime61) {
    if (a.mode == kTwoForOne) return launch_query_pm<kPrime61, kTwoForOne>(a, st);
    if (a.mode == kTwoForOneMsb) return launch_query_pm<kPrime61, kTwoForOneMsb>(a, st);
    if (a.mode == kArbR) return launch_query_pm<kPrime61, kArbR>(a, st);
    return launch_query_pm<kPrime61, kTwoPoly>(a, st);
  }
  if (a.mode == kTwoForOne) return launch_query_pm<kPrime89, kTwoForOne>(a, st);
  if (a.mode == kTwoForOneMsb) return launch_query_pm<kPrime89, kTwoForOneMsb>(a, st);
  if (a.mode == kArbR) return launch_query_pm<kPrime89, kArbR>(a, st);
  return launch_query_pm<kPrime89, kTwoPoly>(a, st);
}

hipError_t launch_estimate(const int64_t* table, uint32_t rows, uint32_t log2m, uint32_t slices, EstPartial* part,
                           int64_t* out, uint32_t* flags, hipStream_t st) {
  hipLaunchKernelGGL(k_estimate_partial, dim3(slices, rows), dim3(kBlock), 0, st, table, log2m, slices, part);
  hipLaunchKernelGGL(k_estimate_final, dim3(1), dim3(kBlock), 0, st, part, rows, slices, out, flags);
  return hipGetLastError();
}

hipError_t launch_batch_estimate(const BatchEstItem* items, uint32_t nitems, uint32_t total_blocks, int64_t* out,
                                 uint32_t cus, hipStream_t st) {
  if (nitems == 0) return hipSuccess;
  const uint32_t pb = std::max<uint32_t>(1, std::min<uint32_t>(total_blocks, cus * 8));
  hipLaunchKernelGGL(k_batch_est_partial, dim3(pb), dim3(kBlock), 0, st, items, nitems, total_blocks);
  const uint32_t fb = std::max<uint32_t>(1, std::min<uint32_t>(nitems, cus * 8));
  hipLaunchKernelGGL(k_batch_est_final, dim3(fb), dim3(kBlock), 0, st, items, nitems, out);
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
